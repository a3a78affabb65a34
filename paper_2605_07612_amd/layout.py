"""Caller-side helpers for writing initial conditions into a mesh's state
tensor and reading results back (host work, not part of the hot path).

Block n of the state tensor is leaf n of the mesh.  Each (block, variable)
group of P^ndim values (P = N + 2g) holds first the rows (k, j) of N interior
x cells, then the 2g x ghosts of every row (include/foap4.h); `rows_view`,
`to_padded` and `from_padded` convert between that and the padded cube
[P]^ndim in which cell (i, j, k) sits at (k+g, j+g, i+g)."""
from __future__ import annotations

import numpy as np


def rows_view(u, N, g, ndim):
    """u: [..., P^ndim] -> view [..., P, (P,) N] of the row part (k, j, i)."""
    P = N + 2 * g
    R = P ** (ndim - 1)
    lead = tuple(u.shape[:-1])
    return u[..., : R * N].reshape(lead + (P,) * (ndim - 1) + (N,))


def xghost_view(u, N, g, ndim):
    """u: [..., P^ndim] -> view [..., P, (P,) 2g] of the x ghosts (c = i+g for
    i < 0, i-N+g for i >= N)."""
    P = N + 2 * g
    R = P ** (ndim - 1)
    lead = tuple(u.shape[:-1])
    return u[..., R * N:].reshape(lead + (P,) * (ndim - 1) + (2 * g,))


def to_padded(u, N, g, ndim):
    """A copy of u ([..., P^ndim], torch or numpy) as padded cubes [..., P^ndim as (P,)*ndim]."""
    P = N + 2 * g
    shape = tuple(u.shape[:-1]) + (P,) * ndim
    if isinstance(u, np.ndarray):
        out = np.empty(shape, dtype=u.dtype)
    else:
        out = u.new_empty(shape)
    rows, xg = rows_view(u, N, g, ndim), xghost_view(u, N, g, ndim)
    out[..., g:g + N] = rows
    out[..., :g] = xg[..., :g]
    out[..., g + N:] = xg[..., g:]
    return out


def from_padded(cube, N, g, ndim):
    """Inverse of to_padded: [..., (P,)*ndim] -> [..., P^ndim]."""
    P = N + 2 * g
    R = P ** (ndim - 1)
    lead = tuple(cube.shape[:-ndim])
    if isinstance(cube, np.ndarray):
        out = np.empty(lead + (P ** ndim,), dtype=cube.dtype)
    else:
        out = cube.new_empty(lead + (P ** ndim,))
    rows, xg = rows_view(out, N, g, ndim), xghost_view(out, N, g, ndim)
    rows[...] = cube[..., g:g + N]
    xg[..., :g] = cube[..., :g]
    xg[..., g:] = cube[..., g + N:]
    return out


def global_coords(mesh):
    """(level[nb], G[nb][3]): global integer block coordinates at each block's level."""
    lev, tree, anc = mesh.export()
    nt = list(mesh.desc.n_trees)
    t = np.stack([tree % nt[0], (tree // nt[0]) % nt[1], tree // (nt[0] * nt[1])], axis=1)
    G = (t.astype(np.int64) << lev[:, None].astype(np.int64)) + anc
    return lev, G


def cell_centres(mesh):
    """Cell-centre coordinates [nb][ndim][N]*ndim (index order k, j, i)."""
    lev, G = global_coords(mesh)
    N, ndim = mesh.N, mesh.ndim
    ts = mesh.desc.tree_size
    org = list(mesh.desc.origin)
    dx = ts / (N * (2.0 ** lev))
    idx = np.arange(N) + 0.5
    out = np.empty((len(lev), ndim) + (N,) * ndim)
    for d in range(ndim):
        c = org[d] + (G[:, d, None] * N + idx[None, :]) * dx[:, None]  # [nb][N]
        shape = [len(lev)] + [1] * ndim
        shape[ndim - d] = N
        out[:, d] = np.broadcast_to(c.reshape(shape), (len(lev),) + (N,) * ndim)
    return out


def set_interior(mesh, values):
    """values: [nb][nvar][N]*ndim (numpy) written into the current state."""
    torch = __import__("torch")
    t = torch.from_numpy(np.ascontiguousarray(values)).to(mesh.dtype).to(mesh.state[0].device)
    mesh.interior().copy_(t)


def set_from_field(mesh, field):
    """Evaluate field(x, y[, z]) -> [nvar][nb][N..] at the cell centres."""
    xc = cell_centres(mesh)
    vals = field(*[xc[:, d] for d in range(mesh.ndim)])
    set_interior(mesh, np.moveaxis(vals, 0, 1))


def set_from_field_device(mesh, field):
    """Evaluate field(x, y[, z], xp=torch) at the cell centres on the device
    (float64 torch tensors) and store it: for initial data too large to
    build on the host."""
    torch = __import__("torch")
    dev = mesh.state[0].device
    lev, G = global_coords(mesh)
    N, ndim, nb = mesh.N, mesh.ndim, len(lev)
    ts = mesh.desc.tree_size
    org = list(mesh.desc.origin)
    dx = torch.tensor(ts / (N * (2.0 ** lev)), dtype=torch.float64, device=dev)
    Gt = torch.tensor(G, dtype=torch.float64, device=dev)
    idx = torch.arange(N, dtype=torch.float64, device=dev) + 0.5
    coords = []
    for d in range(ndim):
        c = org[d] + (Gt[:, d, None] * N + idx[None, :]) * dx[:, None]  # [nb][N]
        shape = [nb] + [1] * ndim
        shape[ndim - d] = N
        coords.append(c.reshape(shape).expand((nb,) + (N,) * ndim))
    vals = field(*coords, xp=torch)  # [nvar][nb][N..]
    mesh.interior().copy_(vals.movedim(0, 1).to(mesh.dtype))


def set_from_grid(mesh, grid):
    """grid: [nvar][nz][ny][nx] (or [nvar][ny][nx]) on a uniform-level mesh."""
    lev, G = global_coords(mesh)
    N, ndim = mesh.N, mesh.ndim
    nv = grid.shape[0]
    if ndim == 3:
        nz, ny, nx = grid.shape[1:]
        blk = grid.reshape(nv, nz // N, N, ny // N, N, nx // N, N).transpose(1, 3, 5, 0, 2, 4, 6)
        vals = blk[G[:, 2], G[:, 1], G[:, 0]]
    else:
        ny, nx = grid.shape[1:]
        blk = grid.reshape(nv, ny // N, N, nx // N, N).transpose(1, 3, 0, 2, 4)
        vals = blk[G[:, 1], G[:, 0]]
    set_interior(mesh, vals)
