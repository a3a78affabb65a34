"""Pins of the oracle's physical boundary conditions (Sec. 2.4: Dirichlet and
Neumann values per face direction and variable), CPU only.  Each check is an
exact solution, a symmetry or a conservation law fixed by the mathematics."""
import itertools

import numpy as np
import pytest

import synth
from oracle import OracleMesh

COEF = (1.0, 2.0, 3.0)
# per-variable affine maps u_v = A_v + B_v phi, so each variable needs its own
# boundary values
A = (0.0, 1.0, -1.0, 2.0, 5.0)
B = (1.0, -2.0, 0.5, 3.0, 0.0)


def wall_bc(ndim):
    """Reflecting wall: normal momentum Dirichlet 0, every other variable
    Neumann 0 (ghosts = mirror images with the normal momentum negated)."""
    t = np.ones((6, 5), np.int32)
    for f in range(2 * ndim):
        t[f, 1 + f // 2] = 0
    return t, np.zeros((6, 5))


def linear_mesh(ndim, g, levels, rref, mode):
    """Non-periodic unit square/cube with the linear data on its one root
    block, refined `levels` times around rref (the remap prolongs the data).
    mode 'neumann': u_v = A_v + B_v (x + 2y + 3z) with the outward normal
    derivative of u_v on every face; mode 'dirichlet': u_v = A_v + B_v c z
    (2D: y) with its face values on the faces normal to that axis and
    Neumann 0 on the others."""
    nv = ndim + 2
    t = np.ones((6, 5), np.int32)
    val = np.zeros((6, 5))
    for f in range(2 * ndim):
        ax, side = f // 2, f % 2
        sgn = 1.0 if side else -1.0
        for v in range(nv):
            if mode == "neumann":
                val[f, v] = sgn * B[v] * COEF[ax]
            elif ax == ndim - 1:
                t[f, v] = 0
                val[f, v] = A[v] + B[v] * COEF[ax] * (1.0 if side else 0.0)
    m = OracleMesh(ndim, (1, 1, 1), 8, g, 1.0, periodic=(False,) * 3, bc_type=t, bc_value=val)
    xc = m.forest.cell_centres(m.N, 1.0)
    for v in range(nv):
        m.interior()[:, v] = exact(mode, ndim, [xc[:, d] for d in range(ndim)], v)
    for _ in range(levels):
        flags = np.zeros(m.nb, np.int8)
        for n, (l, G) in enumerate(m.forest.leaves):
            h = 1.0 / (1 << l)
            if all(G[d] * h <= rref[d] < (G[d] + 1) * h for d in range(ndim)):
                flags[n] = 1
        m.regrid(flags, 0, 20)
    return m


def exact(mode, ndim, cent, v):
    """cent: [ndim][...] cell centres."""
    if mode == "neumann":
        phi = sum(COEF[d] * cent[d] for d in range(ndim))
    else:
        phi = COEF[ndim - 1] * cent[ndim - 1]
    return A[v] + B[v] * phi


@pytest.mark.parametrize("mode", ["neumann", "dirichlet"])
@pytest.mark.parametrize("ndim,g,levels", [(2, 2, 5), (2, 3, 4), (2, 4, 3), (3, 2, 3), (3, 3, 2), (3, 4, 2)])
def test_linear_solution_exact_with_physical_boundaries(ndim, g, levels, mode):
    """Sec. 4.3 (eq. refinement-test, eq. refinement-coord) with the solution
    given on the domain boundary (Sec. 2.4): every face ghost of every block
    - same-level, restricted, prolonged and physical-boundary ghosts, also
    where refinement reaches a corner, an edge or a face of the domain - is
    exact for a linear solution to 1e-15 of its magnitude, and so are the
    interiors prolonged during the refinement sequence."""
    nv = ndim + 2
    for ijk in itertools.product([-1, 0, 1], repeat=ndim):
        rref = [0.5 + 0.49 * o for o in ijk]
        m = linear_mesh(ndim, g, levels, rref, mode)
        N, P = m.N, m.P
        xc = m.forest.cell_centres(N, 1.0)
        for v in range(nv):
            assert np.max(np.abs(m.interior()[:, v] - exact(mode, ndim, [xc[:, d] for d in range(ndim)], v))) \
                <= 1e-15 * (abs(A[v]) + abs(B[v]) * 6.0)
        ghost = np.ones((P,) * ndim, bool)
        ghost[(slice(g, g + N),) * ndim] = False
        m.u[:, :, ghost] = np.nan  # stale-value sentinel
        m.ghost_fill()
        idx = np.arange(-g, N + g) + 0.5
        checked = 0
        for n, (l, G) in enumerate(m.forest.leaves):
            dx = 1.0 / (N << l)
            cent = []
            for d in range(ndim):
                shape = [1] * ndim
                shape[ndim - 1 - d] = P
                cent.append(np.broadcast_to(((G[d] * N + idx) * dx).reshape(shape), (P,) * ndim))
            for f in range(2 * ndim):
                ax, side = f // 2, f % 2
                sl = [slice(g, g + N)] * ndim
                sl[ndim - 1 - ax] = slice(g + N, P) if side else slice(0, g)
                sl = tuple(sl)
                for v in range(nv):
                    got = m.u[n, v][sl]
                    want = exact(mode, ndim, [c[sl] for c in cent], v)
                    scale = abs(A[v]) + abs(B[v]) * 6.0
                    assert np.all(np.abs(got - want) <= 1e-15 * max(scale, 1.0)), (rref, n, f, v)
                    checked += got.size
        assert checked > 0


def test_uniform_state_fixed_under_matching_dirichlet_values():
    """A closed box whose Dirichlet values equal a uniform state keeps it
    bitwise (every ghost is 2 u_b - u_b = u_b)."""
    U = [1.3, 0.2, -0.1, 0.3, 2.7]
    m = OracleMesh(3, (2, 2, 2), 8, 2, 0.5, periodic=(False,) * 3,
                   bc_type=np.zeros((6, 5), np.int32), bc_value=np.tile(U, (6, 1)))
    m.interior()[...] = np.asarray(U).reshape(1, 5, 1, 1, 1)
    u0 = m.interior().copy()
    m.step(4)
    assert np.array_equal(m.interior(), u0)


@pytest.mark.parametrize("ndim", [2, 3])
def test_reflecting_wall_equals_mirrored_periodic_domain(ndim):
    """Walls at x = 0 and x = 1 (normal momentum Dirichlet 0, the rest
    Neumann 0) give the flow of the periodic domain [0, 2] whose right half
    is the mirror image of the left: after 5 steps the walled solution
    equals the left half (to rounding of the mirrored arithmetic, 1e-14)."""
    nt = (2, 2, 2)[:ndim] + (1,) * (3 - ndim)
    t, val = wall_bc(ndim)
    per = (False, True, True)
    a = OracleMesh(ndim, nt, 8, 2, 0.5, periodic=per, bc_type=t, bc_value=val)
    nt2 = (4,) + nt[1:]
    b = OracleMesh(ndim, nt2, 8, 2, 0.5)
    xc = a.forest.cell_centres(8, 0.5)
    rng = np.random.default_rng(4)
    k = rng.random(6)
    x, y = xc[:, 0], xc[:, 1]
    z = xc[:, 2] if ndim == 3 else 0 * x
    rho = 1 + 0.3 * np.sin(2 * np.pi * (x + k[0])) * np.cos(2 * np.pi * (y + k[1])) + 0.1 * np.sin(2 * np.pi * z)
    vel = [0.3 * np.sin(2 * np.pi * (y + k[2])) + 0.2 * x, 0.2 * np.cos(2 * np.pi * (x + k[3]))]
    if ndim == 3:
        vel.append(0.1 * np.sin(2 * np.pi * (x + y + k[4])))
    U = synth.conserved_from_primitive(rho, vel, 1 + 0.2 * np.cos(2 * np.pi * (z + x + k[5])), 1.4)
    a.interior()[...] = np.moveaxis(U, 0, 1)
    for n, (l, G) in enumerate(a.forest.leaves):
        left = b.forest.index[(l, G)]
        right = b.forest.index[(l, (3 - G[0],) + tuple(G[1:]))]
        b.interior()[left] = a.interior()[n]
        mirror = a.interior()[n][(slice(None),) + (slice(None),) * (ndim - 1) + (slice(None, None, -1),)].copy()
        mirror[1] *= -1
        b.interior()[right] = mirror
    a.step(5)
    b.step(5)
    assert a.t == b.t
    err = max(float(np.max(np.abs(a.interior()[n] - b.interior()[b.forest.index[(l, G)]])))
              for n, (l, G) in enumerate(a.forest.leaves))
    assert err <= 1e-14, err


@pytest.mark.parametrize("ndim", [2, 3])
def test_closed_box_conserves_mass_and_energy(ndim):
    """All faces walls, a refined centre (flux fixing): the wall faces carry
    no mass or energy flux (the mirrored states cancel exactly), so those
    totals change only by rounding; the momenta change by the wall pressure
    force."""
    t, val = wall_bc(ndim)
    m = OracleMesh(ndim, (4, 4, 4), 8, 2, 0.25, periodic=(False,) * 3, bc_type=t, bc_value=val)
    cent = [(np.array([G[d] for _, G in m.forest.leaves]) + 0.5) / 4 for d in range(ndim)]
    m.regrid(np.where(sum((c - 0.5) ** 2 for c in cent) < 0.09, 1, 0).astype(np.int8), 0, 1)
    assert set(m.level.tolist()) == {0, 1}
    m.set_interior_from_field(synth.blast_field(p_in=10.0, p_out=0.1, r0=0.15, centre=(0.4, 0.55, 0.5))
                              if ndim == 3 else
                              (lambda x, y: synth.conserved_from_primitive(
                                  1.0 + 0 * x, [0 * x, 0 * x], np.where((x - 0.4) ** 2 + (y - 0.55) ** 2 < 0.0225, 10.0, 0.1), 1.4)))
    t0 = m.totals()
    m.step(30)
    t1 = m.totals()
    scale = np.abs(t0) + 1.0
    assert abs(t1[0] - t0[0]) <= 1e-13 * scale[0]
    assert abs(t1[-1] - t0[-1]) <= 1e-13 * scale[-1]
    # the blast has reached the walls, so the normal momenta have moved
    assert np.max(np.abs(m.interior()[:, 1])) > 1e-3


def face_values(m, fn):
    """bc_data of mesh m (eq. bc-data): fn(v, x) at the centre of every face
    cell of every boundary record, x = [ndim][N^(ndim-1)] coordinates, face
    cells with the lower tangential axis fastest."""
    pat, N, nd = m.pat, m.N, m.ndim
    nbf = int(pat["bc_off"][-1])
    n2 = N if nd == 3 else 1
    out = np.zeros((nbf, m.nvar, N * n2))
    p1, p2 = np.meshgrid(np.arange(N), np.arange(n2), indexing="xy")
    p1, p2 = p1.ravel(), p2.ravel()
    for f in range(2 * nd):
        ax, side = f // 2, f % 2
        t = [d for d in range(nd) if d != ax]
        for r in range(pat["bc_off"][f], pat["bc_off"][f + 1]):
            b = int(np.asarray(pat["bc"][r]).reshape(-1)[0])
            l, G = m.forest.leaves[b]
            dx = m.tree_size / (N << l)
            x = [None] * nd
            x[ax] = np.full(N * n2, (G[ax] * N + (N if side else 0)) * dx)
            x[t[0]] = (G[t[0]] * N + p1 + 0.5) * dx
            if nd == 3:
                x[t[1]] = (G[t[1]] * N + p2 + 0.5) * dx
            for v in range(m.nvar):
                out[r, v] = fn(v, x)
    return out


@pytest.mark.parametrize("ndim,g,levels", [(2, 2, 4), (2, 3, 3), (3, 2, 2), (3, 3, 2)])
def test_linear_solution_exact_with_bc_data(ndim, g, levels):
    """The paper's form of the Sec. 4.3 test: the linear solution is given on
    the whole domain boundary through the spatially varying boundary array
    (eq. bc-data, Dirichlet on every face, values at the face centres),
    refreshed by the mesh-change callback at every regrid; every face ghost
    stays exact to 1e-15 of the magnitude."""
    nv = ndim + 2
    fn = lambda v, x: A[v] + B[v] * sum(COEF[d] * x[d] for d in range(ndim))
    for ijk in itertools.product([-1, 0, 1], repeat=ndim):
        rref = [0.5 + 0.49 * o for o in ijk]
        m = OracleMesh(ndim, (1, 1, 1), 8, g, 1.0, periodic=(False,) * 3,
                       bc_type=np.zeros((6, 5), np.int32), bc_value=np.full((6, 5), 1e9))
        m.set_bc_data(face_values(m, fn), callback=lambda mm: face_values(mm, fn))
        xc = m.forest.cell_centres(m.N, 1.0)
        for v in range(nv):
            m.interior()[:, v] = fn(v, [xc[:, d] for d in range(ndim)])
        for _ in range(levels):
            flags = np.zeros(m.nb, np.int8)
            for n, (l, G) in enumerate(m.forest.leaves):
                h = 1.0 / (1 << l)
                if all(G[d] * h <= rref[d] < (G[d] + 1) * h for d in range(ndim)):
                    flags[n] = 1
            m.regrid(flags, 0, 20)
        N, P = m.N, m.P
        ghost = np.ones((P,) * ndim, bool)
        ghost[(slice(g, g + N),) * ndim] = False
        m.u[:, :, ghost] = np.nan
        m.ghost_fill()
        idx = np.arange(-g, N + g) + 0.5
        for n, (l, G) in enumerate(m.forest.leaves):
            dx = 1.0 / (N << l)
            cent = []
            for d in range(ndim):
                shape = [1] * ndim
                shape[ndim - 1 - d] = P
                cent.append(np.broadcast_to(((G[d] * N + idx) * dx).reshape(shape), (P,) * ndim))
            for f in range(2 * ndim):
                sl = [slice(g, g + N)] * ndim
                sl[ndim - 1 - f // 2] = slice(g + N, P) if f % 2 else slice(0, g)
                sl = tuple(sl)
                for v in range(nv):
                    want = fn(v, [c[sl] for c in cent])
                    assert np.all(np.abs(m.u[n, v][sl] - want) <= 1e-15 * max(1.0, abs(A[v]) + 6 * abs(B[v]))), \
                        (rref, n, f, v)
