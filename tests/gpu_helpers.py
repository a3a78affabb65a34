"""Shared set-up for the GPU parity tests: build the same workload on the HIP
path (through the C ABI) and in the FP64 oracle from the same seeded inputs."""
import numpy as np

import synth
from oracle import OracleMesh


def gpu_mesh(w, prec, max_level=None, max_blocks=None):
    import paper_2605_07612_amd as f4
    ml = w.get("level", 0) if max_level is None else max_level
    return f4.Mesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], level=w.get("level", 0),
                   max_level=ml, max_blocks=max_blocks, prec=prec, gamma=w["gamma"], cfl=w["cfl"], **scheme(w))


def oracle_mesh(w):
    return OracleMesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], level=w.get("level", 0),
                      gamma=w["gamma"], cfl=w["cfl"], **scheme(w))


def scheme(w):
    """Limiter, flux, gravity, boundaries and system of a workload (defaults:
    minmod, Rusanov, no source, periodic, the Euler equations)."""
    return dict(limiter=w.get("limiter", "minmod"), flux=w.get("flux", "rusanov"),
                gravity=tuple(w.get("gravity", (0.0, 0.0, 0.0))), periodic=tuple(w.get("periodic", (True,) * 3)),
                bc_type=w.get("bc_type"), bc_value=w.get("bc_value"), physics=w.get("physics", "euler"),
                velocity=tuple(w.get("velocity", (0.0, 0.0, 0.0))))


def refine_flags_base(w, mesh_tree_xyz):
    return w["refine_flags"](mesh_tree_xyz)


def build_pair(w, prec, static_refine=True):
    """(gpu mesh, oracle mesh) with the initial condition written."""
    from paper_2605_07612_amd import layout
    max_level = 1 if "refine_flags" in w else w.get("level", 0)
    base = int(np.prod(w["trees"][: w["ndim"]]))
    max_blocks = base * (1 << w["ndim"]) if "refine_flags" in w else None
    gm = gpu_mesh(w, prec, max_level=max_level, max_blocks=max_blocks)
    om = oracle_mesh(w)
    if "refine_flags" in w and static_refine:
        # flags of the level-0 base blocks (one block per tree)
        lev, G = layout.global_coords(gm)
        flags = w["refine_flags"](G)
        gm.regrid(flags)
        om.regrid(flags, 0, 1)
    if "grid_field" in w:
        grid = w["grid_field"]()
        layout.set_from_grid(gm, grid)
        om.set_interior_from_grid(grid)
    else:
        layout.set_from_field(gm, w["field"])
        om.set_interior_from_field(w["field"])
    return gm, om


def gpu_state(gm):
    """Current state of the leaf blocks as float64 numpy."""
    return gm.current().double().cpu().numpy()


def interior(a, g, N, ndim):
    sl = (slice(None), slice(None)) + (slice(g, g + N),) * ndim
    return a[sl]


def rel_l1_vol(a, b, levels, ndim, tree_size, N):
    """sum |a - b| dV / sum |b| dV over interior cells and all variables."""
    vol = (tree_size / (N * 2.0 ** levels)) ** ndim
    w = vol.reshape((-1,) + (1,) * (a.ndim - 1))
    return float(np.sum(np.abs(a - b) * w) / np.sum(np.abs(b) * w))


def face_ghost_mask(ndim, N, g):
    P = N + 2 * g
    m = np.zeros((P,) * ndim, bool)
    inner = slice(g, g + N)
    for ax in range(ndim):
        for s in (slice(0, g), slice(g + N, P)):
            sl = [inner] * ndim
            sl[ndim - 1 - ax] = s
            m[tuple(sl)] = True
    return m


# Bounds of a GPU state against the FP64 oracle: the volume-weighted relative
# L1 error of the parity target (FP64 1e-12, FP32 2e-5) and, so that an error
# confined to a few cells cannot hide in the global norm, a per-element bound
# max |a - b| <= tol * max |b| over every cell and variable (FP64 1e-10,
# FP32 1e-5: a few hundred roundings of the state's own precision).
REL_L1 = {0: 2e-5, 1: 1e-12}
PER_ELEM = {0: 1e-5, 1: 1e-10}


def max_elem_err(a, b):
    """max |a - b| / max |b| over all cells and variables."""
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def check_state(a, b, levels, ndim, tree_size, N, prec, l1=None, elem=None):
    """Asserts both bounds; returns (rel L1, per-element) errors."""
    e1 = rel_l1_vol(a, b, levels, ndim, tree_size, N)
    e2 = max_elem_err(a, b)
    assert e1 <= (REL_L1[prec] if l1 is None else l1), ("rel L1", e1)
    assert e2 <= (PER_ELEM[prec] if elem is None else elem), ("per element", e2)
    return e1, e2
