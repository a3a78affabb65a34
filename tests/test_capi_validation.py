"""Argument validation of the C ABI on a machine without a GPU: every check
below returns its status before the library makes any HIP call, so the
calls are safe here (the state pointers are host dummies never touched)."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2605_07612_amd", "libfoap4.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfoap4.so not built")

E_INVALID, E_CAPACITY = -1, -2


@pytest.fixture(scope="module")
def f4():
    import paper_2605_07612_amd as f4
    f4.lib()
    return f4


def desc(f4, **kw):
    d = f4.MeshDesc()
    v = dict(ndim=3, n_trees=(2, 2, 2), periodic=(1, 1, 1), origin=(0.0, 0.0, 0.0), tree_size=0.5,
             block_n=8, n_ghost=2, init_level=0, min_level=0, max_level=0, max_blocks=8, prec=0,
             gamma=1.4, cfl=0.5)
    v.update(kw)
    for k, x in v.items():
        if isinstance(x, tuple):
            getattr(d, k)[:] = list(x)
        else:
            setattr(d, k, x)
    return d


def create(f4, d, nbytes=None, same=False, misalign=0):
    buf = np.zeros(128, np.uint8)
    a = (buf.ctypes.data + 15) // 16 * 16  # 16-byte aligned host dummies, never touched
    p0 = ctypes.c_void_p(a)
    p1 = p0 if same else ctypes.c_void_p(a + 32 + misalign)
    if nbytes is None:
        P = d.block_n + 2 * d.n_ghost
        nbytes = d.max_blocks * (d.ndim + 2) * P ** d.ndim * (8 if d.prec == 1 else 4)
    h = ctypes.c_void_p(123)
    st = f4.lib().foap4_mesh_create(ctypes.byref(d), p0, p1, nbytes, None, ctypes.byref(h))
    msg = f4.lib().foap4_last_error(None).decode()
    return st, h.value, msg


BAD = [
    dict(ndim=1),
    dict(ndim=4),
    dict(block_n=12),
    dict(block_n=64),
    dict(n_ghost=1),
    dict(n_ghost=5),
    dict(n_trees=(0, 2, 2)),
    dict(periodic=(1, 2, 1)),
    dict(n_trees=(256, 256, 1)),
    dict(max_level=15),
    dict(min_level=1, max_level=0),
    dict(init_level=1, max_level=0),
    dict(tree_size=0.0),
    dict(gamma=1.0),
    dict(cfl=0.0),
    dict(prec=2),
    dict(max_blocks=0),
    dict(limiter=2),
    dict(flux=-1),
    dict(gravity=(0.0, float("inf"), 0.0)),
    dict(gravity=(float("nan"), 0.0, 0.0)),
    dict(physics=2),
    dict(physics=1, velocity=(0.0, 0.0, 0.0)),
    dict(physics=1, velocity=(0.0, 0.0, 0.0), ndim=2, n_trees=(2, 2, 1)),
    dict(physics=1, velocity=(1.0, float("nan"), 0.0)),
    dict(physics=1, velocity=(1.0, 0.0, 0.0), gravity=(0.0, 0.0, -1.0)),
]


@pytest.mark.parametrize("kw", BAD, ids=[",".join(f"{k}={v}" for k, v in b.items()) for b in BAD])
def test_bad_descriptor_is_refused(f4, kw):
    st, h, msg = create(f4, desc(f4, **kw))
    assert st == E_INVALID, (st, msg)
    assert not h and msg


def test_state_buffers_must_be_distinct_and_large_enough(f4):
    d = desc(f4)
    st, h, _ = create(f4, d, same=True)
    assert st == E_INVALID and not h
    P = 12
    st, h, msg = create(f4, d, nbytes=8 * 5 * P ** 3 * 4 - 1)
    assert st == E_INVALID and not h and "smaller" in msg


def test_state_buffers_must_be_16_byte_aligned(f4):
    st, h, msg = create(f4, desc(f4), misalign=8)
    assert st == E_INVALID and not h and "aligned" in msg


def test_initial_mesh_beyond_capacity(f4):
    st, h, msg = create(f4, desc(f4, init_level=1, max_level=1, max_blocks=63))
    assert st == E_CAPACITY and not h and "max_blocks" in msg


def test_null_handles_are_refused(f4):
    L = f4.lib()
    out = ctypes.c_void_p()
    assert L.foap4_mesh_create(None, None, None, 0, None, ctypes.byref(out)) == E_INVALID
    assert L.foap4_step(None, 1, None, None) == E_INVALID
    assert L.foap4_regrid(None, None, None) == E_INVALID
    assert L.foap4_ghost_pattern_build(None) == E_INVALID
    assert L.foap4_ghost_fill(None, 0) == E_INVALID
    assert L.foap4_compute_dt(None) == E_INVALID
    assert L.foap4_time(None, None, None) == E_INVALID
    assert L.foap4_batch_create(None, 0, ctypes.byref(out)) == E_INVALID
    assert L.foap4_mesh_capture_features(None, 1) == E_INVALID
    assert L.foap4_set_bc_data(None, None, 0, None, None) == E_INVALID


@pytest.mark.parametrize("field,value", [("bc_type", 2), ("bc_type", -1), ("bc_value", float("inf")),
                                         ("bc_value", float("nan"))])
def test_bad_boundary_condition_is_refused(f4, field, value):
    """On a bounded axis every face's boundary type must be Dirichlet (0) or
    Neumann (1) and its value finite."""
    d = desc(f4, periodic=(1, 0, 1))
    getattr(d, field)[3][2] = value  # +y face, m_y
    st, h, msg = create(f4, d)
    assert st == E_INVALID and not h and field in msg


def test_boundary_entries_of_periodic_axes_are_ignored(f4):
    """Boundary entries of a periodic axis are not read: with garbage there
    the descriptor gets past the boundary checks to the later buffer-size
    check (one byte is too small), which refuses it before any HIP call."""
    d = desc(f4, periodic=(1, 0, 1))
    d.bc_type[0][0] = 7            # -x face: periodic axis
    d.bc_value[1][1] = float("nan")
    st, h, msg = create(f4, d, nbytes=1)
    assert st == E_INVALID and not h and "smaller" in msg


def test_advection_velocity_of_the_unused_axis_is_ignored(f4):
    """Scalar advection in 2-D reads velocity[0..1] only: a zero velocity in
    the plane is refused even with velocity[2] set, a non-zero one gets past
    the checks to the buffer-size check (one byte is too small)."""
    d = desc(f4, ndim=2, n_trees=(2, 2, 1), physics=1, velocity=(0.0, 0.0, 3.0))
    st, h, msg = create(f4, d)
    assert st == E_INVALID and not h and "velocity" in msg
    d = desc(f4, ndim=2, n_trees=(2, 2, 1), physics=1, velocity=(0.0, -1.0, float("nan")))
    st, h, msg = create(f4, d, nbytes=1)
    assert st == E_INVALID and not h and "smaller" in msg


def test_advection_state_holds_one_variable(f4):
    """The state of scalar advection holds nvar = 1 variable per block: one
    byte less than max_blocks single-variable blocks is refused by the size
    check (before any HIP call)."""
    d = desc(f4, physics=1, velocity=(1.0, 0.5, 0.0))
    P = 12
    need = 8 * 1 * P ** 3 * 4
    st, h, msg = create(f4, d, nbytes=need - 1)
    assert st == E_INVALID and not h and "smaller" in msg
