"""GPU parity of the SSP Runge-Kutta schemes with three and four sub-steps
(Sec. 3.1, eq. feuler) and of classical RK4 (eq. rk4, its last sub-step with
three earlier states) against the FP64 oracle, through the C ABI: FP64
within 1e-12 and FP32 within 2e-5 relative L1 on two-level meshes (ghost
rounds and flux fixing in every sub-step), with walls and the scheme
options; the batched form equal to the plain one bit for bit."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_helpers import build_pair, gpu_state, interior, check_state

pytestmark = pytest.mark.gpu

TOL = {0: 2e-5, 1: 1e-12}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def f4():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_07612_amd as f4
    f4.lib()
    return f4


def blast2d():
    def field(x, y):
        r = np.sqrt((x - 0.45) ** 2 + (y - 0.52) ** 2)
        p = np.where(r < 0.12, 10.0, 0.1)
        return synth.conserved_from_primitive(1.0 + 0 * r, [0 * r, 0 * r], p, 1.4)

    def refine_flags(G):
        G = np.asarray(G)
        return np.all((G[:, :2] >= 3) & (G[:, :2] <= 4), axis=1).astype(np.int8)

    return dict(name="blast2d", ndim=2, trees=(8, 8, 1), N=8, g=2, tree_size=1.0 / 8, level=0, gamma=1.4,
                cfl=0.5, field=field, refine_flags=refine_flags)


def walls(ndim):
    t = np.ones((6, 5), np.int32)
    for f in range(2 * ndim):
        t[f, 1 + f // 2] = 0
    return t, np.zeros((6, 5))


def case(name, integ):
    if name == "blast3d":
        w = synth.two_level_blast(base_trees=4, block=8)
    elif name == "blast2d":
        w = blast2d()
    elif name == "box3d_options":
        w = synth.two_level_blast(base_trees=4, block=8)
        w["field"] = synth.blast_field(p_in=10.0, p_out=0.1, r0=0.15, centre=(0.4, 0.55, 0.47))
        t, v = walls(3)
        w.update(periodic=(False, False, False), bc_type=t, bc_value=v, limiter="vanleer", flux="hll",
                 gravity=(0.0, 0.0, -1.0))
    else:
        w = synth.rayleigh_taylor(block=16, n=64)
    w = dict(w)
    w["integrator"] = integ
    w["name"] = f'{w["name"]}_{integ}'
    return w


def build(w, prec):
    """build_pair with the workload's integrator on both sides."""
    import paper_2605_07612_amd as f4
    from oracle import OracleMesh
    from paper_2605_07612_amd import layout
    from tests.gpu_helpers import scheme
    integ = w["integrator"]
    max_level = 1 if "refine_flags" in w else 0
    base = int(np.prod(w["trees"][: w["ndim"]]))
    gm = f4.Mesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], level=0, max_level=max_level,
                 max_blocks=base * (1 << w["ndim"]) if "refine_flags" in w else None, prec=prec, gamma=w["gamma"],
                 cfl=w["cfl"], integrator=integ, **scheme(w))
    om = OracleMesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], gamma=w["gamma"], cfl=w["cfl"],
                    integrator=integ, **scheme(w))
    if "refine_flags" in w:
        _, G = layout.global_coords(gm)
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


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("name", ["blast3d", "blast2d", "box3d_options", "rt3d"])
@pytest.mark.parametrize("integ", ["ssprk3", "ssprk43", "rk4"])
def test_parity(f4, integ, name, prec):
    w = case(name, integ)
    gm, om = build(w, prec)
    steps = 8
    gm.step(steps)
    om.step(steps)
    t, _ = gm.time()
    lev = gm.export()[0]
    a = interior(gpu_state(gm), w["g"], w["N"], w["ndim"])
    err, err_elem = check_state(a, om.interior(), lev, w["ndim"], w["tree_size"], w["N"], prec)
    say(w["name"], "prec", prec, "rel L1", err, "t", t, om.t)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-13 if prec == 1 else 1e-5) * om.t


@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
@pytest.mark.parametrize("integ", ["ssprk3", "ssprk43", "rk4"])
def test_batch_equals_plain(f4, integ, prec):
    """Two meshes (8^3 blocks on two levels, 16^3 blocks with z walls) of one
    scheme and integrator: the batched sub-steps equal the plain ones."""
    rt = case("rt3d", integ)
    bl = case("blast3d", integ)
    bl.update(limiter=rt["limiter"], flux=rt["flux"], gravity=(0.1, 0.0, -1.0))
    ws = [bl, rt]
    plain = [build(w, prec)[0] for w in ws]
    batched = [build(w, prec)[0] for w in ws]
    for m in plain:
        m.step(4)
    b = f4.Batch(batched)
    b.set_config(kslabs=2, wg_per_cu=2, xcd_order=1)
    b.step(4)
    for w, p, q in zip(ws, plain, batched):
        A = interior(gpu_state(p), w["g"], w["N"], w["ndim"])
        B = interior(gpu_state(q), w["g"], w["N"], w["ndim"])
        assert np.array_equal(A, B), w["name"]
        assert p.time() == q.time()
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        b.phase_times(1)
    b.close()


def test_refusals(f4):
    """An extra state that is too small, or at an index other than 2 or 3,
    is refused; feature capture needs the Heun integrator; meshes of
    different integrators do not batch."""
    import ctypes
    import torch
    w = case("blast3d", "ssprk3")
    gm, _ = build(w, 0)
    small = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        from paper_2605_07612_amd import _check, lib
        _check(lib().foap4_mesh_set_extra_state(gm.h, 2, ctypes.c_void_p(small.data_ptr()), 64), gm.h)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        _check(lib().foap4_mesh_set_extra_state(gm.h, 4, ctypes.c_void_p(small.data_ptr()), 1 << 30), gm.h)
    gm.capture_features(True)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        gm.step(1)
    gm.capture_features(False)
    gm.step(1)
    other, _ = build(case("blast3d", "ssprk43"), 0)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        f4.Batch([gm, other])


@pytest.mark.parametrize("integ", ["ssprk3", "rk4"])
def test_regrid_between_steps(f4, integ):
    """Steps, a regrid by the Lohner flags (bit-exact maps), more steps: the
    extra states hold intermediate stages only, so the integrators continue
    across the mesh change and match the oracle (FP64)."""
    w = case("blast3d", integ)
    import paper_2605_07612_amd as f4m
    from oracle import OracleMesh
    from paper_2605_07612_amd import layout
    from tests.gpu_helpers import scheme
    gm = f4m.Mesh(3, w["trees"], 8, 2, w["tree_size"], level=0, max_level=2, max_blocks=4 ** 3 * 64, prec=f4.F64,
                  gamma=w["gamma"], cfl=w["cfl"], integrator=integ, **scheme(w))
    om = OracleMesh(3, w["trees"], 8, 2, w["tree_size"], gamma=w["gamma"], cfl=w["cfl"], integrator=integ,
                    **scheme(w))
    _, G = layout.global_coords(gm)
    f0 = w["refine_flags"](G)
    gm.regrid(f0)
    om.regrid(f0, 0, 2)
    layout.set_from_field(gm, w["field"])
    om.set_interior_from_field(w["field"])
    gm.step(4)
    om.step(4)
    flags = gm.refine_flags()
    om.u[...] = 0.0
    om.interior()[...] = interior(gpu_state(gm), 2, 8, 3)
    om.ghost_fill()
    assert np.array_equal(flags, om.lohner_flags())
    assert gm.regrid(flags)
    om.regrid(flags, 0, 2)
    assert all(np.array_equal(a, b) for a, b in zip(gm.export(), om.forest.export()))
    gm.step(4)
    om.step(4)
    lev = gm.export()[0]
    err, err_elem = check_state(interior(gpu_state(gm), 2, 8, 3), om.interior(), lev, 3, w["tree_size"], 8, 1)
    say("regrid", integ, "levels", sorted(set(lev.tolist())), "rel L1", err)
    assert err <= TOL[1]


def test_bc_data_with_rk4(f4):
    """Spatially varying boundary values under RK4 (ghost fills of every
    sub-step read them) against the oracle given the same array (FP64)."""
    import torch
    w = case("box3d_options", "rk4")
    t = np.ones((6, 5), np.int32)
    t[:, 0] = t[:, 4] = 0
    val = np.zeros((6, 5))
    val[:, 0], val[:, 4] = 1.0, 0.25
    w.update(bc_type=t, bc_value=val, gravity=(0.0, 0.0, 0.0))
    gm, om = build(w, 1)
    pat = gm.pattern_export()
    nbc = len(pat["bc"])
    rng = np.random.default_rng(5)
    data = np.zeros((nbc, 5, 64))
    data[:, 0] = 1.0 + 0.1 * rng.random((nbc, 64))
    data[:, 4] = 0.25 + 0.05 * rng.random((nbc, 64))
    data[:, 1:4] = 0.05 * rng.standard_normal((nbc, 3, 64))
    gm.set_bc_data(torch.tensor(data, device="cuda"))
    om.set_bc_data(data)
    gm.step(5)
    om.step(5)
    lev = gm.export()[0]
    err, err_elem = check_state(interior(gpu_state(gm), 2, 8, 3), om.interior(), lev, 3, w["tree_size"], 8, 1)
    say("bc_data rk4 rel L1", err)
    assert err <= TOL[1]
