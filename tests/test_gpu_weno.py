"""GPU parity of the WENO5 reconstruction (Sec. 3.2 limiter list, three ghost
layers) against the FP64 oracle, through the C ABI: FP64 within 1e-12 and
FP32 within 2e-5 relative L1, on two-level meshes (restriction, prolongation
and flux fixing with g = 3) and on the Rayleigh-Taylor workload with its
walls, with Heun, SSP-RK3 and RK4, Rusanov and HLL."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_helpers import gpu_state, interior, check_state

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
        return synth.conserved_from_primitive(1.0 + 0 * r, [0 * r, 0 * r], np.where(r < 0.12, 10.0, 0.1), 1.4)

    def refine_flags(G):
        G = np.asarray(G)
        return np.all((G[:, :2] >= 3) & (G[:, :2] <= 4), axis=1).astype(np.int8)

    return dict(name="blast2d", ndim=2, trees=(8, 8, 1), N=8, g=3, tree_size=1.0 / 8, level=0, gamma=1.4,
                cfl=0.5, field=field, refine_flags=refine_flags)


def case(name, integ, flux="rusanov"):
    if name == "blast3d":
        w = dict(synth.two_level_blast(base_trees=4, block=8))
        w["field"] = synth.blast_field(p_in=10.0, p_out=0.1, r0=0.15, centre=(0.45, 0.55, 0.5))
    elif name == "blast2d":
        w = blast2d()
    else:
        w = dict(synth.rayleigh_taylor(block=16, n=64))
    w.update(g=3, limiter="weno5", flux=flux, integrator=integ, name=f'{w["name"]}_weno5_{integ}_{flux}')
    return w


def build(w, prec):
    import paper_2605_07612_amd as f4
    from oracle import OracleMesh
    from paper_2605_07612_amd import layout
    from tests.gpu_helpers import scheme
    max_level = 1 if "refine_flags" in w else 0
    base = int(np.prod(w["trees"][: w["ndim"]]))
    gm = f4.Mesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], level=0, max_level=max_level,
                 max_blocks=base * (1 << w["ndim"]) if "refine_flags" in w else None, prec=prec, gamma=w["gamma"],
                 cfl=w["cfl"], integrator=w["integrator"], **scheme(w))
    om = OracleMesh(w["ndim"], w["trees"], w["N"], w["g"], w["tree_size"], gamma=w["gamma"], cfl=w["cfl"],
                    integrator=w["integrator"], **scheme(w))
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
@pytest.mark.parametrize("name,integ,flux", [("blast3d", "heun", "rusanov"), ("blast3d", "ssprk3", "hll"),
                                             ("blast3d", "rk4", "rusanov"), ("blast2d", "heun", "hll"),
                                             ("blast2d", "rk4", "rusanov"), ("rt3d", "heun", "rusanov"),
                                             ("rt3d", "rk4", "hll")])
def test_parity(f4, name, integ, flux, prec):
    w = case(name, integ, flux)
    gm, om = build(w, prec)
    steps = 6
    gm.step(steps)
    om.step(steps)
    t, _ = gm.time()
    lev = gm.export()[0]
    a = interior(gpu_state(gm), w["g"], w["N"], w["ndim"])
    err, err_elem = check_state(a, om.interior(), lev, w["ndim"], w["tree_size"], w["N"], prec)
    say(w["name"], "prec", prec, "levels", sorted(set(lev.tolist())), "rel L1", err, "t", t, om.t)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-13 if prec == 1 else 1e-5) * om.t


def test_conservation_on_two_levels(f4):
    w = case("blast3d", "heun")
    gm, _ = build(w, 1)
    t0 = gm.totals()
    gm.step(20)
    drift = np.abs(gm.totals() - t0) / (np.abs(t0) + 1.0)
    say("WENO5 two-level drift", drift)
    assert drift[0] <= 1e-13 and drift[-1] <= 1e-13


def test_refusals(f4):
    """WENO5 needs three ghost layers, a batch takes WENO5 meshes only
    together, and feature capture needs a two-ghost limiter."""
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        f4.Mesh(3, (2, 2, 2), 8, 2, 0.5, prec=f4.F32, limiter="weno5")
    w = case("blast3d", "heun")
    gm, _ = build(w, 0)
    other = f4.Mesh(3, (2, 2, 2), 8, 3, 0.5, prec=f4.F32)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        f4.Batch([gm, other])
    gm.capture_features(True)
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        gm.step(1)
    gm.capture_features(False)
    gm.step(1)


@pytest.mark.parametrize("integ", ["heun", "rk4"])
@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
def test_batch_equals_plain(f4, integ, prec):
    """WENO5 meshes in a batch (the two-level blast and the walled
    Rayleigh-Taylor workload, one scheme and integrator): the captured step
    launches the WENO5 kernel per mesh and equals the plain step bit for bit."""
    rt = case("rt3d", integ)
    bl = case("blast3d", integ)
    bl.update(gravity=rt["gravity"])
    ws = [bl, rt]
    plain = [build(w, prec)[0] for w in ws]
    batched = [build(w, prec)[0] for w in ws]
    for m in plain:
        m.step(3)
    b = f4.Batch(batched)
    b.step(3)
    for w, p, q in zip(ws, plain, batched):
        A = interior(gpu_state(p), w["g"], w["N"], w["ndim"])
        B = interior(gpu_state(q), w["g"], w["N"], w["ndim"])
        assert np.array_equal(A, B), w["name"]
        assert p.time() == q.time()
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        b.phase_times(1)
    b.close()


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("N,g", [(32, 3), (16, 4), (8, 4)])
def test_parity_block_shapes(f4, N, g, prec):
    """Both 3-D WENO5 kernels on two levels (one of eight trees refined, the
    blast across the level boundary): 32^3 blocks take the per-cell kernel,
    16^3 and 8^3 blocks the marching kernel, here with four ghost layers of
    which the stencil reads the inner three.  The jump is 4:1: WENO5 has no
    positivity limiter, and a 100:1 jump over the one- and two-cell steps of
    the sampled sphere at the level boundary drives reconstructed pressures
    negative (the oracle reports such states as unphysical)."""
    w = dict(name=f"blast3d_b{N}_g{g}_weno5", ndim=3, trees=(2, 2, 2), N=N, g=g, tree_size=0.5, level=0, gamma=1.4,
             cfl=0.5, field=synth.blast_field(p_in=4.0, p_out=1.0, r0=0.15, centre=(0.42, 0.47, 0.5)),
             refine_flags=lambda G: np.all(np.asarray(G)[:, :3] == 0, axis=1).astype(np.int8),
             limiter="weno5", flux="hll", integrator="heun")
    gm, om = build(w, prec)
    steps = 4
    gm.step(steps)
    om.step(steps)
    lev = gm.export()[0]
    assert sorted(set(lev.tolist())) == [0, 1]
    err, err_elem = check_state(interior(gpu_state(gm), g, N, 3), om.interior(), lev, 3, w["tree_size"], N, prec)
    say(w["name"], "prec", prec, "blocks", len(lev), "rel L1", err)
    assert err <= TOL[prec]
