"""GPU parity of the scheme options (Sec. 3.2 limiters and fluxes, the
gravity source of Sec. 4.2) against the FP64 oracle, through the C ABI:
FP64 states within 1e-12 and FP32 states within 2e-5 relative L1 (volume
weighted, all variables), on two-level meshes (restriction, prolongation,
flux fixing) and on the Rayleigh-Taylor workload; the batched form equal to
the plain one bit for bit."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_helpers import build_pair, gpu_state, interior, check_state

pytestmark = pytest.mark.gpu

TOL = {0: 2e-5, 1: 1e-12}
# scheme bit mask: 1 van Leer, 2 HLL, 4 gravity
SCHEMES = list(range(8))


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


def with_scheme(w, sch, grav=(0.3, -0.5, -1.0)):
    w = dict(w)
    w["limiter"] = "vanleer" if sch & 1 else "minmod"
    w["flux"] = "hll" if sch & 2 else "rusanov"
    w["gravity"] = tuple(grav[: w["ndim"]]) if sch & 4 else (0.0, 0.0, 0.0)
    w["name"] = f'{w["name"]}_s{sch}'
    return w


def two_level_2d():
    """2D two-level blast: 8x8 base blocks of 8^2, the central 2x2 refined."""
    gamma = 1.4

    def field(x, y):
        r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2)
        rho = 1.0 + 0 * r
        p = np.where(r < 0.1, 10.0, 0.1)
        zero = 0 * r
        return synth.conserved_from_primitive(rho, [zero, zero], p, gamma)

    def refine_flags(G):
        G = np.asarray(G)
        return np.all((G[:, :2] >= 3) & (G[:, :2] <= 4), axis=1).astype(np.int8)

    return dict(name="blast2d", ndim=2, trees=(8, 8, 1), N=8, g=2, tree_size=1.0 / 8, level=0, gamma=gamma,
                cfl=0.5, field=field, refine_flags=refine_flags)


def run_pair(w, prec, steps):
    gm, om = build_pair(w, prec)
    gm.step(steps)
    t_gpu, _ = gm.time()
    om.step(steps)
    lev = gm.export()[0]
    a = interior(gpu_state(gm), w["g"], w["N"], w["ndim"])
    err, err_elem = check_state(a, om.interior(), lev, w["ndim"], w["tree_size"], w["N"], prec)
    say(w["name"], "prec", prec, "steps", steps, "levels", sorted(set(lev.tolist())), "rel L1", err, "t", t_gpu, om.t)
    return gm, om, err, t_gpu


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("sch", SCHEMES)
def test_two_level_blast_3d(f4, sch, prec):
    """Every scheme on the 3D two-level blast (4^3 base of 8^3 blocks, the
    ball refined once): 10 steps against the oracle."""
    w = with_scheme(synth.two_level_blast(base_trees=4, block=8), sch)
    gm, om, err, t = run_pair(w, prec, 10)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-13 if prec == 1 else 1e-5) * om.t


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("sch", SCHEMES)
def test_two_level_blast_2d(f4, sch, prec):
    w = with_scheme(two_level_2d(), sch, grav=(0.4, -1.0, 0.0))
    gm, om, err, t = run_pair(w, prec, 20)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
@pytest.mark.parametrize("block", [8, 16, 32])
def test_rayleigh_taylor(f4, block, prec):
    """The Rayleigh-Taylor workload of Sec. 4.2 (van Leer, gravity) on 64^3
    cells: one, several and four-per-workgroup tiles per block."""
    w = synth.rayleigh_taylor(block=block, n=64)
    gm, om, err, t = run_pair(w, prec, 10)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [1, 0], ids=["f64", "f32"])
def test_rayleigh_taylor_2d(f4, prec):
    w = synth.rayleigh_taylor(block=16, n=128, ndim=2)
    gm, om, err, t = run_pair(w, prec, 30)
    assert err <= TOL[prec]


@pytest.mark.parametrize("sch", [1, 2, 5, 7])
@pytest.mark.parametrize("prec", [0, 1], ids=["f32", "f64"])
def test_batch_equals_plain(f4, sch, prec):
    """The batched step (two meshes of 8^3 and 16^3 blocks, one two-level)
    equals the plain step of each mesh bit for bit under every scheme."""
    ws = [with_scheme(synth.two_level_blast(base_trees=4, block=8), sch),
          with_scheme(synth.rayleigh_taylor(block=16, n=64), sch)]
    plain, batched = [], []
    for w in ws:
        a, _ = build_pair(w, prec)
        b, _ = build_pair(w, prec)
        plain.append(a)
        batched.append(b)
    for m in plain:
        m.step(5)
    b = f4.Batch(batched)
    b.set_config(kslabs=2, wg_per_cu=2, xcd_order=1)
    b.step(5)
    for w, p, q in zip(ws, plain, batched):
        A = interior(gpu_state(p), w["g"], w["N"], w["ndim"])
        B = interior(gpu_state(q), w["g"], w["N"], w["ndim"])
        say(w["name"], "max |batch - plain|", float(np.max(np.abs(A - B))))
        assert np.array_equal(A, B)
        assert p.time() == q.time()
    b.close()


def test_batch_refuses_mixed_schemes(f4):
    a, _ = build_pair(with_scheme(synth.two_level_blast(base_trees=2, block=8), 0), 0)
    for sch in (1, 2, 4):
        b, _ = build_pair(with_scheme(synth.two_level_blast(base_trees=2, block=8), sch), 0)
        with pytest.raises(f4.Foap4Error, match="E_INVALID"):
            f4.Batch([a, b])
    # gravity of another value is the same scheme
    c, _ = build_pair(with_scheme(synth.two_level_blast(base_trees=2, block=8), 4, grav=(0.0, 0.0, -2.0)), 0)
    d, _ = build_pair(with_scheme(synth.two_level_blast(base_trees=2, block=8), 4), 0)
    f4.Batch([c, d]).close()


@pytest.mark.parametrize("sch", [5, 7])
def test_feature_capture_keeps_the_step(f4, sch):
    """The stage-1 kernel that also reduces block features runs the same
    scheme: a step with capture on equals a step with capture off, and the
    captured features equal those computed from the step's input state."""
    w = with_scheme(synth.two_level_blast(base_trees=4, block=8), sch)
    a, _ = build_pair(w, 0)
    b, _ = build_pair(w, 0)
    a.step(2)
    b.step(2)
    ref = b.block_features().cpu().numpy()
    b.capture_features(True)
    a.step(1)
    b.step(1)
    assert np.array_equal(interior(gpu_state(a), 2, 8, 3), interior(gpu_state(b), 2, 8, 3))
    cap = b.captured_features().cpu().numpy()
    # FP32 state: both kernels round the log features in FP32
    assert np.max(np.abs(cap - ref)) <= 2e-5 * max(1.0, float(np.max(np.abs(ref))))
