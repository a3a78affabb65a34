"""GPU parity of the learned refinement indicator against its FP64 oracle
(oracle/mlp.py, which rounds every matrix-product operand to BF16 as the
matrix cores do).  Raw per-block maxima are FP64 and must match bit for bit;
features within FP32 rounding; logits and gradients within the error of FP32
accumulation (gradients <= 1e-3 relative); flags equal except where the
oracle's top-two logit margin or its distance to the confidence threshold is
below what that error can flip."""
import sys

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from tests.gpu_helpers import build_pair

pytestmark = pytest.mark.gpu


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


def wave2d_refined():
    w = synth.periodic_2d_wave()
    w["refine_flags"] = lambda G: (((G[:, 0] + 2 * G[:, 1]) % 3) == 0).astype(np.int8)
    return w


def noise3d_refined():
    """Seeded density noise on 4^3 trees of 8^3 cells, a diagonal band of
    trees refined once."""
    gamma = 1.4

    def field(x, y, z):
        u = synth.uniform_pm1(77, x.size).reshape(x.shape)
        rho = 1.0 + 0.3 * u
        p = 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * z)
        return synth.conserved_from_primitive(rho, [0.1 + 0 * x, 0 * x, 0 * x], p, gamma)

    return dict(name="noise3d_refined", ndim=3, trees=(4, 4, 4), N=8, g=2, tree_size=0.25, level=0,
                gamma=gamma, cfl=0.5, field=field,
                refine_flags=lambda G: ((G[:, 0] + G[:, 1] + G[:, 2]) % 4 == 1).astype(np.int8))


def noise3d_bounded():
    """noise3d_refined bounded along x and z by random Dirichlet / Neumann
    faces: the raw features read boundary ghosts, and boundary faces have no
    neighbour summary (zero on both sides)."""
    w = noise3d_refined()
    rng = np.random.default_rng(31)
    t = rng.integers(0, 2, (6, 5)).astype(np.int32)
    # Dirichlet values that keep mirrored ghosts physical: rho in [1, 1.5]
    # (interior 0.7 .. 1.3), momenta small, E in [2, 3] (interior 1.25 .. 3.8)
    lo, hi = np.array([1.0, -0.2, -0.2, -0.2, 2.0]), np.array([1.5, 0.2, 0.2, 0.2, 3.0])
    v = rng.uniform(lo, hi, (6, 5))
    v[t == 1] = rng.uniform(-0.3, 0.3, int((t == 1).sum()))
    w.update(name="noise3d_bounded", periodic=(False, True, False), bc_type=t, bc_value=v)
    return w


WORKLOADS = {"wave2d_refined": wave2d_refined, "noise3d_refined": noise3d_refined,
             "noise3d_bounded": noise3d_bounded,
             "blast_small": lambda: synth.two_level_blast(base_trees=4, block=8),
             "blast_b16": lambda: synth.two_level_blast(base_trees=4, block=16),
             "blast_b32": lambda: synth.two_level_blast(base_trees=4, block=32)}


def oracle_features(om, lmax):
    om.ghost_fill()
    raw = om.raw_features()
    return raw, omlp.features(om.forest, raw, lmax=lmax, ndim=om.ndim)


@pytest.mark.parametrize("wname", list(WORKLOADS))
def test_features_match_oracle(f4, wname):
    w = WORKLOADS[wname]()
    say("case", wname)
    gm, om = build_pair(w, f4.F64)
    assert gm.export()[0].tolist() == om.level.tolist()
    feat, raw = gm.block_features(raw=True)
    raw_o, F_o = oracle_features(om, lmax=1)
    raw_g = raw.cpu().numpy()
    assert np.array_equal(raw_g, raw_o), np.max(np.abs(raw_g - raw_o))
    F_g = feat.cpu().numpy().astype(np.float64)
    # FP32 rounding of FP64 values (log1p may differ in its last FP64 bit)
    assert np.all(np.abs(F_g - F_o) <= 1.2e-7 * np.abs(F_o) + 1e-38), np.max(np.abs(F_g - F_o))
    assert np.all(F_g[:, 15] == 0)
    if w["ndim"] == 2:
        assert np.all(F_g[:, 11:15] == 0)
    # a refined mesh: coarse/fine neighbour slots were exercised
    assert len(set(om.level.tolist())) == 2


def test_features_fp32_state(f4):
    """FP32 state: the oracle evaluates the same initial values (rounded to
    FP32 by the input generator) in FP64; ghosts of the F2C/C2F rounds are
    rounded to FP32 on the GPU, so agreement is to FP32 rounding."""
    w = noise3d_refined()
    gm, om = build_pair(w, f4.F32)
    om.interior()[...] = om.interior().astype(np.float32).astype(np.float64)
    feat = gm.block_features().cpu().numpy().astype(np.float64)
    _, F_o = oracle_features(om, lmax=1)
    assert np.max(np.abs(feat - F_o)) <= 2e-5 * np.max(np.abs(F_o))


def rows(n, seed):
    X = (synth.uniform_pm1(seed, n * 16).reshape(n, 16) * 2.0).astype(np.float32)
    X[:, 15] = 0.0
    y = (np.floor(synth.uniform01(seed + 1, n) * 3) - 1).astype(np.int8)
    return X, y


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [1, 45, 5000])
def test_forward_logits(f4, n):
    X, _ = rows(n, 21)
    w = omlp.init_weights(4).astype(np.float32)
    net = f4.Mlp(w)
    z = net.forward(to_dev(X)).cpu().numpy().astype(np.float64)
    zo = omlp.forward(w.astype(np.float64), X.astype(np.float64), emulate=True)["z3"]
    scale = np.max(np.abs(zo))
    err = np.abs(z - zo)
    say("n", n, "max err", err.max() / scale, "rel", np.linalg.norm(z - zo) / np.linalg.norm(zo))
    assert np.linalg.norm(z - zo) <= 1e-4 * np.linalg.norm(zo)
    assert err.max() <= 1e-2 * scale


@pytest.mark.parametrize("n", [7, 3001])
def test_gradient_matches_oracle(f4, n):
    X, y = rows(n, 31)
    w = omlp.init_weights(6).astype(np.float32)
    cw = np.array([2.0, 0.5, 3.0])
    net = f4.Mlp(w)
    loss, g = net.loss_grad(to_dev(X), to_dev(y), cw)
    lo, go = omlp.loss_and_grad(w.astype(np.float64), X.astype(np.float64), y, cw, emulate=True)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    say("n", n, "loss", loss, lo, "grad rel", rel)
    assert loss == pytest.approx(lo, rel=1e-5)
    assert rel <= 1e-3
    # each parameter block separately (a transposed or misplaced block fails here)
    o = 0
    for name, shape in omlp.SIZES:
        k = int(np.prod(shape))
        gb, ob = g[o:o + k], go[o:o + k]
        assert np.linalg.norm(gb - ob) <= 2e-3 * np.linalg.norm(ob) + 1e-9, name
        o += k


def test_gradient_deterministic(f4):
    X, y = rows(20000, 41)
    net = f4.Mlp(omlp.init_weights(2).astype(np.float32))
    a = net.loss_grad(to_dev(X), to_dev(y))
    b = net.loss_grad(to_dev(X), to_dev(y))
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_adam_training_follows_oracle(f4):
    """Full-batch Adam on the GPU against the oracle's own Adam trajectory
    (each side uses its own gradients)."""
    X, _ = rows(2000, 51)
    y = np.where(X[:, 0] > 0.5, 1, np.where(X[:, 0] < -0.5, -1, 0)).astype(np.int8)
    w0 = omlp.init_weights(3).astype(np.float32)
    net = f4.Mlp(w0)
    iters, lr = 10, 1e-2
    losses = net.train(to_dev(X), to_dev(y), iters, lr=lr)
    wg = net.get_params().astype(np.float64)
    wo = w0.astype(np.float64)
    m = np.zeros_like(wo)
    v = np.zeros_like(wo)
    lo = []
    for t in range(1, iters + 1):
        l, g = omlp.loss_and_grad(wo, X.astype(np.float64), y, np.ones(3), emulate=True)
        lo.append(l)
        wo, m, v = omlp.adam_step(wo, g, m, v, t, lr=lr)
    say("losses", losses[:3], lo[:3], "final", losses[-1], lo[-1])
    assert np.allclose(losses, lo, rtol=1e-4)
    d = np.abs(wg - wo)
    # a parameter whose gradient is near zero may take the other sign step
    assert np.mean(d <= 1e-5 + 1e-5 * np.abs(wo)) >= 0.99
    assert d.max() <= 2 * iters * lr


def test_training_reduces_loss(f4):
    X, _ = rows(4000, 61)
    y = np.where(X[:, 1] + 0.5 * X[:, 2] > 0.6, 1, np.where(X[:, 1] < -0.6, -1, 0)).astype(np.int8)
    net = f4.Mlp(omlp.init_weights(8).astype(np.float32))
    losses = net.train(to_dev(X), to_dev(y), 300, lr=1e-2)
    say("loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.3 * losses[0]
    assert np.all(np.isfinite(losses))


def test_bad_labels_rejected(f4):
    X, y = rows(100, 71)
    y[17] = 2
    net = f4.Mlp(omlp.init_weights(1).astype(np.float32))
    with pytest.raises(f4.Foap4Error, match="E_INVALID"):
        net.loss_grad(to_dev(X), to_dev(y))


def scaled_weights(seed, scale):
    w = omlp.unpack(omlp.init_weights(seed))
    w["W3"] = w["W3"] * scale
    w["b3"] = np.array([0.3, -0.2, 0.1])
    return omlp.pack(w).astype(np.float32)


@pytest.mark.parametrize("wname", ["noise3d_refined", "blast_small"])
def test_refine_flags_mlp(f4, wname):
    """MLP flags with and without the Lohner fallback against the oracle's
    prediction on its own features and Lohner flags."""
    w = WORKLOADS[wname]()
    say("case", wname)
    gm, om = build_pair(w, f4.F64)
    wt = scaled_weights(12, 8.0)
    net = f4.Mlp(wt)
    with pytest.raises(f4.Foap4Error, match="E_ORDER"):
        gm.refine_flags(f4.IND_MLP)
    gm.set_indicator(f4.IND_MLP, net)
    _, F_o = oracle_features(om, lmax=1)
    z = omlp.forward(wt.astype(np.float64), F_o, emulate=True)["z3"]
    P = omlp.softmax(z)
    zs = np.sort(z, axis=1)
    margin = zs[:, 2] - zs[:, 1]
    lohner = om.lohner_flags()
    # pure network (threshold 0)
    net.set_threshold(0.0)
    fg = gm.refine_flags(f4.IND_MLP)
    fo, _ = omlp.predict_flags(wt.astype(np.float64), F_o, lohner=None)
    safe = margin > 1e-3
    assert np.array_equal(fg[safe], fo[safe]), np.nonzero(fg != fo)
    assert gm.fallbacks() == 0
    # with the fallback
    net.set_threshold(0.5)
    fg = gm.refine_flags(f4.IND_MLP)
    fo, _ = omlp.predict_flags(wt.astype(np.float64), F_o, lohner=lohner, threshold=0.5)
    safe &= np.abs(P.max(axis=1) - 0.5) > 1e-3
    say("fallbacks", gm.fallbacks(), "of", len(fg), "safe", int(safe.sum()))
    assert np.array_equal(fg[safe], fo[safe])
    low = P.max(axis=1) < 0.5
    assert abs(gm.fallbacks() - int(low.sum())) <= int((~safe).sum())
    assert 0 < gm.fallbacks() < len(fg) or wname == "blast_small"
    # the Lohner indicator is unchanged by an attached network
    assert np.array_equal(gm.refine_flags(f4.IND_LOHNER), lohner)


def test_regrid_uses_attached_indicator(f4):
    w = noise3d_refined()
    g1, _ = build_pair(w, f4.F64)
    g2, _ = build_pair(w, f4.F64)
    net = f4.Mlp(scaled_weights(12, 8.0))
    g1.set_indicator(f4.IND_MLP, net)
    g2.set_indicator(f4.IND_MLP, net)
    flags = g2.refine_flags(f4.IND_MLP)
    c1 = g1.regrid()
    c2 = g2.regrid(flags)
    assert c1 == c2
    l1, l2 = g1.export(), g2.export()
    assert all(np.array_equal(a, b) for a, b in zip(l1, l2))
    assert np.array_equal(g1.current().cpu().numpy(), g2.current().cpu().numpy())


@pytest.mark.parametrize("wname,prec", [("noise3d_refined", 1), ("noise3d_refined", 0), ("noise3d_bounded", 1),
                                        ("noise3d_bounded", 0), ("wave2d_refined", 1),
                                        ("blast_small", 1), ("blast_b16", 1), ("blast_b16", 0)])
def test_captured_features_match_oracle(f4, wname, prec):
    """Features captured inside the first stage of a step describe the state
    at the start of that step: compare with the oracle's features of that
    state (FP64: to rounding of the reciprocal-multiply; FP32: to FP32
    rounding of the log features)."""
    w = WORKLOADS[wname]()
    say("case", wname, prec)
    gm, om = build_pair(w, prec)
    if prec == 0:
        om.interior()[...] = om.interior().astype(np.float32).astype(np.float64)
    raw_o, F_o = oracle_features(om, lmax=1)
    with pytest.raises(f4.Foap4Error, match="E_ORDER"):
        gm.captured_features()
    gm.capture_features(True)
    gm.step(1)
    feat, raw = gm.captured_features(raw=True)
    raw_g, F_g = raw.cpu().numpy(), feat.cpu().numpy().astype(np.float64)
    if prec == 1:
        # r is a ratio of O(1) state values: rounding differences are ~1e-16
        # absolute (a uniform pressure gives r1 ~ 1e-16 of pure rounding)
        assert np.allclose(raw_g, raw_o, rtol=1e-12, atol=1e-13), np.max(np.abs(raw_g - raw_o))
        assert np.all(np.abs(F_g - F_o) <= 1.2e-7 * np.abs(F_o) + 1e-13)
    else:
        assert np.max(np.abs(F_g - F_o)) <= 2e-5 * max(1.0, np.max(np.abs(F_o)))
    # the values are those of one step: a later step without capture retires them
    gm.capture_features(False)
    gm.step(1)
    with pytest.raises(f4.Foap4Error, match="E_ORDER"):
        gm.captured_features()


def test_mlp_flags_from_captured_features(f4):
    """With captured features the MLP flags equal the network on those
    features (the fallback taking the criterion's flag of the current state)."""
    w = noise3d_refined()
    gm, om = build_pair(w, 1)
    wt = scaled_weights(12, 8.0)
    net = f4.Mlp(wt)
    gm.set_indicator(f4.IND_MLP, net)
    raw_o, F_o = oracle_features(om, lmax=1)
    gm.capture_features(True)
    gm.step(1)
    net.set_threshold(0.0)
    fg = gm.refine_flags(f4.IND_MLP)
    z = omlp.forward(wt.astype(np.float64), F_o, emulate=True)["z3"]
    zs = np.sort(z, axis=1)
    safe = (zs[:, 2] - zs[:, 1]) > 1e-3
    fo, _ = omlp.predict_flags(wt.astype(np.float64), F_o, lohner=None)
    assert np.array_equal(fg[safe], fo[safe])
    assert gm.fallbacks() == 0
    # with the fallback: undecided blocks get the criterion's flag of the
    # current state; the oracle follows the same two steps
    net.set_threshold(0.5)
    om.step(1)
    _, F_o1 = oracle_features(om, lmax=1)   # the state the second step starts from
    gm.step(1)
    om.step(1)
    om.ghost_fill()
    fl_o = om.lohner_flags()
    fm = gm.refine_flags(f4.IND_MLP)
    P = omlp.softmax(omlp.forward(wt.astype(np.float64), F_o1, emulate=True)["z3"])
    pm = P.max(axis=1)
    low, ok = pm < 0.5, np.abs(pm - 0.5) > 1e-3
    say("fallbacks", gm.fallbacks(), "oracle low", int(low.sum()))
    assert np.array_equal(fm[low & ok], fl_o[low & ok])
    fo1, _ = omlp.predict_flags(wt.astype(np.float64), F_o1, lohner=fl_o, threshold=0.5)
    zs = np.sort(omlp.forward(wt.astype(np.float64), F_o1, emulate=True)["z3"], axis=1)
    safe = ok & ((zs[:, 2] - zs[:, 1]) > 1e-3)
    assert np.array_equal(fm[safe], fo1[safe])
    assert abs(gm.fallbacks() - int(low.sum())) <= int((~ok).sum())
