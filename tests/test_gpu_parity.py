"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Integer work (leaf tables, ghost patterns, flags, regrid
maps) must match bit for bit; FP64 states within 1e-12 and FP32 states within
2e-5 relative L1 (all variables, volume weighted)."""
import os
import sys

import numpy as np
import pytest

import synth
from oracle import OracleMesh
from tests.gpu_helpers import (build_pair, face_ghost_mask, gpu_mesh, gpu_state, interior, oracle_mesh,
                               check_state)

pytestmark = pytest.mark.gpu

TOL = {0: 2e-5, 1: 1e-12}  # by precision code: F32, F64


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


def small_uniform(N, trees, seed=0, ndim=3):
    """Noise/shear workload on a small periodic brick (any tree counts)."""
    gamma = 1.4
    nt = list(trees) + [1] * (3 - len(trees))

    def field(x, y, z=None):
        n = x.size
        u = synth.uniform_pm1(seed, n).reshape(x.shape)
        rho = 1 + 0.1 * u
        vx = 0.2 * np.sin(2 * np.pi * y)
        zero = 0 * x
        vel = [vx, zero] + ([zero] if ndim == 3 else [])
        return synth.conserved_from_primitive(rho, vel, 2.5 + 0 * x, gamma)

    return dict(name=f"small_{N}_{trees}", ndim=ndim, trees=tuple(nt), N=N, g=2,
                tree_size=1.0 / max(nt[:ndim]), level=0, gamma=gamma, cfl=0.5, field=field)


# ------------------------------------------------------------ topology parity

@pytest.mark.parametrize("wname", ["wave2d", "blast_small"])
def test_leaf_table_and_pattern_bit_exact(f4, wname):
    w = synth.periodic_2d_wave() if wname == "wave2d" else synth.two_level_blast(base_trees=4, block=8)
    say("case", wname)
    gm, om = build_pair(w, f4.F64)
    lev, tree, anc = gm.export()
    olev, otree, oanc = om.forest.export()
    assert np.array_equal(lev, olev) and np.array_equal(tree, otree)
    assert np.array_equal(anc[:, : w["ndim"]], oanc[:, : w["ndim"]])
    pg = gm.pattern_export()
    po = om.pat
    for key in ("srl", "srl_off", "f2c", "f2c_off", "c2f", "c2f_off"):
        assert np.array_equal(pg[key], po[key]), key


def test_pattern_counts_closed_forms(f4):
    """Uniform periodic: d * n_blocks SRL records; two-level blast (16^3 base
    of 8^3 blocks, ball of radius 1/4): 19956 SRL, 1440 F2C, 1440 C2F records."""
    w = synth.uniform_noise_shear(block=16, n=64)
    gm = gpu_mesh(w, f4.F32)
    c = gm.pattern_counts()
    assert c[0].sum() == 3 * gm.nb and c[1:].sum() == 0
    w3 = synth.two_level_blast(base_trees=16, block=8)
    gm3, _ = build_pair(w3, f4.F32, static_refine=False)
    from paper_2605_07612_amd import layout
    lev, G = layout.global_coords(gm3)
    gm3.regrid(w3["refine_flags"](G))
    c3 = gm3.pattern_counts()
    say("two-level counts", c3.sum(axis=1), gm3.nb)
    assert gm3.nb == 6952
    assert tuple(c3.sum(axis=1)[:3]) == (19956, 1440, 1440)


# ---------------------------------------------------------- ghost-fill parity

@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("wname", ["wave2d", "blast_small", "blast_small_2d", "blast_b16", "blast_b32"])
def test_ghost_fill_bit_exact(f4, prec, wname):
    """SRL copies, FP64 restriction sums and FP64 prolongation slopes equal the
    oracle bit for bit (FP32 states: the oracle on the same FP32 values, its
    FP64 result rounded once to FP32)."""
    if wname == "wave2d":
        w = synth.periodic_2d_wave()
    elif wname == "blast_small":
        w = synth.two_level_blast(base_trees=4, block=8)
    elif wname == "blast_b16":
        w = synth.two_level_blast(base_trees=4, block=16)
    elif wname == "blast_b32":
        w = synth.two_level_blast(base_trees=4, block=32)
    else:
        w = two_level_2d()
    say("case", wname, prec)
    gm, om = build_pair(w, prec)
    # identical inputs: the oracle takes the GPU's (possibly FP32) interior values
    om.u[...] = 0.0
    om.interior()[...] = interior(gpu_state(gm), w["g"], w["N"], w["ndim"])
    gm.ghost_fill()
    # an FP32 state stores the R1 ghosts in FP32 before R2 reads them
    om.ghost_round(1)
    if prec == 0:
        om.u[...] = om.u.astype(np.float32)
    om.ghost_round(2)
    mask = face_ghost_mask(w["ndim"], w["N"], w["g"])
    G = gpu_state(gm)[:, :, mask]
    O = om.u[:, :, mask]
    if prec == 0:
        O = O.astype(np.float32).astype(np.float64)
    assert np.array_equal(G, O)


# ------------------------------------------------------------------ time step

@pytest.mark.parametrize("prec", [1, 0])
def test_dt_bit_exact_on_identical_state(f4, prec):
    w = small_uniform(16, (2, 1, 3), seed=4)
    gm, om = build_pair(w, prec)
    om.interior()[...] = interior(gpu_state(gm), 2, 16, 3)
    gm.compute_dt()
    t, dt = gm.time()
    assert t == 0.0 and dt == om.dt()


# ------------------------------------------------------------- state parity

def run_pair(w, prec, steps, **kw):
    gm, om = build_pair(w, prec)
    t0 = gm.totals()
    gm.step(steps)
    t_gpu, dt_gpu = gm.time()
    om.step(steps)
    lev = gm.export()[0]
    a = interior(gpu_state(gm), w["g"], w["N"], w["ndim"])
    b = om.interior()
    err, err_elem = check_state(a, b, lev, w["ndim"], w["tree_size"], w["N"], prec)
    say(w["name"], "prec", prec, "steps", steps, "rel L1", err, "t", t_gpu, om.t)
    return gm, om, err, t_gpu, t0


@pytest.mark.parametrize("prec", [1, 0])
def test_wave2d_20_steps(f4, prec):
    w = synth.periodic_2d_wave()
    gm, om, err, t, _ = run_pair(w, prec, 20)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-13 if prec == 1 else 1e-5) * om.t


@pytest.mark.parametrize("prec", [1, 0])
@pytest.mark.parametrize("N,trees", [(16, (4, 4, 4)), (8, (3, 1, 2)), (32, (2, 1, 1))])
def test_uniform_noise_shear(f4, prec, N, trees):
    """Several tiles per block (N = 32), four blocks per workgroup with a
    ragged tail (N = 8, 6 blocks), one tile per block (N = 16)."""
    w = small_uniform(N, trees, seed=1)
    steps = 50 if N == 16 else 10
    gm, om, err, t, _ = run_pair(w, prec, steps)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [1, 0])
def test_noise_shear_64cubed_50_steps(f4, prec):
    w = synth.uniform_noise_shear(block=16, n=64, seed=0)
    gm, om, err, t, t0 = run_pair(w, prec, 50)
    assert err <= TOL[prec]
    drift = np.abs(gm.totals() - t0) / np.maximum(np.abs(t0), 1e-300)
    assert drift[0] <= (1e-12 if prec == 1 else 1e-6)


@pytest.mark.parametrize("prec", [1, 0])
def test_two_level_blast_small(f4, prec):
    """Restriction/prolongation ghosts and flux fixing on a static two-level
    mesh (8^3 base of 8^3-cell blocks): parity after 20 steps, conservation."""
    w = synth.two_level_blast(base_trees=8, block=8)
    gm, om, err, t, t0 = run_pair(w, prec, 20)
    assert err <= TOL[prec]
    tot = gm.totals()
    scale = np.abs(t0) + 1e-300
    assert abs(tot[0] - t0[0]) / scale[0] <= (1e-12 if prec == 1 else 1e-6)
    assert abs(tot[-1] - t0[-1]) / scale[-1] <= (1e-12 if prec == 1 else 1e-6)


def test_determinism_bitwise(f4):
    w = synth.two_level_blast(base_trees=4, block=8)
    a, _ = build_pair(w, 0)
    b, _ = build_pair(w, 0)
    a.step(10)
    b.step(10)
    assert np.array_equal(gpu_state(a), gpu_state(b))


# ---------------------------------------------------------------- regrid

@pytest.mark.parametrize("block", [8, 16])
def test_lohner_flags_and_regrid_bit_exact(f4, block):
    """Flags on identical states equal the oracle's; the regrid map (leaf
    table) and the remapped FP64 data equal the oracle's bit for bit."""
    w = synth.two_level_blast(base_trees=4, block=block)
    say("regrid parity, block", block)
    gm, om = build_pair(w, 1)
    gm.step(5)
    om.u[...] = 0.0
    om.interior()[...] = interior(gpu_state(gm), 2, block, 3)
    om.ghost_fill()
    fg = gm.refine_flags()
    fo = om.lohner_flags()
    say("flags", np.bincount(fg + 1, minlength=3))
    assert np.array_equal(fg, fo)
    # regrid both with the same flags (allow one more level)
    gm2 = gpu_mesh(w, 1, max_level=2, max_blocks=4 ** 3 * 64)
    om2 = oracle_mesh(w)
    from paper_2605_07612_amd import layout
    lev, G = layout.global_coords(gm2)
    f0 = w["refine_flags"](G)
    gm2.regrid(f0)
    om2.regrid(f0, 0, 2)
    layout.set_from_field(gm2, w["field"])
    om2.set_interior_from_field(w["field"])
    gm2.step(3)
    om2.u[...] = 0.0
    om2.interior()[...] = interior(gpu_state(gm2), 2, block, 3)
    flags = gm2.refine_flags()
    om2.ghost_fill()
    assert np.array_equal(flags, om2.lohner_flags())
    changed = gm2.regrid(flags)
    res = om2.regrid(flags, 0, 2)
    assert changed == (res is not None)
    lev2, tree2, anc2 = gm2.export()
    olev, otree, oanc = om2.forest.export()
    assert np.array_equal(lev2, olev) and np.array_equal(tree2, otree) and np.array_equal(anc2, oanc)
    a = interior(gpu_state(gm2), 2, block, 3)
    assert np.array_equal(a, om2.interior())


# ---------------------------------------------------------------- batch

@pytest.mark.parametrize("ks,order,wg1,wg2", [(2, 0, 2, 2), (2, 1, 2, 2), (2, 2, 2, 2), (2, 1, 8, 3), (2, 1, 0, 1),
                                             (4, 1, 0, 4), (1, 1, 3, 6)])
def test_batch_equals_plain_bitwise(f4, ks, order, wg1, wg2):
    """The persistent, graph-replayed batched form computes exactly what the
    plain per-kernel form computes (k-slabs, workgroup mapping, per-stage
    grids and item order only change who computes a face, not how)."""
    ws = [small_uniform(16, (2, 2, 2), seed=5), small_uniform(32, (1, 2, 1), seed=6),
          small_uniform(8, (3, 2, 1), seed=7)]
    plain = [build_pair(w, 0)[0] for w in ws]
    batched = [build_pair(w, 0)[0] for w in ws]
    for m in plain:
        m.step(4)
    b = f4.Batch(batched)
    b.set_config(kslabs=ks, wg_per_cu=wg1, xcd_order=order, wg_stage2=wg2)
    b.step(4)
    for w, p, q in zip(ws, plain, batched):
        a, c = interior(gpu_state(p), 2, w["N"], 3), interior(gpu_state(q), 2, w["N"], 3)
        say(w["name"], "times", p.time(), q.time(), "max |diff|", float(np.max(np.abs(a - c))))
        assert p.time() == q.time()
        assert np.array_equal(a, c)


def two_level_2d():
    """2D two-level workload: 4x4 base blocks of 8x8 cells, the blocks that
    meet the disc |x - 1/2| < 1/4 refined once, smooth non-trivial data."""
    w = dict(synth.two_level_blast(base_trees=4, block=8))
    w.update(ndim=2, trees=(4, 4, 1))
    base = w["refine_flags"]
    w["refine_flags"] = lambda G: base(np.concatenate([G[:, :2], np.full((len(G), 1), 1)], axis=1))
    w["field"] = lambda x, y: synth.conserved_from_primitive(1 + 0.3 * np.sin(7 * x) * np.cos(5 * y),
                                                              [0.1 + 0 * x, 0.2 + 0 * x], 1 + 0.5 * x * y, 1.4)
    return w


@pytest.mark.parametrize("ndim,block", [(3, 8), (2, 8), (3, 16), (3, 32)])
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("gather", [1, 0])
def test_batch_two_level_equals_plain(f4, prec, gather, ndim, block):
    """Refinement boundaries in the batched form: restriction and
    prolongation ghosts, halos gathered across same-level faces only, the
    SRL copies kept where the prolongation reads them, flux fixing and the
    per-stage grids give exactly the plain form's state, which is within
    tolerance of the oracle."""
    w = synth.two_level_blast(base_trees=4, block=block) if ndim == 3 else two_level_2d()
    steps = 12 if block < 32 else 4
    say("two-level batched vs plain, ndim", ndim, "block", block, "prec", prec, "gather", gather)
    gp, om = build_pair(w, prec)
    gb, _ = build_pair(w, prec)
    assert len(set(gp.export()[0].tolist())) == 2
    gp.step(steps)
    b = f4.Batch([gb])
    b.set_config(kslabs=2, wg_per_cu=2, xcd_order=1, gather_halos=gather, wg_stage2=3)
    b.step(steps)
    a, c = interior(gpu_state(gp), 2, block, ndim), interior(gpu_state(gb), 2, block, ndim)
    say("times", gp.time(), gb.time(), "max |diff|", float(np.max(np.abs(a - c))))
    assert gp.time() == gb.time()
    assert np.array_equal(a, c)
    om.step(steps)
    lev = gb.export()[0]
    err, err_elem = check_state(c, om.interior(), lev, ndim, w["tree_size"], block, prec)
    say("rel L1 vs oracle", err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_follows_regrid(f4, prec):
    """A batch keeps working across a regrid of its mesh (new leaf table,
    pattern and work items; the step graph is captured again): step, regrid
    with the criterion's flags, step again - bit for bit the plain form's
    result, and the same leaf table."""
    w = synth.two_level_blast(base_trees=4, block=8)
    pair = []
    for _ in range(2):
        gm = f4.Mesh(3, w["trees"], 8, 2, w["tree_size"], level=1, max_level=2,
                     max_blocks=4 ** 3 * 8 * 8, prec=prec)
        from paper_2605_07612_amd import layout
        layout.set_from_field(gm, w["field"])
        pair.append(gm)
    gp, gb = pair
    b = f4.Batch([gb])
    b.set_config(kslabs=1, wg_per_cu=0, xcd_order=1, wg_stage2=4)
    gp.step(4)
    b.step(4)
    fp, fb = gp.refine_flags(), gb.refine_flags()
    assert np.array_equal(fp, fb) and (fp == 1).any()
    assert gp.regrid(fp) and gb.regrid(fb)
    say("blocks after regrid", gp.nb, gb.nb)
    gp.step(4)
    b.step(4)
    assert all(np.array_equal(x, y) for x, y in zip(gp.export(), gb.export()))
    a, c = interior(gpu_state(gp), 2, 8, 3), interior(gpu_state(gb), 2, 8, 3)
    assert gp.time() == gb.time()
    assert np.array_equal(a, c)


@pytest.mark.parametrize("g", [3, 4])
@pytest.mark.parametrize("two_level", [False, True], ids=["uniform", "two_level"])
def test_wider_ghost_layers(f4, g, two_level):
    """Blocks with 3 or 4 ghost layers (the stencil reads 2 of them): the
    ghost rounds fill all g layers bit for bit as the oracle does, and the
    plain and batched steps agree with the oracle (FP64) and with each other."""
    if two_level:
        w = dict(synth.two_level_blast(base_trees=4, block=16), g=g)
    else:
        w = dict(small_uniform(16, (2, 2, 2), seed=9), g=g)
    say("ghost layers", g, "two-level", two_level)
    gm, om = build_pair(w, 1)
    gb, _ = build_pair(w, 1)
    # ghost rounds on identical data, all g layers
    om.u[...] = 0.0
    om.interior()[...] = interior(gpu_state(gm), g, 16, 3)
    gm.ghost_fill()
    om.ghost_fill()
    mask = face_ghost_mask(3, 16, g)
    assert np.array_equal(gpu_state(gm)[:, :, mask], om.u[:, :, mask])
    gm.step(6)
    b = f4.Batch([gb])
    b.set_config(kslabs=2, wg_per_cu=0, xcd_order=1, wg_stage2=4)
    b.step(6)
    om.step(6)
    a, c = interior(gpu_state(gm), g, 16, 3), interior(gpu_state(gb), g, 16, 3)
    assert gm.time() == gb.time() and np.array_equal(a, c)
    lev = gm.export()[0]
    err, err_elem = check_state(a, om.interior(), lev, 3, w["tree_size"], 16, 1)
    say("rel L1 vs oracle", err)
    assert err <= TOL[1]


def test_batch_mixed_sizes_vs_oracle(f4):
    ws = [synth.batch_problem(p) for p in (51, 34, 1, 9, 6, 52)]  # the six smallest
    pairs = [build_pair(w, 0) for w in ws]
    b = f4.Batch([g for g, _ in pairs])
    b.set_config(kslabs=2, wg_per_cu=4)
    b.step(5)
    for w, (gm, om) in zip(ws, pairs):
        om.step(5)
        lev = gm.export()[0]
        err, err_elem = check_state(interior(gpu_state(gm), 2, w["N"], 3), om.interior(), lev, 3, w["tree_size"], w["N"], 0)
        say(w["name"], w["N"], gm.nb, err)
        assert err <= TOL[0]
