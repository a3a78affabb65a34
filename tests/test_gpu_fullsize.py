"""GPU parity at the workloads' full sizes, in the launch configuration that
bench.py times (batched: stage 1 one workgroup per work item, stage 2 a
persistent grid of 4 workgroups per CU, XCD-contiguous item order, gathered
halos).  The oracle computes the same steps at full size where it finishes
in seconds; otherwise properties that hold at any size are checked."""
import sys

import numpy as np
import pytest

import synth
from tests.gpu_helpers import build_pair, gpu_state, interior, rel_l1_vol

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


@pytest.mark.parametrize("prec", [0, 1])
def test_noise_shear_256cubed_full_size(f4, prec):
    """The benchmark workload (256^3 cells, 4096 blocks of 16^3): two batched
    steps against two oracle steps, every cell compared."""
    w = synth.uniform_noise_shear(block=16, n=256, seed=0)
    say("case 256^3 prec", prec)
    gm, om = build_pair(w, prec)
    b = f4.Batch([gm])
    b.set_config(kslabs=1, wg_per_cu=0, xcd_order=1, wg_stage2=4)  # the configuration the benchmark times
    b.step(2)
    t, dt = gm.time()
    om.step(2)
    lev = np.zeros(gm.nb, np.int32)
    err = rel_l1_vol(interior(gpu_state(gm), 2, 16, 3), om.interior(), lev, 3, w["tree_size"], 16)
    say("256^3 rel L1", err, "t", t, om.t)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-14 if prec == 1 else 1e-6) * om.t


@pytest.mark.parametrize("prec", [0, 1])
def test_rayleigh_taylor_256cubed_full_size(f4, prec):
    """The benchmark's Rayleigh-Taylor leg (256^3 cells in 16^3 blocks, van
    Leer, gravity, walls along z), batched in the profiled configuration:
    two steps against two oracle steps, every cell compared; then the mass
    (periodic sides, closed walls) over 20 more steps."""
    w = synth.rayleigh_taylor(block=16, n=256)
    say("case RT 256^3 prec", prec)
    gm, om = build_pair(w, prec)
    t0 = gm.totals()
    b = f4.Batch([gm])
    b.set_config(kslabs=1, wg_per_cu=0, xcd_order=1, wg_stage2=4)
    b.step(2)
    t, _ = gm.time()
    om.step(2)
    lev = np.zeros(gm.nb, np.int32)
    err = rel_l1_vol(interior(gpu_state(gm), 2, 16, 3), om.interior(), lev, 3, w["tree_size"], 16)
    say("RT 256^3 rel L1", err, "t", t, om.t)
    assert err <= TOL[prec]
    assert abs(t - om.t) <= (1e-14 if prec == 1 else 1e-6) * om.t
    b.step(20)
    drift = abs(gm.totals()[0] - t0[0]) / t0[0]
    say("RT mass drift after 22 steps", drift)
    assert drift <= (1e-13 if prec == 1 else 1e-6)
    b.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_rayleigh_taylor_weno5_256cubed_full_size(f4, prec):
    """The benchmark's WENO5 leg (the same 256^3 Rayleigh-Taylor workload with
    three ghost layers, plain form): one step against one oracle step,
    every cell compared."""
    w = dict(synth.rayleigh_taylor(block=16, n=256))
    w.update(g=3, limiter="weno5")
    say("case RT WENO5 256^3 prec", prec)
    gm, om = build_pair(w, prec)
    gm.step(1)
    t, _ = gm.time()
    om.step(1)
    lev = np.zeros(gm.nb, np.int32)
    err = rel_l1_vol(interior(gpu_state(gm), 3, 16, 3), om.interior(), lev, 3, w["tree_size"], 16)
    say("RT WENO5 256^3 rel L1", err, "t", t, om.t)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [0, 1])
def test_two_level_blast_full_base(f4, prec):
    """Static two-level blast at full size (128^3 base, 6952 blocks of 8^3):
    10 steps against the oracle, then conservation over 100 steps."""
    w = synth.two_level_blast(base_trees=16, block=8)
    say("case two-level blast prec", prec)
    gm, om = build_pair(w, prec)
    assert gm.nb == 6952
    t0 = gm.totals()
    gm.step(10)
    om.step(10)
    lev = gm.export()[0]
    err = rel_l1_vol(interior(gpu_state(gm), 2, 8, 3), om.interior(), lev, 3, w["tree_size"], 8)
    say("two-level rel L1 after 10 steps", err)
    assert err <= TOL[prec]
    gm.step(90)
    t, _ = gm.time()
    tot = gm.totals()
    drift = np.abs(tot - t0) / np.maximum(np.abs(t0), 1e-300)
    say("after 100 steps t", t, "mass/energy drift", drift[0], drift[-1])
    assert drift[0] <= (1e-12 if prec == 1 else 2e-6) and drift[-1] <= (1e-12 if prec == 1 else 2e-6)


def test_batch_of_64_problems(f4):
    """The 64-problem batch (mixed 8^3/16^3/32^3 blocks, 38540 blocks, 4.4e8
    cells) in one persistent launch per stage: all problems conserve mass and
    energy over 20 steps; the 16 smallest agree with the oracle after 5."""
    ws = [synth.batch_problem(p) for p in range(64)]
    sizes = [int(np.prod(w["trees"])) * w["N"] ** 3 for w in ws]
    order = np.argsort(sizes)
    small = set(int(p) for p in order[:16])
    from paper_2605_07612_amd import layout
    from tests.gpu_helpers import gpu_mesh
    gms, oms = [], {}
    for p, w in enumerate(ws):
        if p in small:
            gm, oms[p] = build_pair(w, 0)
        else:  # initial data evaluated on the device
            gm = gpu_mesh(w, 0)
            layout.set_from_field_device(gm, w["field"])
        gms.append(gm)
    say("batch: blocks", sum(g.nb for g in gms))
    t0 = [g.totals() for g in gms]
    b = f4.Batch(gms)
    b.set_config(kslabs=1, wg_per_cu=0, xcd_order=0, wg_stage2=4)  # as the benchmark's autotuner chose
    b.step(5)
    for p in sorted(small):
        w, gm, om = ws[p], gms[p], oms[p]
        om.step(5)
        lev = gm.export()[0]
        err = rel_l1_vol(interior(gpu_state(gm), 2, w["N"], 3), om.interior(), lev, 3, w["tree_size"], w["N"])
        assert err <= TOL[0], (p, err)
    b.step(15)
    worst = 0.0
    for gm, tt in zip(gms, t0):
        tot = gm.totals()
        worst = max(worst, float(np.max(np.abs(tot[[0, -1]] - tt[[0, -1]]) / np.abs(tt[[0, -1]]))))
        gm.time()  # raises on an unphysical state
    say("batch worst relative drift of mass/energy after 20 steps", worst)
    assert worst <= 2e-6


def test_noise_shear_long_run_batched_equals_plain(f4):
    """500 steps of the benchmark workload (256^3 cells, FP32): the batched
    form in the benchmark's configuration and the plain form stay bit for bit
    equal (state and time) over the whole run, and mass and energy are
    conserved to FP32 rounding."""
    w = synth.uniform_noise_shear(block=16, n=256, seed=0)
    gp, _ = build_pair(w, 0)
    gb, _ = build_pair(w, 0)
    t0 = gp.totals()
    b = f4.Batch([gb])
    b.set_config(kslabs=1, wg_per_cu=0, xcd_order=1, wg_stage2=4)
    for chunk in range(5):
        gp.step(100)
        b.step(100)
        say("steps", 100 * (chunk + 1), "t", gp.time()[0], gb.time()[0])
        assert gp.time() == gb.time()
    # interiors: the plain form stores ghosts, the batched form gathers them
    assert np.array_equal(interior(gpu_state(gp), 2, 16, 3), interior(gpu_state(gb), 2, 16, 3))
    tot = gb.totals()
    drift = np.abs(tot - t0) / np.maximum(np.abs(t0), 1e-300)
    say("mass/energy drift after 500 steps", drift[0], drift[-1])
    assert drift[0] <= 1e-5 and drift[-1] <= 1e-5
