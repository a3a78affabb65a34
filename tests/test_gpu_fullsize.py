"""GPU parity at the workloads' full sizes and stated step counts, in the
launch configurations bench.py times: the batched FP32 form in the
configuration the autotuner's committed cache gives for the workload (the
one bench.py and the committed profiles use) and the plain FP64 form.

* 256^3 noise/shear, 4096 blocks of 16^3: 50 steps, FP32 batched and FP64
  plain, every cell against one 50-step oracle run.
* Two-level blast, 128^3 base in 8^3 blocks (6952 blocks): 100 steps, FP32
  batched and FP64 plain, every cell against one 100-step oracle run.
* Batch of 64 problems (38540 blocks of 8^3 / 16^3 / 32^3, 4.4e8 cells):
  every problem after 2 batched steps against its oracle, the 8 smallest
  also after 20.
* The benchmark's Rayleigh-Taylor legs (van Leer + gravity + walls, and
  WENO5) at 256^3.

Every comparison bounds the volume-weighted relative L1 error (FP64 1e-12,
FP32 2e-5) and the largest per-element error (FP64 1e-10, FP32 1e-5 of the
largest magnitude)."""
import os
import sys
import time

import numpy as np
import pytest

import synth
from tests.gpu_helpers import build_pair, check_state, gpu_mesh, gpu_state, interior, oracle_mesh

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNE_CACHE = os.path.join(ROOT, "paper_2605_07612_amd", "autotune_mi355x.json")


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


def bench_batch(f4, meshes):
    """A batch in the configuration bench.py uses: the autotuner's choice
    from the committed cache (tuned on the spot if the cache has no entry)."""
    b = f4.Batch(meshes)
    cfg = b.autotune(TUNE_CACHE)
    say("batch config", cfg)
    return b


def check_full(gm, om, w, prec, label):
    lev = gm.export()[0]
    a = interior(gpu_state(gm), w["g"], w["N"], 3)
    e1, e2 = check_state(a, om.interior(), lev, 3, w["tree_size"], w["N"], prec)
    t, _ = gm.time()
    say(label, "rel L1", e1, "per element", e2, "t", t, om.t)
    assert abs(t - om.t) <= (1e-13 if prec == 1 else 1e-6) * om.t
    return e1, e2


# ------------------------------------------------------------ 256^3, 50 steps
@pytest.fixture(scope="module")
def noise_shear_50():
    """The benchmark workload after 50 oracle steps (one FP64 run serves both
    GPU precisions)."""
    w = synth.uniform_noise_shear(block=16, n=256, seed=0)
    grid = w["grid_field"]()
    om = oracle_mesh(w)
    om.set_interior_from_grid(grid)
    t0 = time.perf_counter()
    om.step(50)
    say("oracle 256^3 x 50 steps:", round(time.perf_counter() - t0, 1), "s")
    return w, grid, om


@pytest.mark.parametrize("prec", [0, 1], ids=["f32_batched", "f64_plain"])
def test_noise_shear_256cubed_50_steps(f4, noise_shear_50, prec):
    from paper_2605_07612_amd import layout
    w, grid, om = noise_shear_50
    say("case 256^3 x 50 prec", prec)
    gm = gpu_mesh(w, prec)
    layout.set_from_grid(gm, grid)
    if prec == 0:
        b = bench_batch(f4, [gm])
        b.step(50)
    else:
        gm.step(50)
    check_full(gm, om, w, prec, "256^3 after 50 steps")
    if prec == 0:
        b.close()
    gm.close()


# ------------------------------------------------- two-level blast, 100 steps
@pytest.fixture(scope="module")
def two_level_100():
    """The two-level blast after 100 oracle steps (one FP64 run serves both
    GPU precisions)."""
    w = synth.two_level_blast(base_trees=16, block=8)
    om = oracle_mesh(w)
    G = np.array([g for _, g in om.forest.leaves])
    om.regrid(w["refine_flags"](G), 0, 1)
    om.set_interior_from_field(w["field"])
    t0 = time.perf_counter()
    om.step(100)
    say("oracle two-level blast x 100 steps:", round(time.perf_counter() - t0, 1), "s")
    return w, om


@pytest.mark.parametrize("prec", [0, 1], ids=["f32_batched", "f64_plain"])
def test_two_level_blast_100_steps(f4, two_level_100, prec):
    """Static two-level blast at full size: 100 steps (restriction,
    prolongation and flux fixing at every stage) against the oracle, every
    cell; mass and energy conserved to rounding."""
    from paper_2605_07612_amd import layout
    w, om = two_level_100
    say("case two-level blast x 100 prec", prec)
    gm = gpu_mesh(w, prec, max_level=1, max_blocks=16 ** 3 * 8)
    lev, G = layout.global_coords(gm)
    gm.regrid(w["refine_flags"](G))
    layout.set_from_field(gm, w["field"])
    assert gm.nb == 6952 and np.array_equal(gm.export()[0], np.asarray(om.level))
    t0 = gm.totals()
    if prec == 0:
        b = bench_batch(f4, [gm])
        b.step(100)
    else:
        gm.step(100)
    check_full(gm, om, w, prec, "two-level blast after 100 steps")
    drift = np.abs(gm.totals() - t0) / np.maximum(np.abs(t0), 1e-300)
    say("mass/energy drift", drift[0], drift[-1])
    assert drift[0] <= (1e-12 if prec == 1 else 2e-6) and drift[-1] <= (1e-12 if prec == 1 else 2e-6)
    if prec == 0:
        b.close()
    gm.close()


# ------------------------------------------------------- the 64-problem batch
def field_on_host(w, om):
    """The problem's initial data at the oracle's cell centres, evaluated on
    the host with torch (multi-threaded) in FP64."""
    import torch
    xc = om.forest.cell_centres(om.N, om.tree_size, om.origin)
    vals = w["field"](*[torch.from_numpy(np.ascontiguousarray(xc[:, d])) for d in range(3)], xp=torch)
    return vals.numpy()


def test_batch_of_64_problems(f4):
    """All 64 problems in one batch (one persistent launch per stage over
    38540 blocks of mixed sizes): every problem after 2 steps against its own
    oracle run, then the 8 smallest after 20 steps; mass and energy of every
    problem conserved over the 20 steps."""
    from oracle import OracleMesh  # noqa: F401
    from paper_2605_07612_amd import layout
    ws = [synth.batch_problem(p) for p in range(64)]
    sizes = [int(np.prod(w["trees"])) * w["N"] ** 3 for w in ws]
    smallest = [int(p) for p in np.argsort(sizes)[:8]]
    gms = []
    for w in ws:
        gm = gpu_mesh(w, 0)
        layout.set_from_field_device(gm, w["field"])
        gms.append(gm)
    say("batch: blocks", sum(g.nb for g in gms), "cells", sum(sizes))
    t0 = [g.totals() for g in gms]
    b = bench_batch(f4, gms)
    b.step(2)
    keep = {}
    worst = (0.0, 0.0)
    for p, (w, gm) in enumerate(zip(ws, gms)):
        om = oracle_mesh(w)
        om.interior()[...] = np.moveaxis(field_on_host(w, om), 0, 1)
        om.step(2)
        e1, e2 = check_full(gm, om, w, 0, f"problem {p} (N={w['N']}, {gm.nb} blocks) after 2 steps")
        worst = (max(worst[0], e1), max(worst[1], e2))
        if p in smallest:
            keep[p] = om
        else:
            del om
    say("64 problems after 2 steps: worst rel L1", worst[0], "worst per element", worst[1])
    b.step(18)
    for p in smallest:
        keep[p].step(18)
        check_full(gms[p], keep[p], ws[p], 0, f"problem {p} after 20 steps")
    drift = 0.0
    for gm, tt in zip(gms, t0):
        tot = gm.totals()
        drift = max(drift, float(np.max(np.abs(tot[[0, -1]] - tt[[0, -1]]) / np.abs(tt[[0, -1]]))))
    say("worst relative drift of mass/energy after 20 steps", drift)
    assert drift <= 2e-6
    b.close()
    for gm in gms:
        gm.close()


# ------------------------------------------------ Rayleigh-Taylor legs, 256^3
@pytest.mark.parametrize("prec", [0, 1])
def test_rayleigh_taylor_256cubed_full_size(f4, prec):
    """The benchmark's Rayleigh-Taylor leg (256^3 cells in 16^3 blocks, van
    Leer, gravity, walls along z), batched in the benchmark's configuration:
    two steps against two oracle steps, every cell compared; then the mass
    (periodic sides, closed walls) over 20 more steps."""
    w = synth.rayleigh_taylor(block=16, n=256)
    say("case RT 256^3 prec", prec)
    gm, om = build_pair(w, prec)
    t0 = gm.totals()
    b = bench_batch(f4, [gm])
    b.step(2)
    om.step(2)
    check_full(gm, om, w, prec, "RT 256^3 after 2 steps")
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
    om.step(1)
    check_full(gm, om, w, prec, "RT WENO5 256^3 after 1 step")


def test_noise_shear_long_run_batched_equals_plain(f4):
    """500 steps of the benchmark workload (256^3 cells, FP32): the batched
    form in the benchmark's configuration and the plain form stay bit for bit
    equal (state and time) over the whole run, and mass and energy are
    conserved to FP32 rounding."""
    w = synth.uniform_noise_shear(block=16, n=256, seed=0)
    gp, _ = build_pair(w, 0)
    gb, _ = build_pair(w, 0)
    t0 = gp.totals()
    b = bench_batch(f4, [gb])
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
