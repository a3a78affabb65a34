"""Benchmark of the foap4 hot path on one MI355X.

Workload: 3D Euler on a static uniform periodic mesh of 256^3 cells in 16^3
blocks of 16^3 cells (4096 blocks, 2 ghost layers), smoothed seeded noise
density, sinusoidal shear, p = 2.5 (synthetic; the paper's tests use analytic
initial conditions).  A step is one Heun (SSP-RK2) step: per stage ghost fill
R1 (+R2), fused stage kernel, flux fix, plus the FP64 dt reduction.

Reported: cell updates per second (each Heun step updates every cell twice,
as in the paper's GCUPS) of the FP32 batched form (persistent launches,
HIP-graph replay, autotuned work decomposition), the FP64 plain form beside
it, the roofline of the dominant kernel (the stage kernel) from HIP-event
timings taken on the batch's stream, and the FP64 CPU oracle on a bounded
sample on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "cell-updates/s per GPU + % HBM roofline, 16^3 blocks, FP32 batched vs FP64 plain"
HBM_PEAK_GBS = 8000.0
# the autotuner's choices for the benchmark's batches on MI355X, cached by
# foap4_batch_autotune (keyed by architecture, precision, scheme and block
# mix); the timed runs, the committed profiles and the full-size parity tests
# all take their launch configuration from here
TUNE_CACHE = os.path.join(ROOT, "paper_2605_07612_amd", "autotune_mi355x.json")


def halo_share(N, g=2, ndim=3):
    """Face-ghost (halo) cells per interior cell of an N^ndim block: 2 ndim g / N."""
    return 2.0 * ndim * g / N


def stage_bytes_per_cell(S, N=16):
    """Algorithmic HBM bytes per cell of one stage-kernel launch, averaged
    over the two Heun stages, with h = halo_share(N) (0.75 for 16^3 blocks,
    g = 2): stage 1 reads the interior and halo of u^n ((1 + h) S) and writes
    u1 (1 S); stage 2 reads u1 with its halo ((1 + h) S) and u^n (1 S) and
    writes u^{n+1} (1 S).  (2.5 + h) S: 3.25 S at N = 16."""
    return (2.5 + halo_share(N)) * S


def step_bytes_per_update(S, gather, N=16):
    """Whole step per cell update.  Gathered halos on a mesh without
    refinement boundaries (the batched form): no ghost fill, (2.5 + h) S.
    Stored ghosts (the paper's design, the plain form): each stage's ghost
    fill also reads and writes h S, (2.5 + 3 h) S (4.75 S at N = 16)."""
    h = halo_share(N)
    return (2.5 + h if gather else 2.5 + 3.0 * h) * S


def parse_config(text):
    """'kslabs,wg_stage1,wg_stage2,xcd_order' (or 'kslabs,wg,xcd_order': both stages wg)."""
    v = [int(x) for x in text.split(",")]
    if len(v) == 3:
        v = [v[0], v[1], v[1], v[2]]
    if len(v) != 4:
        raise SystemExit("--config takes kslabs,wg_stage1,wg_stage2,xcd_order")
    return tuple(v)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Before each timed region the leg's own steps run, untimed, for up to
# SPINUP_S seconds (at most SPINUP_MAX_STEPS steps), so that the GPU's
# clocks have left their idle state: a timed region of a few milliseconds
# right after host-side set-up otherwise reads up to ~10 % low.
SPINUP_S = 0.3
SPINUP_MAX_STEPS = 200


def timed_steps(run, steps, sync):
    import torch
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sync()
    t0, done = time.perf_counter(), 0
    while time.perf_counter() - t0 < SPINUP_S and done < SPINUP_MAX_STEPS:
        run(10)
        sync()
        done += 10
    sync()
    t0 = time.perf_counter()
    start.record()
    run(steps)
    end.record()
    sync()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / 1e3, wall


def traffic_from_counters(path, kernel, launch_bytes):
    """HBM bytes per launch of the kernels matching `kernel` (a regular
    expression; the mean over them, e.g. the two Heun stages) from a counter
    summary under profiles/ (paper_2605_07612_amd.profiling: two rocprofv3
    --pmc passes, FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled
    by the factor that makes the same counter read the known size of a plain
    1 GiB device copy).  None once the kernel's sources differ from the ones
    the counters were taken on."""
    import re
    from paper_2605_07612_amd.profiling import sources_sha256
    try:
        d = json.load(open(path))
        if sources_sha256([os.path.join(ROOT, f) for f in d["source_files"]]) != d["source_sha256"]:
            return None  # the kernel changed since the counters were taken
        recs = [r for r in d["dispatch_means"] if re.search(kernel, r["kernel"])]
        if not recs:
            return None
        fetch = sum(r["FETCH_SIZE_scaled"] for r in recs) / len(recs)
        write = sum(r["WRITE_SIZE_scaled"] for r in recs) / len(recs)
        return {"bytes_per_launch": int((fetch + write) * 1024), "fetch_kib": round(fetch, 1),
                "write_kib": round(write, 1), "algorithmic_bytes_per_launch": int(launch_bytes),
                "source": os.path.relpath(path, ROOT)}
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis")
    ap.add_argument("--block", type=int, default=16)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-batch64", action="store_true")
    ap.add_argument("--skip-rt", action="store_true")
    ap.add_argument("--skip-adv", action="store_true")
    ap.add_argument("--skip-two-level", action="store_true")
    ap.add_argument("--skip-sweep", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="autotuner cache (JSON); entries missing from it are tuned and added")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for hardware-counter passes: a 1 GiB device copy (counter calibration) "
                         "then 3 batched FP32 steps in the given configuration")
    ap.add_argument("--profile-workload", default="noise_shear",
                    choices=["noise_shear", "noise_shear_fp64_plain", "rayleigh_taylor", "rayleigh_taylor_weno5",
                             "advection", "two_level"],
                    help="workload of --profile-run")
    ap.add_argument("--config", default=None,
                    help="kslabs,wg_stage1,wg_stage2,xcd_order instead of the autotuner's cached choice, for "
                         "every FP32 single-mesh leg (and --profile-run)")
    ap.add_argument("--counters", default=os.path.join(ROOT, "profiles", "stage_traffic_noise_shear_256cubed_b16.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this benchmark runs on one GPU; --gpus must be 1 (the multi-GPU sharding is a design "
              "note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2605_07612_amd as f4
    from paper_2605_07612_amd import layout

    torch.cuda.set_device(0)
    w = synth.uniform_noise_shear(block=args.block, n=args.n, seed=0)
    cells = args.n ** 3
    log(f"workload {w['name']}: {cells} cells, {np.prod(w['trees'])} blocks")
    grid = w["grid_field"]()

    def make(prec):
        m = f4.Mesh(3, w["trees"], w["N"], w["g"], w["tree_size"], prec=prec, gamma=w["gamma"], cfl=w["cfl"])
        layout.set_from_grid(m, grid)
        return m

    wr = synth.rayleigh_taylor(block=args.block, n=args.n)

    def make_rt(prec):
        m = f4.Mesh(3, wr["trees"], wr["N"], wr["g"], wr["tree_size"], prec=prec, gamma=wr["gamma"],
                    cfl=wr["cfl"], limiter=wr["limiter"], flux=wr["flux"], gravity=wr["gravity"],
                    periodic=wr["periodic"], bc_type=wr["bc_type"], bc_value=wr["bc_value"])
        layout.set_from_grid(m, wr["grid_field"]())
        return m

    def make_rt_weno(prec):
        m = f4.Mesh(3, wr["trees"], wr["N"], 3, wr["tree_size"], prec=prec, gamma=wr["gamma"], cfl=wr["cfl"],
                    limiter="weno5", flux=wr["flux"], gravity=wr["gravity"], periodic=wr["periodic"],
                    bc_type=wr["bc_type"], bc_value=wr["bc_value"])
        layout.set_from_grid(m, wr["grid_field"]())
        return m

    if args.profile_run:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        bb = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        bb.copy_(a)  # calibration: reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, bb
        if args.profile_workload == "two_level":
            wt = synth.two_level_blast(base_trees=16, block=8)
            for prec in (f4.F32, f4.F64):  # three steps batched FP32 (cached configuration), plain FP64
                m = f4.Mesh(3, wt["trees"], wt["N"], wt["g"], wt["tree_size"], max_level=1,
                            max_blocks=int(np.prod(wt["trees"])) * 8, prec=prec, gamma=wt["gamma"], cfl=wt["cfl"])
                _, G = layout.global_coords(m)
                m.regrid(wt["refine_flags"](G))
                layout.set_from_field_device(m, wt["field"])
                if prec == f4.F32:
                    bt = f4.Batch([m])
                    log("two-level profile run, batch configuration", bt.autotune(args.tune_cache))
                    bt.step(3)
                    torch.cuda.synchronize()
                    bt.close()
                else:
                    m.step(3)
                    torch.cuda.synchronize()
                m.close()
                del m
                torch.cuda.empty_cache()
            log("profile run done")
            return
        if args.profile_workload == "advection":
            wa = synth.advection(3, args.block, args.n, init="sphere", limiter="vanleer")
            for prec in (f4.F32, f4.F64):  # three Heun steps of each advection kernel, batched FP32, plain FP64
                m = f4.Mesh(3, wa["trees"], wa["N"], wa["g"], wa["tree_size"], prec=prec, cfl=wa["cfl"],
                            limiter="vanleer", physics="advection", velocity=wa["velocity"])
                layout.set_from_field_device(m, wa["field"])
                if prec == f4.F32:
                    ba = f4.Batch([m])
                    ba.step(3)
                    torch.cuda.synchronize()
                    ba.close()
                else:
                    m.step(3)
                    torch.cuda.synchronize()
                m.close()
                del m
                torch.cuda.empty_cache()
            log("profile run done")
            return
        if args.profile_workload == "noise_shear_fp64_plain":  # three plain FP64 steps (stored ghosts)
            m = make(f4.F64)
            m.step(3)
            torch.cuda.synchronize()
            log("profile run done")
            return
        if args.profile_workload == "rayleigh_taylor_weno5":
            for prec in (f4.F32, f4.F64):  # three Heun steps of each WENO5 kernel
                m = make_rt_weno(prec)
                m.step(3)
                torch.cuda.synchronize()
                m.close()
                del m
                torch.cuda.empty_cache()
            log("profile run done")
            return
        m32 = make(f4.F32) if args.profile_workload == "noise_shear" else make_rt(f4.F32)
        batch = f4.Batch([m32])
        if args.config:  # else the configuration the timed run uses
            ks, wg1, wg2, xcd = parse_config(args.config)
            batch.set_config(ks, wg1, xcd, 1, wg_stage2=wg2)
        else:
            ks, wg1, wg2, xcd = batch.autotune(args.tune_cache)
        log(f"profile run in configuration kslabs={ks} wg_per_cu stage 1={wg1} stage 2={wg2} xcd_order={xcd}")
        batch.step(3)
        torch.cuda.synchronize()
        log("profile run done")
        return

    S32, S64 = 5 * 4, 5 * 8

    # ---------------- FP32 batched: persistent + graph + autotuned
    m32 = make(f4.F32)
    batch = f4.Batch([m32])
    if args.config:
        ks, wg1, wg2, xcd = parse_config(args.config)
        batch.set_config(ks, wg1, xcd, 1, wg_stage2=wg2)
    else:
        ks, wg1, wg2, xcd = batch.autotune(args.tune_cache)
    log(f"autotune: kslabs={ks} wg_per_cu stage 1={wg1} stage 2={wg2} xcd_order={xcd}")
    batch.step(args.warmup)
    secs, wall = timed_steps(batch.step, args.steps, torch.cuda.synchronize)
    gcups32 = cells * 2 * args.steps / secs / 1e9
    log(f"FP32 batched: {secs / args.steps * 1e3:.3f} ms/step, {gcups32:.2f} Gcell-updates/s (wall {wall:.3f}s)")
    # four more timed regions of the same K steps, reported beside the value
    # (the value is the first region): the spread of repeated measurements
    reps = [secs] + [timed_steps(batch.step, args.steps, torch.cuda.synchronize)[0] for _ in range(4)]
    rep_ms = sorted(r / args.steps * 1e3 for r in reps)
    log("repeats (ms/step):", " ".join(f"{x:.4f}" for x in rep_ms))
    phases = batch.phase_times(5)
    log("phases (ms):", json.dumps({k: round(v, 4) for k, v in phases.items()}))
    stage_bytes = cells * stage_bytes_per_cell(S32, args.block)
    achieved = stage_bytes / (phases["stage"] * 1e-3) / 1e9
    step_gbs = gcups32 * step_bytes_per_update(S32, True, args.block)

    result = {
        "metric": METRIC,
        "value": round(gcups32, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "spinup": {"seconds": SPINUP_S, "max_steps": SPINUP_MAX_STEPS},
        "ms_per_step": round(secs / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "cells": cells, "blocks": int(np.prod(w["trees"])),
                   "block": args.block, "ghost": 2, "form": "batched: persistent stage launch, hipGraph, autotuned",
                   "kslabs": ks, "wg_per_cu_stage1": wg1, "wg_per_cu_stage2": wg2, "xcd_order": xcd, "gather_halos": 1, "reductions": "f64"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     # the committed counters cover the 256^3 workload in 16^3 blocks only
                     "traffic": (traffic_from_counters(args.counters, r"stage_kernel<float, 3, 2, [12], 0>",
                                                       stage_bytes) if (args.block, args.n) == (16, 256) else None),
                     "kernel": f"stage_kernel<float,3,N={args.block}>", "bytes_per_launch": int(stage_bytes),
                     "avg_launch_ms": round(phases["stage"], 5)},
        "step_hbm": {"bytes_per_update": step_bytes_per_update(S32, True, args.block), "achieved_gbs": round(step_gbs, 1),
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "phases_ms": {k: round(v, 5) for k, v in phases.items()},
        "repeats": {"timed_regions": len(rep_ms), "ms_per_step_min": round(rep_ms[0], 4),
                    "ms_per_step_median": round(rep_ms[len(rep_ms) // 2], 4),
                    "ms_per_step_max": round(rep_ms[-1], 4),
                    "value_at_median": round(cells * 2 / (rep_ms[len(rep_ms) // 2] * 1e-3) / 1e9, 4)},
    }
    del batch, m32
    torch.cuda.empty_cache()

    if not args.skip_fp64:
        # ---------------- FP64 plain: one workgroup per block, stored ghosts, one launch per kernel
        m64 = make(f4.F64)
        m64.step(args.warmup)
        secs64, _ = timed_steps(lambda n: m64.step(n), args.steps, torch.cuda.synchronize)
        gcups64 = cells * 2 * args.steps / secs64 / 1e9
        log(f"FP64 plain: {secs64 / args.steps * 1e3:.3f} ms/step, {gcups64:.2f} Gcell-updates/s")
        result["fp64_plain"] = {"value": round(gcups64, 4), "unit": "Gcell-updates/s",
                                "ms_per_step": round(secs64 / args.steps * 1e3, 4),
                                "step_hbm_frac": round(gcups64 * step_bytes_per_update(S64, False, args.block) / HBM_PEAK_GBS, 4),
                                "batched_fp32_over_plain_fp64": round(gcups32 / gcups64, 3)}
        del m64
        torch.cuda.empty_cache()
        # ---------------- FP64 batched, for reference
        m64 = make(f4.F64)
        b64 = f4.Batch([m64])
        cfg64 = b64.autotune(args.tune_cache)
        b64.step(args.warmup)
        secs64b, _ = timed_steps(b64.step, args.steps, torch.cuda.synchronize)
        gcups64b = cells * 2 * args.steps / secs64b / 1e9
        log(f"FP64 batched: {secs64b / args.steps * 1e3:.3f} ms/step, {gcups64b:.2f} Gcell-updates/s")
        result["fp64_batched"] = {"value": round(gcups64b, 4), "unit": "Gcell-updates/s",
                                  "ms_per_step": round(secs64b / args.steps * 1e3, 4), "config": list(cfg64),
                                  "step_hbm_frac": round(gcups64b * step_bytes_per_update(S64, True, args.block) / HBM_PEAK_GBS, 4)}
        del b64, m64
        torch.cuda.empty_cache()

    # ---------------- the paper's own benchmark workload: Rayleigh-Taylor with the
    # van Leer limiter and the gravity source (Sec. 4.2), same cells and blocks
    if not args.skip_rt:
        mr = make_rt(f4.F32)
        br = f4.Batch([mr])
        if args.config:
            cfg_rt = parse_config(args.config)
            br.set_config(cfg_rt[0], cfg_rt[1], cfg_rt[3], 1, wg_stage2=cfg_rt[2])
        else:
            cfg_rt = br.autotune(args.tune_cache)
        br.step(args.warmup)
        sr, _ = timed_steps(br.step, args.steps, torch.cuda.synchronize)
        g_rt = cells * 2 * args.steps / sr / 1e9
        ph_rt = br.phase_times(5)
        log(f"Rayleigh-Taylor FP32 batched: {sr / args.steps * 1e3:.3f} ms/step, {g_rt:.2f} Gcell-updates/s, "
            f"config {cfg_rt}")
        del br, mr
        torch.cuda.empty_cache()
        mr = make_rt(f4.F64)
        mr.step(args.warmup)
        sr64, _ = timed_steps(lambda n: mr.step(n), args.steps, torch.cuda.synchronize)
        g_rt64 = cells * 2 * args.steps / sr64 / 1e9
        log(f"Rayleigh-Taylor FP64 plain: {sr64 / args.steps * 1e3:.3f} ms/step, {g_rt64:.2f} Gcell-updates/s")
        del mr
        torch.cuda.empty_cache()
        # the paper's H100 figures for this workload (other hardware: context, not the target)
        paper = {32: (2.702, 1.366), 16: (2.599, 1.302), 8: (2.081, 1.097)}.get(args.block)
        rt_stage_gbs = stage_bytes / (ph_rt["stage"] * 1e-3) / 1e9  # same bytes per cell as above
        result["rayleigh_taylor"] = {
            "workload": wr["name"], "scheme": "van Leer, Rusanov, gravity (0, 0, -1), gamma 5/3, "
                                              "periodic x, y, reflecting walls in z",
            "value": round(g_rt, 4), "unit": "Gcell-updates/s", "dtype": "f32",
            "ms_per_step": round(sr / args.steps * 1e3, 4), "config": list(cfg_rt),
            "stage_ms": round(ph_rt["stage"], 5), "stage_hbm_frac": round(rt_stage_gbs / HBM_PEAK_GBS, 4),
            "stage_traffic": (traffic_from_counters(os.path.join(ROOT, "profiles",
                                                                 "stage_traffic_rayleigh_taylor_256cubed_b16.json"),
                                                    r"stage_kernel<float, 3, 2, [12], 5>", stage_bytes)
                              if (args.block, args.n) == (16, 256) else None),
            "step_hbm_frac": round(g_rt * step_bytes_per_update(S32, True, args.block) / HBM_PEAK_GBS, 4),
            "fp64_plain": {"value": round(g_rt64, 4), "ms_per_step": round(sr64 / args.steps * 1e3, 4)},
            "paper_h100_context": (None if paper is None or args.n != 256 else
                                   {"fp32": paper[0], "fp64": paper[1],
                                    "source": "table of results on different hardware, 256^3, van Leer"}),
        }

    # ---------------- the same Rayleigh-Taylor workload with WENO5 (three ghost
    # layers), plain form, Heun steps
    if not args.skip_rt:
        weno = {}
        for prec, name in ((f4.F32, "fp32_plain"), (f4.F64, "fp64_plain")):
            m = make_rt_weno(prec)
            m.step(2)
            sw, _ = timed_steps(lambda n: m.step(n), 5, torch.cuda.synchronize)
            weno[name] = {"value": round(cells * 2 * 5 / sw / 1e9, 4), "ms_per_step": round(sw / 5 * 1e3, 3)}
            log(f"Rayleigh-Taylor WENO5 {name}: {sw / 5 * 1e3:.3f} ms/step, {weno[name]['value']:.2f} Gcell-updates/s")
            m.close()
            del m
            torch.cuda.empty_cache()
        paper_w = {32: 0.53, 16: 0.48, 8: 0.40}.get(args.block)
        result["rayleigh_taylor_weno5"] = dict(
            weno, unit="Gcell-updates/s", scheme="WENO5 (g = 3), Rusanov, gravity, walls in z, Heun",
            paper_h100_context=(None if paper_w is None or args.n != 256 else
                                {"fp64": paper_w, "source": "table of results on uniform grids, 256^3, WENO5"}))

    # ---------------- block-size sweep: the same 256^3 workload in 8^3 (32768)
    # and 32^3 (512) blocks, as the paper's table of results on different
    # hardware has them; FP32 batched (the autotuner's cached choice) and
    # FP64 plain
    if not args.skip_sweep and args.n == 256:
        sweep = {}
        for nb_ in (8, 32):
            if nb_ == args.block:
                continue
            ws_ = synth.uniform_noise_shear(block=nb_, n=args.n, seed=0)

            def make_s(prec):
                m = f4.Mesh(3, ws_["trees"], ws_["N"], ws_["g"], ws_["tree_size"], prec=prec, gamma=ws_["gamma"],
                            cfl=ws_["cfl"])
                layout.set_from_grid(m, grid)
                return m

            m = make_s(f4.F32)
            bs = f4.Batch([m])
            cfg_s = bs.autotune(args.tune_cache)
            bs.step(args.warmup)
            ss_, _ = timed_steps(bs.step, args.steps, torch.cuda.synchronize)
            g_s = cells * 2 * args.steps / ss_ / 1e9
            ph_s = bs.phase_times(5)
            del bs, m
            torch.cuda.empty_cache()
            m = make_s(f4.F64)
            m.step(args.warmup)
            ss64, _ = timed_steps(lambda k: m.step(k), args.steps, torch.cuda.synchronize)
            g_s64 = cells * 2 * args.steps / ss64 / 1e9
            del m
            torch.cuda.empty_cache()
            sb = cells * stage_bytes_per_cell(S32, nb_)
            paper_s = {32: (2.702, 1.366), 8: (2.081, 1.097)}.get(nb_)
            sweep[f"b{nb_}"] = {
                "blocks": int(np.prod(ws_["trees"])), "value": round(g_s, 4), "unit": "Gcell-updates/s",
                "dtype": "f32", "ms_per_step": round(ss_ / args.steps * 1e3, 4), "config": list(cfg_s),
                "stage_ms": round(ph_s["stage"], 5),
                "stage_hbm_frac": round(sb / (ph_s["stage"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "step_hbm_frac": round(g_s * step_bytes_per_update(S32, True, nb_) / HBM_PEAK_GBS, 4),
                "fp64_plain": {"value": round(g_s64, 4), "ms_per_step": round(ss64 / args.steps * 1e3, 4),
                               "step_hbm_frac": round(g_s64 * step_bytes_per_update(S64, False, nb_) / HBM_PEAK_GBS,
                                                      4)},
                "paper_h100_context_rt": (None if paper_s is None else
                                          {"fp32": paper_s[0], "fp64": paper_s[1],
                                           "source": "table of results on different hardware, Rayleigh-Taylor, "
                                                     "256^3, van Leer"})}
            log(f"noise/shear 256^3 in {nb_}^3 blocks: FP32 batched {g_s:.2f}, FP64 plain {g_s64:.2f} "
                f"Gcell-updates/s, config {cfg_s}")
        result["block_sweep"] = sweep

    # ---------------- the static two-level blast (128^3 base in 8^3 blocks, the
    # ball |x - 1/2| < 1/4 refined once: 6952 blocks, 3.56e6 cells): every
    # stage restricts, prolongs and fixes fluxes at the level boundaries
    if not args.skip_two_level:
        wt = synth.two_level_blast(base_trees=16, block=8)

        def make_tl(prec):
            m = f4.Mesh(3, wt["trees"], wt["N"], wt["g"], wt["tree_size"], max_level=1,
                        max_blocks=int(np.prod(wt["trees"])) * 8, prec=prec, gamma=wt["gamma"], cfl=wt["cfl"])
            _, G = layout.global_coords(m)
            m.regrid(wt["refine_flags"](G))
            layout.set_from_field_device(m, wt["field"])
            return m

        tl = {}
        m = make_tl(f4.F32)
        cells_tl = m.nb * wt["N"] ** 3
        bt = f4.Batch([m])
        cfg_tl = bt.autotune(args.tune_cache)
        bt.step(args.warmup)
        st_, _ = timed_steps(bt.step, args.steps, torch.cuda.synchronize)
        g_tl = cells_tl * 2 * args.steps / st_ / 1e9
        ph_tl = bt.phase_times(5)
        ghost_share = 2 * (ph_tl["ghost_r1"] + ph_tl["ghost_r2"]) / ph_tl["step"]
        tl.update(workload=wt["name"], blocks=int(m.nb), cells=int(cells_tl), value=round(g_tl, 4),
                  unit="Gcell-updates/s", dtype="f32", ms_per_step=round(st_ / args.steps * 1e3, 4),
                  config=list(cfg_tl), phases_ms={k: round(v, 5) for k, v in ph_tl.items()},
                  ghost_share=round(ghost_share, 4),
                  stage_share=round(2 * ph_tl["stage"] / ph_tl["step"], 4),
                  fluxfix_share=round(ph_tl["fluxfix"] / ph_tl["step"], 4))
        del bt, m
        torch.cuda.empty_cache()
        # the other three forms: FP32 plain (per-kernel launches, stored
        # ghosts), FP64 plain (the paper's form) and FP64 batched (the FP32
        # leg's launch configuration, not tuned for FP64)
        for prec, form in ((f4.F32, "fp32_plain"), (f4.F64, "fp64_plain"), (f4.F64, "fp64_batched")):
            m = make_tl(prec)
            if form.endswith("batched"):
                run = f4.Batch([m])
                run.set_config(cfg_tl[0], cfg_tl[1], cfg_tl[3], 1, wg_stage2=cfg_tl[2])
                step = run.step
            else:
                run, step = None, (lambda k, m=m: m.step(k))
            step(args.warmup)
            sx, _ = timed_steps(step, args.steps, torch.cuda.synchronize)
            tl[form] = {"value": round(cells_tl * 2 * args.steps / sx / 1e9, 4),
                        "ms_per_step": round(sx / args.steps * 1e3, 4)}
            if run is not None:
                tl[form]["config"] = list(cfg_tl)
                run.close()
            del run, step, m
            torch.cuda.empty_cache()
        log(f"two-level blast: FP32 batched {g_tl:.2f} Gcell-updates/s (ghost rounds {100 * ghost_share:.1f} % "
            f"of the step), FP32 plain {tl['fp32_plain']['value']:.2f}, FP64 plain {tl['fp64_plain']['value']:.2f}, "
            f"FP64 batched {tl['fp64_batched']['value']:.2f}")
        result["two_level_blast"] = tl

    # ---------------- scalar advection (Sec. 3.4): the paper's highest-throughput
    # workload (its table of results on uniform grids, advection rows): the
    # smoothed sphere, v = (1, 1, 1), van Leer, Heun, 16^3 blocks, at 256^3 and
    # 512^3 cells; FP32 batched (graph-replayed) and FP64 plain
    if not args.skip_adv:
        adv = {}
        for n_adv in (256, 512):
            wa = synth.advection(3, args.block, n_adv, init="sphere", limiter="vanleer")
            cells_a = n_adv ** 3

            def make_adv(prec):
                m = f4.Mesh(3, wa["trees"], wa["N"], wa["g"], wa["tree_size"], prec=prec, cfl=wa["cfl"],
                            limiter="vanleer", physics="advection", velocity=wa["velocity"])
                layout.set_from_field_device(m, wa["field"])
                return m

            ma = make_adv(f4.F32)
            ba = f4.Batch([ma])
            ba.step(args.warmup)
            sa, _ = timed_steps(ba.step, args.steps, torch.cuda.synchronize)
            ga = cells_a * 2 * args.steps / sa / 1e9
            pha = ba.phase_times(5)
            del ba, ma
            torch.cuda.empty_cache()
            ma = make_adv(f4.F64)
            ma.step(args.warmup)
            sa64, _ = timed_steps(lambda k: ma.step(k), args.steps, torch.cuda.synchronize)
            ga64 = cells_a * 2 * args.steps / sa64 / 1e9
            del ma
            torch.cuda.empty_cache()
            adv_stage_bytes = cells_a * stage_bytes_per_cell(4, args.block)
            adv_gbs = adv_stage_bytes / (pha["stage"] * 1e-3) / 1e9
            paper_a = ({256: {32: 7.59, 16: 8.64, 8: 6.95}, 512: {32: 12.27, 16: 10.89, 8: 7.79}}
                       .get(n_adv, {}).get(args.block))
            adv[f"{n_adv}^3"] = {
                "value": round(ga, 4), "unit": "Gcell-updates/s", "dtype": "f32",
                "ms_per_step": round(sa / args.steps * 1e3, 4),
                "stage_ms": round(pha["stage"], 5), "ghost_r1_ms": round(pha["ghost_r1"], 5),
                "stage_bytes_per_launch": int(adv_stage_bytes),
                "stage_hbm_frac": round(adv_gbs / HBM_PEAK_GBS, 4),
                "step_hbm_frac": round(ga * step_bytes_per_update(4, False, args.block) / HBM_PEAK_GBS, 4),
                "fp64_plain": {"value": round(ga64, 4), "ms_per_step": round(sa64 / args.steps * 1e3, 4),
                               "step_hbm_frac": round(ga64 * step_bytes_per_update(8, False, args.block)
                                                      / HBM_PEAK_GBS, 4)},
                "paper_h100_context": (None if paper_a is None else
                                       {"fp64": paper_a, "source": "table of results on uniform grids, "
                                                                   "advection, van Leer"})}
            log(f"advection {n_adv}^3: FP32 batched {ga:.2f}, FP64 plain {ga64:.2f} Gcell-updates/s, "
                f"stage {pha['stage']:.4f} ms")
        result["advection"] = dict(adv, workload="advection_sphere_b16", scheme="van Leer, Rusanov, Heun, "
                                                                              "v = (1, 1, 1), stored ghosts")

    # ---------------- the 64-problem batch (mixed 8^3/16^3/32^3 blocks), FP32
    if not args.skip_batch64:
        ws = [synth.batch_problem(p) for p in range(64)]
        ms = []
        for wp in ws:
            m = f4.Mesh(3, wp["trees"], wp["N"], wp["g"], wp["tree_size"], prec=f4.F32, gamma=wp["gamma"],
                        cfl=wp["cfl"])
            layout.set_from_field_device(m, wp["field"])
            ms.append(m)
        cells64 = sum(int(np.prod(wp["trees"])) * wp["N"] ** 3 for wp in ws)
        # algorithmic bytes per update, cell-weighted over the problems' block sizes
        bpu64 = sum(int(np.prod(wp["trees"])) * wp["N"] ** 3 * step_bytes_per_update(S32, True, wp["N"])
                    for wp in ws) / cells64
        b64 = f4.Batch(ms)
        cfg = b64.autotune(args.tune_cache)
        b64.step(args.warmup)
        s64, _ = timed_steps(b64.step, args.steps, torch.cuda.synchronize)
        g64 = cells64 * 2 * args.steps / s64 / 1e9
        ph64 = b64.phase_times(3)
        log(f"batch of 64: {s64 / args.steps * 1e3:.3f} ms/step, {g64:.2f} Gcell-updates/s, config {cfg}")
        result["batch64"] = {"value": round(g64, 4), "unit": "Gcell-updates/s", "problems": 64,
                             "blocks": int(sum(m.nb for m in ms)), "cells": int(cells64),
                             "ms_per_step": round(s64 / args.steps * 1e3, 4), "config": list(cfg),
                             "stage_ms": round(ph64["stage"], 4),
                             "bytes_per_update": round(bpu64, 2),
                             "step_hbm_frac": round(g64 * bpu64 / HBM_PEAK_GBS, 4)}
        del b64, ms
        torch.cuda.empty_cache()

    # ---------------- CPU baseline: the FP64 oracle on a bounded sample, with
    # OpenMP over blocks on every thread the runtime gives it, and on one thread
    if not args.skip_cpu:
        import ctypes
        import ctypes.util
        from oracle import OracleMesh
        gomp = ctypes.CDLL(ctypes.util.find_library("gomp") or "libgomp.so.1")
        threads = int(gomp.omp_get_max_threads())
        nproc = len(os.sched_getaffinity(0))
        om = OracleMesh(3, w["trees"], w["N"], w["g"], w["tree_size"], gamma=w["gamma"], cfl=w["cfl"])
        om.set_interior_from_grid(grid)
        t0 = time.perf_counter()
        om.step(args.cpu_steps)
        el = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": round(cells * 2 * args.cpu_steps / el / 1e9, 5),
                                  "unit": "Gcell-updates/s", "cores": threads, "kind": "oracle",
                                  "sample": f"{args.cpu_steps} Heun steps of the same {args.n}^3 workload "
                                            f"({el:.1f} s, FP64, OpenMP over blocks on {threads} threads; "
                                            f"nproc {nproc})"}
        log(f"CPU oracle: {result['cpu_baseline']['value']} Gcell-updates/s on {threads} threads")
        del om
        # one thread: the same workload (same blocks, fields and scheme) on a
        # 128^3 domain, so that the sample stays at a few seconds
        n1 = min(args.n, 128)
        w1 = synth.uniform_noise_shear(block=args.block, n=n1, seed=0)
        om = OracleMesh(3, w1["trees"], w1["N"], w1["g"], w1["tree_size"], gamma=w1["gamma"], cfl=w1["cfl"])
        om.set_interior_from_grid(w1["grid_field"]())
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        om.step(2)
        el1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(threads)
        result["cpu_baseline_single_thread"] = {"value": round(n1 ** 3 * 2 * 2 / el1 / 1e9, 5),
                                                "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
                                                "sample": f"2 Heun steps of the same workload on {n1}^3 cells in "
                                                          f"{args.block}^3 blocks ({el1:.1f} s, FP64, one thread)"}
        log(f"CPU oracle, one thread: {result['cpu_baseline_single_thread']['value']} Gcell-updates/s")
        del om
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
