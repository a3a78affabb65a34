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
PROFILE_CONFIG = "1,0,4,1"  # the configuration the committed counters and trace were taken in


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


def timed_steps(run, steps, sync):
    import torch
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sync()
    t0 = time.perf_counter()
    start.record()
    run(steps)
    end.record()
    sync()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / 1e3, wall


def traffic_from_counters(path, stage_launch_bytes):
    """HBM bytes per stage launch from a rocprofv3 --pmc counter summary
    (profiles/*.json written from two counter passes, FETCH_SIZE and
    WRITE_SIZE in KiB per dispatch), each scaled by the factor that makes the
    same counter read the known size of a plain 1 GiB device copy."""
    try:
        d = json.load(open(path))
        import hashlib
        csrc = os.path.join(ROOT, "paper_2605_07612_amd", "csrc")
        src = b"".join(open(os.path.join(csrc, f), "rb").read()
                       for f in ("stage.hip", "device_common.h", "foap4_internal.h", "stage_common.h"))
        if hashlib.sha256(src).hexdigest() != d["source_sha256"]:
            return None  # the kernel changed since the counters were taken
        fetch = d["stage_fetch_kib"] * d["fetch_scale"]
        write = d["stage_write_kib"] * d["write_scale"]
        return {"bytes_per_launch": int((fetch + write) * 1024), "fetch_kib": round(fetch, 1),
                "write_kib": round(write, 1), "algorithmic_bytes_per_launch": int(stage_launch_bytes),
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
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for hardware-counter passes: a 1 GiB device copy (counter calibration) "
                         "then 3 batched FP32 steps in the given configuration")
    ap.add_argument("--profile-workload", default="noise_shear", choices=["noise_shear", "rayleigh_taylor", "rayleigh_taylor_weno5"],
                    help="workload of --profile-run")
    ap.add_argument("--config", default=None,
                    help="kslabs,wg_stage1,wg_stage2,xcd_order instead of autotuning, for every FP32 "
                         f"single-mesh leg (--profile-run default: {PROFILE_CONFIG})")
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
        ks, wg1, wg2, xcd = parse_config(args.config or PROFILE_CONFIG)
        batch.set_config(ks, wg1, xcd, 1, wg_stage2=wg2)
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
                     "traffic": (traffic_from_counters(args.counters, stage_bytes)
                                 if (args.block, args.n) == (16, 256) else None),
                     "kernel": f"stage_kernel<float,3,N={args.block}>", "bytes_per_launch": int(stage_bytes),
                     "avg_launch_ms": round(phases["stage"], 5)},
        "step_hbm": {"bytes_per_update": step_bytes_per_update(S32, True, args.block), "achieved_gbs": round(step_gbs, 1),
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4)},
        "phases_ms": {k: round(v, 5) for k, v in phases.items()},
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
                                                    stage_bytes) if (args.block, args.n) == (16, 256) else None),
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

    # ---------------- CPU baseline: the FP64 oracle on a bounded sample
    if not args.skip_cpu:
        from oracle import OracleMesh
        om = OracleMesh(3, w["trees"], w["N"], w["g"], w["tree_size"], gamma=w["gamma"], cfl=w["cfl"])
        om.set_interior_from_grid(grid)
        t0 = time.perf_counter()
        om.step(args.cpu_steps)
        el = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        result["cpu_baseline"] = {"value": round(cells * 2 * args.cpu_steps / el / 1e9, 5),
                                  "unit": "Gcell-updates/s", "cores": threads, "kind": "oracle",
                                  "sample": f"{args.cpu_steps} Heun steps of the same {args.n}^3 workload "
                                            f"({el:.1f} s, FP64, OpenMP over blocks)"}
        log(f"CPU oracle: {result['cpu_baseline']['value']} Gcell-updates/s on {threads} threads")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
