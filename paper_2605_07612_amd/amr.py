"""Adaptive time loop over the C ABI: the paper's cycle of time steps with a
mesh adaptation every few steps (Sec. 2.2, Sec. 3.1), with the refinement
flags of the mesh's indicator (the paper's criterion, or the learned one with
that criterion as fallback).  Host-side orchestration only: every step,
flag, regrid and remap runs in the library's kernels."""
from __future__ import annotations

import time

import numpy as np

from . import IND_LOHNER, IND_MLP, layout


def initial_refine(mesh, field, flags_fn, levels, on_device=False):
    """Write the initial data, flag blocks with flags_fn(level, G), refine,
    rewrite the initial data on the new mesh; at most `levels` times.  The
    field is evaluated with numpy on the host, or with torch on the device
    (on_device=True, field(x, y, z, xp=torch))."""
    put = layout.set_from_field_device if on_device else layout.set_from_field
    put(mesh, field)
    for _ in range(levels):
        lev, G = layout.global_coords(mesh)
        if not mesh.regrid(flags_fn(lev, G)):
            break
        put(mesh, field)


def _sync():
    import torch
    torch.cuda.synchronize()


def advance(mesh, steps, regrid_every, indicator=IND_LOHNER, before_regrid=None, compare=False):
    """Advance `steps` steps, regridding after every `regrid_every` steps
    with the flags of `indicator`.  before_regrid(mesh, flags), if given, is
    called with the state and flags of each regrid before the mesh changes.
    compare=True also evaluates the other indicator on the same state (the
    learned indicator needs a network attached to the mesh) and records both
    flag sets.  Returns one record per regrid."""
    recs = []
    done = 0
    while done < steps:
        k = min(regrid_every, steps - done)
        _sync()
        t0 = time.perf_counter()
        t, dt = mesh.step(k, sync=True)
        t1 = time.perf_counter()
        done += k
        rec = dict(step=done, t=t, dt=dt, blocks=mesh.nb, step_s=t1 - t0)
        if done >= steps:
            rec["levels"] = np.bincount(mesh.export()[0], minlength=mesh.desc.max_level + 1).tolist()
            recs.append(rec)
            break
        t2 = time.perf_counter()
        flags = mesh.refine_flags(indicator)
        t3 = time.perf_counter()
        rec["flag_s"] = t3 - t2
        if indicator == IND_MLP:
            rec["fallbacks"] = mesh.fallbacks()
        if compare:
            other = IND_LOHNER if indicator == IND_MLP else IND_MLP
            rec["flags"] = flags.copy()
            rec["other_flags"] = mesh.refine_flags(other)
        if before_regrid is not None:
            before_regrid(mesh, flags)
        t4 = time.perf_counter()
        changed = mesh.regrid(flags)
        _sync()
        rec["regrid_s"] = time.perf_counter() - t4
        rec["changed"] = changed
        rec["levels"] = np.bincount(mesh.export()[0], minlength=mesh.desc.max_level + 1).tolist()
        recs.append(rec)
    return recs
