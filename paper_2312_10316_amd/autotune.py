"""Autotuner for the step launch: tile shape (rows walked per wave, XCD tile order and its row-block
height, 64- or 256-column tiles), non-temporal or cached stores of the new state, a cap on the waves
resident per SIMD, one buffer updated in place, two steps per launch (tile width and height), and, for a
multi-instance context, the
batch schedule (serial launches, one flat launch, or persistent blocks with a round-robin or
longest-processing-time assignment of tiles).

Candidates are timed on the caller's own instances with graph-replayed steps; the instances' states
and step counters are saved first and restored afterwards, so tuning never advances the simulation
(results do not depend on the launch configuration, bitwise).  Winners are cached in memory and,
optionally, in a JSON file keyed by the device and the instance shapes.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Iterable, Optional

import torch

from . import lbm as L

_MEMO: dict = {}


def _key(solver) -> str:
    dev = torch.cuda.get_device_name()
    shapes = [(p.nx, p.ny, p.nz, p.lattice, p.store, p.math, p.aux, p.boundary, p.tau3 not in (0.0, 1.0))
              for p in solver.params]
    return hashlib.sha256(json.dumps(["launch-v6", dev, shapes]).encode()).hexdigest()[:20]


def _fusable_params(p) -> bool:
    return p.lattice == L.LBM_LATTICE_D2Q9 and p.boundary == L.LBM_BC_PERIODIC and p.tau3 in (0.0, 1.0)


def _fusable(solver) -> bool:
    return len(solver.params) == 1 and _fusable_params(solver.params[0])


def _fusable_batch(solver) -> bool:
    """A uniform batch (one storage and aux form, periodic D2Q9 TRT-R) can run two steps per launch."""
    ps = solver.params
    return (len(ps) > 1 and all(_fusable_params(p) and p.aux != L.LBM_AUX_FLUX for p in ps)
            and len({(p.store, p.math, p.aux) for p in ps}) == 1)


def default_candidates(solver) -> list:
    """(rows, xcd_remap, xcd_rows, tile_width, max_waves, stores, policy, blocks, fuse) tuples worth timing
    for this context.  Stores: both kinds for one instance where they are honoured (not in the local
    form's walking loop); a batch keeps the context's default.  A single periodic D2Q9 TRT-R instance
    with the local or no aux term also tries one buffer in place (one-row launches) and two steps per
    launch (fuse 2: tile width and height, row bands or hardware order, both store kinds); a uniform
    batch of such instances tries two steps per launch too (tile width and height, flat or LPT)."""
    out = []
    st0 = solver.get_launch(0)["stores"]
    p0 = solver.params[0]
    multi = len(solver.params) > 1 and len({(p.store, p.math, p.aux) for p in solver.params}) == 1
    if _fusable(solver):
        flux = p0.aux == L.LBM_AUX_FLUX  # the flux form: 128- or 256-column tiles, never in place
        for width in ((128, 256) if flux else (128, 256, 512)):
            for rows in (8, 16, 32, 64):
                for remap in (0, 1):
                    for stores in (0, 1):
                        out.append((rows, remap, 0, width, 0, stores, L.LBM_BATCH_SERIAL, 0, 2))
    if _fusable(solver) and p0.aux != L.LBM_AUX_FLUX:
        for width in (64, 256):
            for remap, h in [(0, 0), (1, 0)] + ([(3, h) for h in (2, 4, 8)] if width == 256 else []):
                for cap in (0, 4, 5):
                    out.append((1, remap, h, width, cap, 2, L.LBM_BATCH_SERIAL, 0, 1))
    elif not multi and st0 == 2:  # one buffer updated in place (3D): one-row launches only
        for width in (64, 256):
            for remap, h in [(0, 0), (1, 0)] + ([(3, h) for h in (2, 4, 8)] if width == 256 else []):
                for cap in (0, 4, 5):
                    out.append((1, remap, h, width, cap, 2, L.LBM_BATCH_SERIAL, 0, 1))
        return out
    if not multi:
        for width, rows_set in ((64, (1, 2, 4)), (256, (1, 2))):
            for rows in rows_set:
                orders = [(0, 0), (1, 0)] + ([(3, h) for h in (2, 4, 8)] if width == 256 else [])
                for remap, h in orders:
                    for cap in (0, 4, 5):
                        honoured = rows == 1 or p0.aux == L.LBM_AUX_FLUX or p0.lattice != L.LBM_LATTICE_D2Q9
                        for stores in ((0, 1) if honoured else (0,)):
                            out.append((rows, remap, h, width, cap, stores, L.LBM_BATCH_SERIAL, 0, 1))
        return out
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    if _fusable_batch(solver):  # two steps per launch, one batched launch (non-temporal stores)
        for width in (128, 256):
            for rows in (8, 16, 32):
                out.append((rows, 1, 0, width, 0, 0, L.LBM_BATCH_FLAT, 0, 2))
                out.append((rows, 1, 0, width, 0, 0, L.LBM_BATCH_LPT, 4 * ncu, 2))
    for width in (64, 256):
        for rows in (1, 2, 4):
            out.append((rows, 1, 0, width, 0, st0, L.LBM_BATCH_SERIAL, 0, 1))
            for cap in (0, 6):
                out.append((rows, 1, 0, width, cap, st0, L.LBM_BATCH_FLAT, 0, 1))
                out.append((rows, 1, 0, width, cap, st0, L.LBM_BATCH_LPT, 4 * ncu, 1))
            for mult in (2, 8):
                out.append((rows, 1, 0, width, 0, st0, L.LBM_BATCH_LPT, mult * ncu, 1))
            out.append((rows, 1, 0, width, 0, st0, L.LBM_BATCH_STRIDED, 4 * ncu, 1))
    return out


def _apply(solver, cand) -> None:
    rows, remap, h, width, cap, stores, policy, blocks, fuse = (tuple(cand) + (1,))[:9]
    solver.set_launch(rows, remap, tile_width=width, max_waves=cap, xcd_rows=h, stores=stores, fuse=fuse)
    if len(solver.params) > 1:
        try:
            solver.set_batch(policy, blocks, cap)  # the cap applies to the batched launch as well
        except L.LbmError as e:
            if e.status != L.LBM_E_UNSUPPORTED:
                raise


def _time(solver, steps: int, reps: int) -> float:
    solver.step(steps)  # warm-up (captures the graph)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(solver.stream)
        solver.step(steps)
        e1.record(solver.stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / steps)
    return best


def tune(solver, candidates: Optional[Iterable] = None, steps: int = 64, reps: int = 2,
         cache_path: Optional[str] = None, force: bool = False) -> dict:
    """Times every candidate, applies the fastest and returns
    {"best": (rows, xcd_remap, xcd_rows, tile_width, max_waves, stores, policy, blocks, fuse),
    "ms_per_step": {...}, "cached": bool}."""
    key = _key(solver)
    cached = None
    if not force:
        cached = _MEMO.get(key)
        if cached is None and cache_path and os.path.exists(cache_path):
            with open(cache_path) as fh:
                cached = json.load(fh).get(key)
    if cached is not None:
        _apply(solver, tuple(cached["best"]))
        return dict(cached, cached=True)

    n = len(solver.params)
    saved = [solver.state_save(k) for k in range(n)]
    steps0 = [solver.macros(k, raise_nonfinite=False)["step"] for k in range(n)]
    old_launch = [solver.get_launch(k) for k in range(n)]
    old_batch = solver.get_batch() if n > 1 else None
    times = {}
    try:
        for cand in (candidates or default_candidates(solver)):
            _apply(solver, cand)
            times[json.dumps(list(cand))] = _time(solver, steps, reps)
    finally:
        # a fused batch is configured as a whole (inst -1); anything else instance by instance
        whole = n > 1 and old_launch[0]["fuse"] == 2
        for k in ([-1] if whole else range(n)):
            o = old_launch[max(k, 0)]
            solver.set_launch(o["rows"], o["xcd_remap"], inst=k, tile_width=o["tile_width"], max_waves=o["max_waves"],
                              xcd_rows=o["xcd_rows"], stores=o["stores"], fuse=o["fuse"])
        if old_batch is not None:
            solver.set_batch(old_batch["policy"], old_batch["blocks"], old_batch["max_waves"])
        for k in range(n):
            solver.state_load(saved[k], steps0[k], inst=k)
        torch.cuda.synchronize()
    best = min(times, key=times.get)
    result = {"best": json.loads(best), "ms_per_step": times}
    _apply(solver, tuple(result["best"]))
    _MEMO[key] = result
    if cache_path:
        data = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                data = json.load(fh)
        data[key] = result
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1)
        os.replace(tmp, cache_path)
    return dict(result, cached=False)
