"""Autotuner of the stage-kernel tiling and the launch mode.

For a batch of sequences it times the candidate plans on the GPU (per-stage
launches with every combination of tile heights over the size classes
present, and the single persistent launch) and keeps the fastest. Results
are cached in a JSON file keyed by device architecture, compute type, the
size classes present and the batch's row count (rounded to a power of two),
so a later plan of the same shape reuses the choice.

    from paper_2411_17729_amd import tune
    tuning = tune.best_tuning(workload, compute="bf16")   # dict for CascadePlan
"""

from __future__ import annotations

import itertools
import json
import math
import os

import torch

from . import binding as B
from . import cascade as CC

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")
CLASS_MP = (32, 64, 128, 256)


def default_rows(mp, compute):
    """Default rows per stage tile (mirrors the library's defaults)."""
    f64 = compute == "f64"
    if f64:
        return {256: 32, 128: 64, 64: 64, 32: 128}[mp]
    return {256: 64, 128: 64, 64: 128, 32: 256}[mp]


def _pad(m):
    return 32 if m <= 32 else 64 if m <= 64 else 128 if m <= 128 else 256


def signature(wl, compute):
    arch = "unknown"
    if torch.cuda.is_available():
        arch = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu").split(":")[0]
    classes = sorted({_pad(wl.sets[s.param_set].m) for s in wl.seqs})
    rows = sum(s.L for s in wl.seqs)
    ragged = len(classes) > 1 or len({(s.L, s.N) for s in wl.seqs}) > 1
    return f"{arch}/{compute}/mp{'-'.join(map(str, classes))}/rows2^{int(math.log2(max(rows, 1)))}" \
           f"/{'ragged' if ragged else 'uniform'}"


def candidates(wl, compute):
    classes = sorted({_pad(wl.sets[s.param_set].m) for s in wl.seqs})
    opts = []
    for combo in itertools.product(*[(default_rows(mp, compute), default_rows(mp, compute) // 2)
                                     for mp in classes]):
        rows = [0, 0, 0, 0]
        for mp, r in zip(classes, combo):
            rows[CLASS_MP.index(mp)] = r
        opts.append({"launch": "per_stage", "tile_rows": rows})
    opts.append({"launch": "persistent", "tile_rows": [0, 0, 0, 0]})
    return opts


def time_plan(plan, u, reps=5, warm=2):
    y = torch.empty(plan.layout.y_numel, dtype=plan.state_dtype, device=u.device)
    for _ in range(warm):
        plan.apply(u, out=y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        plan.apply(u, out=y)
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def tune(wl, compute="bf16", reps=5, verbose=False):
    """Times every candidate on the current GPU; returns (best, table)."""
    u = CC.pack_u(wl, dtype=torch.float64 if compute == "f64" else torch.float32)
    table = []
    for cand in candidates(wl, compute):
        plan = CC.plan_for_workload(wl, compute=compute, launch=cand["launch"],
                                    tile_rows=tuple(cand["tile_rows"]))
        ms = time_plan(plan, u, reps=reps)
        plan.close()
        table.append(dict(cand, ms=ms))
        if verbose:
            print(f"tune {cand} {ms:.4f} ms", flush=True)
    best = min(table, key=lambda r: r["ms"])
    return best, table


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def best_tuning(wl, compute="bf16", path=CACHE, retune=False, save=True):
    """Cached choice for this batch shape, tuning on a miss."""
    key = signature(wl, compute)
    cache = load_cache(path)
    if not retune and key in cache:
        c = cache[key]
        return {"launch": c["launch"], "tile_rows": tuple(c["tile_rows"])}
    best, table = tune(wl, compute)
    cache[key] = {"launch": best["launch"], "tile_rows": list(best["tile_rows"]),
                  "ms": best["ms"], "candidates": table}
    if save:
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return {"launch": best["launch"], "tile_rows": tuple(best["tile_rows"])}
