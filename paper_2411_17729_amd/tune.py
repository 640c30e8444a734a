"""Autotuner of the stage-kernel tiling, the launch mode and (on request) the
state type kept between passes.

For a batch of sequences it times the candidate plans on the GPU (per-stage
launches with every combination of tile heights over the size classes
present, and the single persistent launch) and keeps the fastest. With
allow_bf16_state, BF16 plans are also timed with the state kept in BF16
between passes; such a candidate counts only if the plan can keep it and its
outputs on the tuning input stay within state_tol (relative, per sequence)
of the same plan with FP32 state. Results are cached in a JSON file keyed by
device architecture, compute type, the size classes present, the batch's row
count (rounded to a power of two) and whether BF16 state was allowed, so a
later plan of the same shape reuses the choice.

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


def signature(wl, compute, allow_bf16_state=False):
    arch = "unknown"
    if torch.cuda.is_available():
        arch = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu").split(":")[0]
    classes = sorted({_pad(wl.sets[s.param_set].m) for s in wl.seqs})
    rows = sum(s.L for s in wl.seqs)
    ragged = len(classes) > 1 or len({(s.L, s.N) for s in wl.seqs}) > 1
    return f"{arch}/{compute}/mp{'-'.join(map(str, classes))}/rows2^{int(math.log2(max(rows, 1)))}" \
           f"/{'ragged' if ragged else 'uniform'}" + ("/bf16state" if allow_bf16_state else "")


def candidates(wl, compute, allow_bf16_state=False):
    classes = sorted({_pad(wl.sets[s.param_set].m) for s in wl.seqs})
    opts = []
    for combo in itertools.product(*[(default_rows(mp, compute), default_rows(mp, compute) // 2)
                                     for mp in classes]):
        rows = [0, 0, 0, 0]
        for mp, r in zip(classes, combo):
            rows[CLASS_MP.index(mp)] = r
        opts.append({"launch": "per_stage", "tile_rows": rows, "state_bf16": 0})
        if allow_bf16_state and compute == "bf16":
            opts.append({"launch": "per_stage", "tile_rows": rows, "state_bf16": 1})
    opts.append({"launch": "persistent", "tile_rows": [0, 0, 0, 0], "state_bf16": 0})
    return opts


def _max_rel_diff(wl, y, ref):
    """Largest per-sequence relative Frobenius difference of two packed outputs."""
    worst = 0.0
    for a, b in zip(CC.unpack_y(wl, y), CC.unpack_y(wl, ref)):
        nb = float(torch.linalg.vector_norm(torch.as_tensor(b)))
        d = float(torch.linalg.vector_norm(torch.as_tensor(a) - torch.as_tensor(b)))
        worst = max(worst, d / nb if nb > 0 else d)
    return worst


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


def tune(wl, compute="bf16", reps=5, verbose=False, allow_bf16_state=False, state_tol=5e-3):
    """Times every candidate on the current GPU; returns (best, table). A
    BF16-state candidate is kept only if the plan can keep the state in BF16
    and its outputs stay within state_tol of the same candidate with FP32
    state (the one before it in the candidate list)."""
    u = CC.pack_u(wl, dtype=torch.float64 if compute == "f64" else torch.float32)
    table = []
    ref = None  # outputs of the last FP32-state candidate
    for cand in candidates(wl, compute, allow_bf16_state):
        plan = CC.plan_for_workload(wl, compute=compute, launch=cand["launch"],
                                    tile_rows=tuple(cand["tile_rows"]), state_bf16=cand["state_bf16"])
        row = dict(cand)
        if cand["state_bf16"]:
            if plan.info()["state_dtype"] != B.SSM_BF16:
                plan.close()
                row["rejected"] = "the plan keeps FP32 state"
                table.append(row)
                continue
            y = plan.apply(u).clone()
            torch.cuda.synchronize()
            row["rel_diff"] = _max_rel_diff(wl, y, ref)
            if row["rel_diff"] > state_tol:
                plan.close()
                row["rejected"] = f"outputs differ by {row['rel_diff']:.2e} > {state_tol:.1e}"
                table.append(row)
                continue
        elif cand["launch"] == "per_stage":
            ref = plan.apply(u).clone()
            torch.cuda.synchronize()
        row["ms"] = time_plan(plan, u, reps=reps)
        plan.close()
        table.append(row)
        if verbose:
            print(f"tune {row}", flush=True)
    best = min((r for r in table if "ms" in r), key=lambda r: r["ms"])
    return best, table


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def best_tuning(wl, compute="bf16", path=CACHE, retune=False, save=True, allow_bf16_state=False,
                state_tol=5e-3):
    """Cached choice for this batch shape, tuning on a miss."""
    key = signature(wl, compute, allow_bf16_state)
    cache = load_cache(path)
    if not retune and key in cache:
        c = cache[key]
        return {"launch": c["launch"], "tile_rows": tuple(c["tile_rows"]),
                "state_bf16": c.get("state_bf16", 0)}
    best, table = tune(wl, compute, allow_bf16_state=allow_bf16_state, state_tol=state_tol)
    cache[key] = {"launch": best["launch"], "tile_rows": list(best["tile_rows"]),
                  "state_bf16": best["state_bf16"], "ms": best["ms"], "candidates": table}
    if save:
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return {"launch": best["launch"], "tile_rows": tuple(best["tile_rows"]),
            "state_bf16": best["state_bf16"]}
