"""Autotuner of the plan choices that shape the hot path.

For a batch of sequences it times plans on the GPU and keeps the fastest, by
coordinate descent from the library's defaults over the choices that the
plan actually uses (a choice the plan ignores is not timed):

  launch        per-stage launches or the one persistent launch
  input_stages  automatic (fold leading stages into the input pass) or none
  chain_blocks  16-row blocks per wave segment of the chain kernel
  pair_blocks   16-row blocks per workgroup segment of a stage pair
  fold_stages   stages folded into the output pass (automatic, none, 4, 5)
  state_bf16    BF16 state between passes (BF16 plans, when allowed)
  min_padded_m  operators of m <= 64 padded to 128 (ragged BF16 batches with
                larger classes too: every class then runs the fused passes),
                timed with FP32 state and, when allowed, with BF16 state
  tile_rows     rows per tile of the tiled stage kernel (plans that use it)

Every candidate's output on the tuning input is compared with the default
plan's; a candidate further away than the tolerance of its compute type
(BF16 5e-3, FP32 1e-6, FP64 1e-12, relative per sequence) is rejected, so a
choice that changes the rounding (BF16 state, the output fold) is kept only
within that bound. Results are cached in a JSON file (``SSM_TUNING_CACHE`` or
``tuning_cache.json`` next to this file) keyed by device architecture,
compute type, size classes, the batch's row count (rounded to a power of
two), whether it is ragged and whether BF16 state was allowed.

    from paper_2411_17729_amd import tune
    kw = tune.best_tuning(workload, compute="bf16")   # keyword arguments for plan_for_workload
"""

from __future__ import annotations

import json
import math
import os

import torch

from . import binding as B
from . import cascade as CC

CACHE = os.environ.get("SSM_TUNING_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json"))
CLASS_MP = (32, 64, 128, 256)
TOL = {"bf16": 5e-3, "f32": 1e-6, "f64": 1e-12}


def default_rows(mp, compute):
    """Default rows per stage tile (mirrors the library's defaults)."""
    if compute == "f64":
        return {256: 32, 128: 64, 64: 64, 32: 128}[mp]
    return {256: 64, 128: 64, 64: 128, 32: 256}[mp]


def _pad(m):
    return 32 if m <= 32 else 64 if m <= 64 else 128 if m <= 128 else 256


def _classes(wl):
    return sorted({_pad(wl.sets[s.param_set].m) for s in wl.seqs})


def signature(wl, compute, allow_bf16_state=False):
    arch = "unknown"
    if torch.cuda.is_available():
        arch = getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gpu").split(":")[0]
    classes = _classes(wl)
    rows = sum(s.L for s in wl.seqs)
    ragged = len(classes) > 1 or len({(s.L, s.N) for s in wl.seqs}) > 1
    return f"{arch}/{compute}/mp{'-'.join(map(str, classes))}/rows2^{int(math.log2(max(rows, 1)))}" \
           f"/{'ragged' if ragged else 'uniform'}" + ("/bf16state" if allow_bf16_state else "")


def defaults():
    return {"launch": "auto", "input_stages": 0, "chain_blocks": 0, "pair_blocks": 0, "fold_stages": 0,
            "state_bf16": 0, "min_padded_m": 0, "tile_rows": (0, 0, 0, 0)}


def knob_values(wl, compute, info, allow_bf16_state):
    """The values worth timing for each choice the plan described by info uses."""
    vals = {"launch": ["per_stage", "persistent"], "input_stages": [0, -1]}
    if info["stage_kernel"] == B.SSM_STAGE_CHAIN and info["launch"] == B.SSM_LAUNCH_PER_STAGE:
        vals["chain_blocks"] = [0, 2, 4, 8, 16, 32]
    if info["pair_launches"] > 0:
        vals["pair_blocks"] = [0, 8, 16, 32, 64, 128]
    if compute == "bf16" and info["launch"] == B.SSM_LAUNCH_PER_STAGE:
        vals["fold_stages"] = [0, -1, 4, 5]
        if allow_bf16_state:
            vals["state_bf16"] = [0, 1]
        cls = _classes(wl)
        if min(cls) <= 64 and max(cls) >= 128:
            vals["min_padded_m"] = [0, 128]
    if info["stage_kernel"] == B.SSM_STAGE_TILED:
        rows = []
        for mp in _classes(wl):
            r = [0, 0, 0, 0]
            r[CLASS_MP.index(mp)] = default_rows(mp, compute) // 2
            rows.append(tuple(r))
        vals["tile_rows"] = [(0, 0, 0, 0)] + rows
    return vals


def _max_rel_diff(wl, y, ref):
    """Largest per-sequence relative Frobenius difference of two packed outputs."""
    worst = 0.0
    for a, b in zip(CC.unpack_y(wl, y), CC.unpack_y(wl, ref)):
        nb = float(torch.linalg.vector_norm(torch.as_tensor(b)))
        d = float(torch.linalg.vector_norm(torch.as_tensor(a) - torch.as_tensor(b)))
        worst = max(worst, d / nb if nb > 0 else d)
    return worst


def time_plan(plan, u, reps=7, warm=2):
    """Median milliseconds of one apply (eager)."""
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


def _plan(wl, compute, kw, with_backward=False):
    k = dict(kw)
    k["tile_rows"] = tuple(k["tile_rows"])
    return CC.plan_for_workload(wl, compute=compute, with_backward=with_backward, **k)


def tune(wl, compute="bf16", reps=7, verbose=False, allow_bf16_state=False, tol=None):
    """Coordinate descent from the defaults; returns (best keyword arguments,
    best ms, table of every timed candidate)."""
    tol = TOL[compute] if tol is None else tol
    u = CC.pack_u(wl, dtype=torch.float64 if compute == "f64" else torch.float32)
    cur = defaults()
    plan = _plan(wl, compute, cur)
    info = plan.info()
    ref = plan.apply(u).clone()
    torch.cuda.synchronize()
    best_ms = time_plan(plan, u, reps)
    plan.close()
    table = [dict(cur, ms=best_ms)]
    # the launch mode first; the other choices are those the plan of the
    # chosen mode uses
    order = ["launch", "input_stages", "chain_blocks", "pair_blocks", "fold_stages", "state_bf16", "min_padded_m",
             "tile_rows"]
    for knob in order:
        if knob != "launch":
            plan = _plan(wl, compute, cur)
            info = plan.info()
            plan.close()
        values = knob_values(wl, compute, info, allow_bf16_state).get(knob, [])
        cands = []
        for v in values:
            if v == cur[knob] or (knob == "launch" and v == "auto"):
                continue
            cand = dict(cur)
            cand[knob] = v
            cands.append(cand)
            if knob == "min_padded_m" and allow_bf16_state and not cur["state_bf16"]:
                cands.append(dict(cand, state_bf16=1))  # the padding is what lets the state be BF16
        for cand in cands:
            row = dict(cand)
            try:
                plan = _plan(wl, compute, cand)
            except B.SSMError as e:
                row["rejected"] = str(e)
                table.append(row)
                continue
            if cand["state_bf16"] and plan.info()["state_dtype"] != B.SSM_BF16:
                plan.close()
                row["rejected"] = "the plan keeps FP32 state"
                table.append(row)
                continue
            y = plan.apply(u).clone()
            torch.cuda.synchronize()
            row["rel_diff"] = _max_rel_diff(wl, y, ref)
            if row["rel_diff"] > tol:
                plan.close()
                row["rejected"] = f"outputs differ by {row['rel_diff']:.2e} > {tol:.1e}"
                table.append(row)
                continue
            row["ms"] = time_plan(plan, u, reps)
            plan.close()
            table.append(row)
            if verbose:
                print(f"tune {row}", flush=True)
            if row["ms"] < best_ms:
                best_ms = row["ms"]
                cur = cand
    return cur, best_ms, table


def load_cache(path=None):
    path = path or CACHE
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def best_tuning(wl, compute="bf16", path=None, retune=False, save=True, allow_bf16_state=False, tol=None):
    """Cached choice for this batch shape (keyword arguments for
    plan_for_workload), tuning on a miss."""
    path = path or CACHE
    key = signature(wl, compute, allow_bf16_state)
    cache = load_cache(path)
    if not retune and key in cache:
        c = cache[key]["choice"]
        c["tile_rows"] = tuple(c["tile_rows"])
        return c
    best, ms, table = tune(wl, compute, allow_bf16_state=allow_bf16_state, tol=tol)
    cache[key] = {"choice": dict(best, tile_rows=list(best["tile_rows"])), "ms": ms, "candidates": table}
    if save:
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True, default=list)
    best = dict(best)
    best["tile_rows"] = tuple(best["tile_rows"])
    return best
