#!/usr/bin/env python
"""Throughput of the fast cascade on one MI355X.

Workload: 16 sequences x L = 16384 of one shared HiPPO-LegS model (m = 256,
p = q = 8, B, C, D ~ N(0, 1/m)), one step size per sequence (log-uniform in
[1e-3, 1e-1]), N = 13 (degree 16383), u ~ N(0, 1), all seeded and synthetic.

A step is one full forward pass over the batch: the input pass (Bbar u with
the leading stages folded) and the remaining stage launches with the fused
C x + D u output, inputs already in HBM, captured once as a HIP graph and
replayed. The headline is the cascade with BF16 MFMA operands (FP32
accumulation) and the state between passes in BF16 (--state f32: in FP32);
the same apply with the other state type, the FP32-MFMA cascade and the
plain FP32 recursion on the same GPU are measured beside it, each with its
relative error against the FP64 oracle, and the FP32 cascade is compared
with the FP32 recursion at the same accuracy. Prepare (discretization and
squarings) is timed on its own and end to end. Kernel statistics for the
roofline come from a separate eager pass with per-launch HIP events. The
CPU oracle leg runs first, in forked worker processes, before the GPU is
initialised. Prints one JSON line. --workload backward|ragged measures the
gradient pass and the ragged persistent batch instead.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype bf16|f32] [--state f32|bf16]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "output steps/s + MFMA util: cascade vs recursion on one GPU at rel err vs FP64"
PEAK = {"hbm_GBps": 8000.0, "bf16_TFLOPs": 2500.0, "f32_TFLOPs": 157.3, "f64_TFLOPs": 78.6}
# stage kernels: the source files each is built from
STAGE_KERNELS = {"k_stage": ("kernels_stage.hip", "stage_common.h"),
                 "k_stage_res": ("kernels_stage_res.hip", "stage_res.h", "stage_common.h"),
                 "k_stage_chain": ("kernels_stage_chain.hip", "stage_chain.h", "stage_res.h",
                                   "stage_common.h"),
                 "k_stage_pair": ("kernels_stage_pair.hip", "stage_common.h")}
# the kernel of each ssm_stage_kernel value
STAGE_KERNEL_IDS = {1: "k_stage", 2: "k_stage_res", 3: "k_stage_chain"}


def kernel_sha256(name):
    """SHA-256 over the concatenated sources of a stage kernel."""
    h = hashlib.sha256()
    for f in STAGE_KERNELS[name]:
        h.update(open(os.path.join(ROOT, "paper_2411_17729_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def dominant_kernel(info):
    """The stage kernel that moves most of an apply's bytes, with its timing kind,
    launches, compulsory bytes and flops per apply: the stage-pair kernel when
    the plan pairs stages, else the plan's per-stage kernel over all stage
    launches."""
    from paper_2411_17729_amd import binding as B
    if info["pair_launches"] > 0:
        return ("k_stage_pair", B.TIMING_PAIR, info["pair_launches"], info["pair_bytes"],
                info["pair_flops"])
    return (STAGE_KERNEL_IDS[info["stage_kernel"]], B.TIMING_STAGE, info["stage_launches"],
            info["stage_bytes"], info["stage_flops"])


def _args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--state", default="bf16", choices=["f32", "bf16"],
                    help="state kept between the passes of a BF16 apply (bf16: where every pass "
                         "supports it, the default: within the BF16 tolerance, errors in the line); "
                         "the other choice is timed beside it")
    ap.add_argument("--workload", default="batched", choices=["batched", "backward", "ragged", "plr"],
                    help="batched: 16 x L=16384, m=256 forward (the headline line); backward: "
                         "8 x L=8192, m=128 FP32 gradients; ragged: 256 sequences of uneven L and m, "
                         "BF16, one persistent launch replayed as a HIP graph, forward and backward; "
                         "plr: the batched workload in FP32 and FP64 with partitioned low-rank powers "
                         "against the dense stages")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--ckpt-every", type=int, default=1,
                    help="backward workloads: stage inputs kept every this many stages (1: every "
                         "stage, no recompute; 0: the library's automatic sqrt rule)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other dtype and the recursion comparator")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU oracle sample")
    ap.add_argument("--stream-probe-mib", type=int, default=0,
                    help="only time plain streams over buffers of this size (torch's fill, sum and "
                         "copy kernels: write-only, read-only, read+write) and print their rates")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the measurement, run one device-to-device copy of this many MiB "
                         "(a reference for hardware byte counters)")
    return ap.parse_args()


def _host_workers():
    """Worker processes for the CPU oracle leg: the host's cores available to
    this process, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _oracle_recursion_job(job):
    """One sequence through the oracle: trapezoid discretization and the
    recursion, numpy FP64, one BLAS thread (the pool supplies the parallelism)."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    A, Bm, C, D, delta, u = job
    with threadpool_limits(limits=1):
        Abar, Bbar = O.trapezoid(A, Bm, delta)
        y, _ = O.recursion(Abar, Bbar, C, D, u)
    return y


def _oracle_grads_job(job):
    """One sequence's gradients through the oracle (BPTT and the trapezoid adjoint)."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    A, Bm, C, D, delta, u, dy, N = job
    with threadpool_limits(limits=1):
        return O.grads_full(A, Bm, C, D, delta, u, dy, N)


def cpu_oracle_leg(fn, jobs, seconds, workers):
    """Runs fn over jobs in a pool of `workers` forked processes, a round of
    `workers` jobs at a time, until the jobs run out or `seconds` have passed
    after a round. Call before anything initialises the GPU (the children are
    forked). Returns (results by job index, wall seconds, workers)."""
    import multiprocessing as mp
    t0 = time.perf_counter()
    res = {}
    with mp.get_context("fork").Pool(workers) as pool:
        for r0 in range(0, len(jobs), workers):
            idx = list(range(r0, min(len(jobs), r0 + workers)))
            for i, out in zip(idx, pool.map(fn, [jobs[i] for i in idx], chunksize=1)):
                res[i] = out
            if time.perf_counter() - t0 >= seconds:
                break
    return res, time.perf_counter() - t0, workers


def traffic_path(workload, dtype, state="f32"):
    suffix = "" if state == "f32" else f"_state_{state}"
    return os.path.join(ROOT, "profiles", f"stage_traffic_{workload}_{dtype}{suffix}.json")


def _stage_traffic(workload, dtype, name, state="f32"):
    """HBM bytes per launch of a stage kernel from committed rocprofv3 counter
    runs, if they were taken on the kernel's current source with this state type."""
    path = traffic_path(workload, dtype, state)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel") != name or rec.get("kernel_sha256") != kernel_sha256(name):
        return None
    if rec.get("state", "f32") != state:
        return None
    return rec.get("traffic_bytes_per_launch")


def stream_probe(mib, reps=20):
    """Rates of plain HBM streams with torch's own kernels on buffers of mib
    MiB: the write, read and read+write rates a simple kernel reaches here."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    acc = torch.empty((), dtype=torch.float32, device="cuda")
    cases = {"write (fill)": (lambda: a.fill_(2.0), n * 4),
             "read (sum)": (lambda: torch.sum(a, dim=0, out=acc), n * 4),
             "read+write (copy)": (lambda: b.copy_(a), 2 * n * 4)}
    res = {}
    for name, (fn, nbytes) in cases.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": round(ms, 4), "GBps": round(nbytes / ms / 1e6, 1)}
    return {"stream_probe_MiB": mib, "reps": reps, "rates": res}


def main():
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_17729_amd import workloads as W

    if args.stream_probe_mib > 0:
        print(json.dumps(stream_probe(args.stream_probe_mib)), flush=True)
        return
    if args.workload == "backward":
        return bench_backward(args)
    if args.workload == "ragged":
        return bench_ragged(args)
    if args.workload == "plr":
        return bench_plr(args)

    wl = W.batched(seed=args.seed)
    # the CPU oracle leg runs first, in forked workers, before the GPU is touched
    cpu = None
    if not args.no_cpu:
        ps0 = wl.sets[0]
        jobs = [(ps0.A, ps0.B, ps0.C, ps0.D, s.delta, s.u.astype(np.float32).astype(np.float64))
                for s in wl.seqs]
        cpu = cpu_oracle_leg(_oracle_recursion_job, jobs, args.cpu_seconds, _host_workers())

    from paper_2411_17729_amd import binding as B
    from paper_2411_17729_amd import cascade as CC

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    B.load()
    s0 = wl.seqs[0]
    ps = wl.sets[0]
    wname = f"hippo_m{ps.m}_p{ps.p}_q{ps.q}_B{len(wl.seqs)}_L{s0.L}_N{s0.N}"
    total_steps = wl.total_steps
    u32 = CC.pack_u(wl, dtype=torch.float32)
    K, Wm = args.steps, args.warmup

    def run(plan, fn_name, steps, warm, timing_kind=None, graph=False):
        """Average ms per call over `steps` calls (graph: replays of one captured
        apply on a side stream), then, with timing_kind, a separate eager pass
        with per-launch HIP events for the kernel statistics."""
        fn = getattr(plan, fn_name)
        y = torch.empty(plan.layout.y_numel, dtype=plan.state_dtype, device="cuda")
        g = None
        if graph:
            stream = torch.cuda.Stream()
            torch.cuda.synchronize()
            g = plan.graph_apply(u32, y, stream)
            launch = lambda: CC.CascadePlan.graph_launch(g, stream)
        else:
            stream = torch.cuda.current_stream()
            launch = lambda: fn(u32, out=y)
        for _ in range(warm):
            launch()
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for _ in range(steps):
            launch()
        t1.record(stream)
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        if g is not None:
            CC.CascadePlan.graph_destroy(g)
        kern = None
        if timing_kind is not None:
            plan.timing_read(timing_kind)  # clear earlier records
            plan.timing(True)
            for _ in range(min(steps, 10)):
                fn(u32, out=y)
            torch.cuda.synchronize()
            plan.timing(False)
            kern = plan.timing_read(timing_kind)
        return y, ms / steps, kern

    def roofline(plan, kern, dtype, steps):
        info = plan.info()
        name, _, launches, nbytes, flops = dominant_kernel(info)
        state = {B.SSM_F32: "f32", B.SSM_BF16: "bf16", B.SSM_F64: "f64"}[info["state_dtype"]]
        n_launch, k_ms = kern
        avg_ms = k_ms / max(n_launch, 1)
        per_launch_bytes = nbytes / launches
        dense_flops = flops / launches
        # every power lower triangular (HiPPO): a stage product needs the
        # m (m + 1) / 2 nonzero entries of P_k, not m^2, so that is the
        # algorithmic count (the dense one stays beside it)
        tri = info["n_ops"] > 0 and info["lower_ops"] == info["n_ops"]
        flops = flops * ((ps.m + 1) / (2 * ps.m) if tri else 1.0)
        per_launch_flops = flops / launches
        gbps = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        tflops = per_launch_flops / (avg_ms * 1e-3) / 1e12
        peak_tf = PEAK["bf16_TFLOPs"] if dtype == "bf16" else PEAK["f32_TFLOPs"]
        intensity = flops / nbytes
        ridge = peak_tf * 1e12 / (PEAK["hbm_GBps"] * 1e9)
        bound = "mfma" if intensity > ridge else "hbm"
        traffic = _stage_traffic(wname, dtype, name, state)
        if bound == "hbm":
            rf = {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK["hbm_GBps"],
                  "unit": "GB/s", "frac": round(gbps / PEAK["hbm_GBps"], 4)}
        else:
            rf = {"bound": "mfma", "achieved": round(tflops, 2), "peak": peak_tf,
                  "unit": "TFLOP/s", "frac": round(tflops / peak_tf, 4)}
        rf["traffic"] = traffic
        rf.update({"kernel": name, "launches_timed": n_launch, "avg_launch_ms": round(avg_ms, 5),
                   "algorithmic_bytes_per_launch": round(per_launch_bytes),
                   "algorithmic_flops_per_launch": round(per_launch_flops),
                   "mfma_util": round(tflops / peak_tf, 4), "hbm_GBps": round(gbps, 1)})
        if tri:
            rf["dense_flops_per_launch"] = round(dense_flops)
            rf["flops_note"] = "lower-triangular powers: m (m + 1) / 2 of the m^2 entries of P_k"
        if name == "k_stage_chain" and dtype == "f32" and tri:
            # the FP32 chain kernel skips the zero 16 x 16 blocks of the lower-triangular
            # powers: of (m/16)^2 blocks per product it runs (m/16)(m/16 + 1)/2, and at
            # padded m 256 (two workgroups per unit, one skip pattern for both) 2 x 76 of 256
            nv = ps.m // 16
            frac = 152 / 256 if ps.m > 128 else nv * (nv + 1) / 2 / (nv * nv)
            rf["mfma_blocks_executed_frac"] = round(frac, 4)
            rf["mfma_util_executed"] = round(dense_flops / (avg_ms * 1e-3) / 1e12 * frac / peak_tf, 4)
        return rf

    # ---------------- headline: the cascade in the chosen dtype ----------------
    # plan choices from the autotuner's cache (tuned on a miss): BF16 state
    # between passes is a candidate with --state bf16, kept only within the
    # tuner's tolerance of the FP32-state plan
    from paper_2411_17729_amd import tune
    allow_sb = args.dtype == "bf16" and args.state == "bf16"
    tkey = tune.signature(wl, args.dtype, allow_sb)
    cached = tkey in tune.load_cache()
    tn = tune.best_tuning(wl, compute=args.dtype, allow_bf16_state=allow_sb)
    sb = int(tn.get("state_bf16", 0))
    torch.cuda.synchronize()
    t_plan = time.perf_counter()
    plan = CC.plan_for_workload(wl, compute=args.dtype, **tn)
    torch.cuda.synchronize()
    plan_ms_first = (time.perf_counter() - t_plan) * 1e3
    y_main, ms_main, kern = run(plan, "apply", K, Wm, timing_kind=dominant_kernel(plan.info())[1],
                                graph=True)
    state_name = {B.SSM_F32: "f32", B.SSM_BF16: "bf16"}[plan.info()["state_dtype"]]
    value = total_steps / (ms_main * 1e-3)
    rf = roofline(plan, kern, args.dtype, K)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "output steps/s", "n_gpus": 1,
        "steps": K, "warmup": Wm, "ms_per_step": round(ms_main, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": wname, "sequences": len(wl.seqs), "L": s0.L, "m": ps.m, "p": ps.p,
                   "q": ps.q, "N": s0.N, "delta": "log-uniform [1e-3, 1e-1] per sequence",
                   "A": "HiPPO-LegS (1-based)", "seed": args.seed},
        "roofline": rf,
        "state": state_name,
        "tuning": {"choice": {k: (list(v) if isinstance(v, tuple) else v) for k, v in tn.items()},
                   "cache_key": tkey, "from_cache": cached},
    }
    ys = {args.dtype: CC.unpack_y(wl, y_main)}

    # prepare (discretization, squarings, packing; FP64 on the GPU, one
    # synchronization at its end): host wall time of ssm_cascade_prepare on the
    # plan's workspace, median of 5, and the first plan built end to end
    # (workspace allocation and parameter upload included)
    prep = []
    for _ in range(5):
        torch.cuda.synchronize()
        t_p = time.perf_counter()
        plan.prepare_again()
        prep.append((time.perf_counter() - t_p) * 1e3)
    prep_ms = sorted(prep)[len(prep) // 2]
    out["prepare_ms"] = round(prep_ms, 3)
    out["prepare"] = {"median_ms": round(prep_ms, 3), "runs_ms": [round(x, 3) for x in prep],
                      "first_plan_ms": round(plan_ms_first, 3),
                      "end_to_end_ms": round(prep_ms + ms_main, 4),
                      "end_to_end_output_steps_per_s": round(total_steps / ((prep_ms + ms_main) * 1e-3), 1),
                      "note": "ssm_cascade_prepare on the plan's own workspace (host wall time, it "
                              "synchronizes its stream); end_to_end = prepare + one apply"}

    # ---------------- comparators on the same GPU ----------------
    if not args.no_compare:
        if args.dtype == "bf16":
            # the same BF16 apply with the other state type between passes
            plan_s = CC.plan_for_workload(wl, compute="bf16", **dict(tn, state_bf16=1 - sb))
            sname = {B.SSM_F32: "f32", B.SSM_BF16: "bf16"}[plan_s.info()["state_dtype"]]
            y_s, ms_s, kern_s = run(plan_s, "apply", K, Wm,
                                    timing_kind=dominant_kernel(plan_s.info())[1], graph=True)
            key = f"bf16_state_{sname}"
            ys[key] = CC.unpack_y(wl, y_s)
            out[f"cascade_{key}"] = {"value": round(total_steps / (ms_s * 1e-3), 1),
                                     "ms_per_step": round(ms_s, 4),
                                     "roofline": roofline(plan_s, kern_s, "bf16", K)}
            plan_s.close()
        other = "f32" if args.dtype == "bf16" else "bf16"
        tn_o = tune.best_tuning(wl, compute=other)  # the autotuner's choice, cached
        plan_o = CC.plan_for_workload(wl, compute=other, **tn_o)
        y_o, ms_o, kern_o = run(plan_o, "apply", K, Wm, timing_kind=dominant_kernel(plan_o.info())[1],
                                graph=True)
        ys[other] = CC.unpack_y(wl, y_o)
        out[f"cascade_{other}"] = {"value": round(total_steps / (ms_o * 1e-3), 1),
                                    "ms_per_step": round(ms_o, 4),
                                    "roofline": roofline(plan_o, kern_o, other, K),
                                    "tuning": {k: (list(v) if isinstance(v, tuple) else v)
                                               for k, v in tn_o.items()}}
        plan_r = plan_o if other == "f32" else plan
        rsteps = max(2, K // 10)
        y_r, ms_r, _ = run(plan_r, "recursion", rsteps, 1)
        ys["recursion_f32"] = CC.unpack_y(wl, y_r)
        out["recursion_f32"] = {"value": round(total_steps / (ms_r * 1e-3), 1),
                                "ms_per_step": round(ms_r, 4), "steps": rsteps}
        # the FP32 cascade against the FP32 recursion: the same operand precision
        # and comparable error against FP64 (both in rel_err_vs_fp64)
        ms_f32 = ms_o if other == "f32" else ms_main
        out["speedup_vs_recursion_same_accuracy"] = round(ms_r / ms_f32, 2)
        if args.dtype != "f32":
            # the headline (BF16 operands) against the FP32 recursion: different accuracies
            out["speedup_vs_recursion_cross_dtype"] = round(ms_r / ms_main, 2)

    # ---------------- CPU oracle: baseline timing and FP64 reference ----------------
    if cpu is not None:
        refs, t_cpu, workers = cpu
        done = sorted(refs)
        steps_cpu = sum(wl.seqs[i].L for i in done)
        out["cpu_baseline"] = {
            "value": round(steps_cpu / t_cpu, 1), "unit": "output steps/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{len(done)} of {len(wl.seqs)} sequences in full (L={s0.L}), oracle.trapezoid + "
                      f"oracle.recursion, numpy FP64, one sequence per worker process with one BLAS "
                      f"thread, {workers} workers, {t_cpu:.2f} s wall"}
        rel = {}
        for name, yl in ys.items():
            ey = max(float(np.linalg.norm(yl[i] - refs[i]) / np.linalg.norm(refs[i])) for i in done)
            du = {i: wl.seqs[i].u.astype(np.float32).astype(np.float64) @ ps.D.T for i in done}
            ex = max(float(np.linalg.norm((yl[i] - du[i]) - (refs[i] - du[i])) /
                           np.linalg.norm(refs[i] - du[i])) for i in done)
            rel[name] = {"y": ey, "Cx": ex}
        out["rel_err_vs_fp64"] = {k: {kk: float(f"{vv:.3e}") for kk, vv in v.items()} for k, v in rel.items()}
        out["rel_err_sample"] = (f"sequences {done}; y: the output, Cx: y - D u (the part that "
                                 f"passes through the state)")

    _copy_probe(args, out)

    print(json.dumps(out), flush=True)


def _copy_probe(args, out):
    """One device-to-device copy of --copy-probe-mib MiB after the measurement:
    a transfer of known size beside the kernels in a counter run."""
    import torch
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = n * 4


def _timed(fn, steps, warm, stream=None):
    """Average milliseconds of fn() over `steps` calls after `warm` untimed ones."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def _stage_flops(wl, ks=None):
    """Sum over sequences and stages of 2 m^2 (L - 2^k) (rows with a partner)."""
    tot = 0.0
    for s in wl.seqs:
        m = wl.sets[s.param_set].m
        last = min(s.N, (s.L - 1).bit_length() - 1) if s.L > 1 else -1
        for k in range(last + 1):
            if ks is None or k in ks:
                tot += 2.0 * m * m * max(0, s.L - (1 << k))
    return tot


def _gpu_init():
    import torch
    from paper_2411_17729_amd import binding as B
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    B.load()


def bench_backward(args):
    """Gradients of sum(dy * y) for 8 sequences x L = 8192, m = 128 (FP32)."""
    import numpy as np
    import torch
    from paper_2411_17729_amd import workloads as W

    wl = W.backward(seed=args.seed)
    ps = wl.sets[0]
    s0 = wl.seqs[0]
    cpu = None
    if not args.no_cpu:  # before the GPU is touched (forked workers)
        jobs = [(ps.A, ps.B, ps.C, ps.D, s.delta, s.u.astype(np.float32).astype(np.float64),
                 d.astype(np.float32).astype(np.float64), s.N) for s, d in zip(wl.seqs, wl.dy)]
        cpu = cpu_oracle_leg(_oracle_grads_job, jobs, args.cpu_seconds, _host_workers())
    _gpu_init()
    from paper_2411_17729_amd import binding as B
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute="f32", with_backward=True, ckpt_every=args.ckpt_every)
    u = CC.pack_u(wl, dtype=torch.float32)
    dy = torch.as_tensor(np.concatenate([d.reshape(-1) for d in wl.dy]), device="cuda").float()
    K, Wm = args.steps, args.warmup
    ms = _timed(lambda: plan.backward(u, dy), K, Wm)
    plan.timing(True)
    du, grads = plan.backward(u, dy)
    torch.cuda.synchronize()
    plan.timing(False)
    n_adj, t_adj = plan.timing_read(B.TIMING_ADJOINT)
    n_fwd, t_fwd = plan.timing_read(B.TIMING_STAGE)
    n_red, t_red = plan.timing_read(B.TIMING_REDUCE)
    flops_adj = _stage_flops(wl)  # the adjoint runs every stage once
    tf = flops_adj / (t_adj * 1e-3) / 1e12
    out = {
        "metric": METRIC, "value": round(wl.total_steps / (ms * 1e-3), 1), "unit": "output steps/s",
        "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"backward_hippo_m{ps.m}_p{ps.p}_q{ps.q}_B{len(wl.seqs)}_L{s0.L}_N{s0.N}",
                   "step": "ssm_cascade_backward: forward with checkpoints, recompute, adjoint "
                           "stages, gradient reductions, FP64 squaring and trapezoid adjoints",
                   "delta": s0.delta, "seed": args.seed, "ckpt_every": args.ckpt_every,
                   "workspace_GiB": round(plan._nbytes / 2**30, 2)},
        "roofline": {"bound": "mfma", "achieved": round(tf, 2), "peak": PEAK["f32_TFLOPs"],
                     "unit": "TFLOP/s", "frac": round(tf / PEAK["f32_TFLOPs"], 4), "traffic": None,
                     "kernel": "adjoint stages", "launches_timed": n_adj,
                     "avg_launch_ms": round(t_adj / max(n_adj, 1), 5)},
        "breakdown_ms": {"forward_and_recompute_stages": round(t_fwd, 4), "adjoint_stages": round(t_adj, 4),
                         "reductions": round(t_red, 4), "launches": [n_fwd, n_adj, n_red]},
    }
    if cpu is not None:
        res, t_cpu, workers = cpu
        done = sorted(res)
        out["cpu_baseline"] = {"value": round(sum(wl.seqs[i].L for i in done) / t_cpu, 1),
                               "unit": "output steps/s", "cores": workers, "kind": "oracle",
                               "sample": f"{len(done)} of {len(wl.seqs)} sequences, oracle.grads_full "
                                         f"(BPTT + trapezoid adjoint), numpy FP64, one sequence per worker "
                                         f"process with one BLAS thread, {workers} workers, {t_cpu:.2f} s wall"}
        du_h = du.double().cpu().numpy()
        off, rel = 0, {"du": 0.0}
        for i, s in enumerate(wl.seqs):
            n = s.L * ps.p
            if i in res:
                ref = res[i]["u"].reshape(-1)
                rel["du"] = max(rel["du"], float(np.linalg.norm(du_h[off:off + n] - ref) / np.linalg.norm(ref)))
            off += n
        if len(done) == len(wl.seqs):  # the parameter gradients are sums over every sequence
            for j, k in enumerate("ABCD"):
                acc = sum(res[i][k] for i in done)
                gk = grads[0][j].cpu().numpy()
                rel[f"d{k}"] = float(np.linalg.norm(gk - acc) / np.linalg.norm(acc))
        out["rel_err_vs_fp64"] = {"f32": {k: float(f"{v:.3e}") for k, v in rel.items()}}
    plan.close()
    print(json.dumps(out), flush=True)


def bench_ragged(args):
    """256 sequences of uneven L and m (BF16): the autotuner's plan for the
    batch (per-stage launches of the fused passes; the cached choice pads
    m <= 64 to 128 so that every class is fused and the state is BF16),
    captured in a HIP graph and replayed; the backward graph likewise, on a
    plan without that padding."""
    import numpy as np
    import torch
    from paper_2411_17729_amd import workloads as W

    wl = W.ragged(seed=args.seed)
    order = sorted(range(len(wl.seqs)), key=lambda i: wl.seqs[i].L)
    fwd_sample = order[::17]  # a spread of lengths and sizes
    bwd_sample = sorted({order[0], order[len(order) // 3], order[2 * len(order) // 3], order[-1]})
    cpu = cpu_bwd = None
    if not args.no_cpu:  # before the GPU is touched (forked workers)
        jobs, gjobs = [], []
        for i in fwd_sample:
            s = wl.seqs[i]
            ps = wl.sets[s.param_set]
            jobs.append((ps.A, ps.B, ps.C, ps.D, s.delta, s.u.astype(np.float32).astype(np.float64)))
        for i in bwd_sample:
            s = wl.seqs[i]
            ps = wl.sets[s.param_set]
            gjobs.append((ps.A, ps.B, ps.C, ps.D, s.delta, s.u.astype(np.float32).astype(np.float64),
                          wl.dy[i].astype(np.float32).astype(np.float64), s.N))
        cpu = cpu_oracle_leg(_oracle_recursion_job, jobs, args.cpu_seconds, _host_workers())
        cpu_bwd = cpu_oracle_leg(_oracle_grads_job, gjobs, 1e9, _host_workers())
    _gpu_init()
    from paper_2411_17729_amd import binding as B
    from paper_2411_17729_amd import cascade as CC
    from paper_2411_17729_amd import tune
    tkey = tune.signature(wl, "bf16", allow_bf16_state=True)
    cached = tkey in tune.load_cache()
    tn = tune.best_tuning(wl, compute="bf16", allow_bf16_state=True)
    # the forward plan as tuned; the backward plan without the extra padding
    # (its passes keep FP32 state and run per stage, so the padded rows would
    # only add work) and with the automatic chain segments (the forward's tuned
    # length is for its few chain launches; short segments re-read a partner
    # block each)
    plan = CC.plan_for_workload(wl, compute="bf16", **tn)
    tb = dict(tn, min_padded_m=0, chain_blocks=0)
    plan_b = CC.plan_for_workload(wl, compute="bf16", with_backward=True, ckpt_every=args.ckpt_every, **tb)
    info = plan.info()
    u = CC.pack_u(wl, dtype=torch.float32)
    dy = torch.as_tensor(np.concatenate([d.reshape(-1) for d in wl.dy]), device="cuda").float()
    y = torch.empty(plan.layout.y_numel, dtype=torch.float32, device="cuda")
    du = torch.empty_like(u)
    gbuf = torch.empty(B.ssm_cascade_param_grad_numel(plan_b.plan), dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    g_fwd = plan.graph_apply(u, y, stream)
    g_bwd = plan_b.graph_backward(u, dy, du, gbuf, stream)
    K, Wm = args.steps, args.warmup
    with torch.cuda.stream(stream):
        ms_f = _timed(lambda: CC.CascadePlan.graph_launch(g_fwd, stream), K, Wm, stream)
        ms_b = _timed(lambda: CC.CascadePlan.graph_launch(g_bwd, stream), max(2, K // 5), 1, stream)
    torch.cuda.synchronize()
    du_h = du.double().cpu().numpy()
    grads = [[t.cpu().numpy() for t in parts] for parts in plan_b.split_param_grads(gbuf)]
    # the stage launches of one eager apply with event timing: the persistent
    # kernel, or the stage, pair and output-fold launches of the per-stage
    # plan (their compulsory bytes together are info["stage_bytes"])
    for kind in (B.TIMING_STAGE, B.TIMING_PAIR, B.TIMING_FOLD):
        plan.timing_read(kind)
    plan.timing(True)
    plan.apply(u, out=y)
    torch.cuda.synchronize()
    plan.timing(False)
    reads = [plan.timing_read(kind) for kind in (B.TIMING_STAGE, B.TIMING_PAIR, B.TIMING_FOLD)]
    n_k = sum(r[0] for r in reads)
    t_k = sum(r[1] for r in reads)
    # one eager backward with event timing: its forward stages (inputs of
    # every stage kept), the adjoint stages and the gradient reductions
    plan_b.timing(True)
    plan_b.backward(u, dy)
    torch.cuda.synchronize()
    plan_b.timing(False)
    b_fwd, b_adj, b_red = (plan_b.timing_read(kind) for kind in (B.TIMING_STAGE, B.TIMING_ADJOINT,
                                                                 B.TIMING_REDUCE))
    # compulsory bytes of the adjoint stages: each reads and writes every
    # adjoint row (FP32, m entries) once per stage the sequence runs
    adj_bytes = sum(8.0 * wl.sets[s.param_set].m * s.L * (min(s.N, (s.L - 1).bit_length() - 1) + 1)
                    for s in wl.seqs if s.L > 1)
    adj_gbps = adj_bytes / (b_adj[1] * 1e-3) / 1e9
    CC.CascadePlan.graph_destroy(g_fwd)
    CC.CascadePlan.graph_destroy(g_bwd)
    gbps = info["stage_bytes"] / (t_k * 1e-3) / 1e9
    ms_list = sorted({wl.sets[s.param_set].m for s in wl.seqs})
    out = {
        "metric": METRIC, "value": round(wl.total_steps / (ms_f * 1e-3), 1), "unit": "output steps/s",
        "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": round(ms_f, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"ragged_{len(wl.seqs)}seq_L{min(s.L for s in wl.seqs)}-{max(s.L for s in wl.seqs)}"
                               f"_m{'-'.join(map(str, ms_list))}_p4_q4",
                   "total_steps": wl.total_steps, "launch": "persistent" if info["launch"] == 2 else "per-stage",
                   "graph": True, "seed": args.seed, "ckpt_every": args.ckpt_every,
                   "workspace_GiB": round(plan._nbytes / 2**30, 2),
                   "backward_workspace_GiB": round(plan_b._nbytes / 2**30, 2)},
        "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                     "frac": round(gbps / PEAK["hbm_GBps"], 4), "traffic": None,
                     "kernel": ("k_persist_res" if info["stage_kernel"] == 3 else "k_persistent")
                               if info["launch"] == 2 else "stage, pair and fold launches of one apply, together",
                     "launches_timed": n_k, "apply_kernel_ms": round(t_k, 5),
                     "algorithmic_bytes_per_apply": round(info["stage_bytes"])},
        "backward": {"value": round(wl.total_steps / (ms_b * 1e-3), 1), "ms_per_step": round(ms_b, 4),
                     "graph": True, "plan": "the forward's tuning with min_padded_m = 0 and automatic chain segments",
                     "breakdown_ms": {"forward_stages": round(b_fwd[1], 3), "adjoint_stages": round(b_adj[1], 3),
                                      "reductions": round(b_red[1], 3),
                                      "launches": [b_fwd[0], b_adj[0], b_red[0]],
                                      "note": "one eager backward with per-launch events; the rest of "
                                              "ms_per_step is FP64 squaring and discretization adjoints, "
                                              "sums, copies and launch gaps"},
                     "roofline": {"bound": "hbm", "achieved": round(adj_gbps, 1), "peak": PEAK["hbm_GBps"],
                                  "unit": "GB/s", "frac": round(adj_gbps / PEAK["hbm_GBps"], 4), "traffic": None,
                                  "kernel": "adjoint stages of one backward, together",
                                  "launches_timed": b_adj[0], "kernel_ms": round(b_adj[1], 4),
                                  "algorithmic_bytes": round(adj_bytes)}},
        "tuning": {"choice": {k: (list(v) if isinstance(v, tuple) else v) for k, v in tn.items()},
                   "cache_key": tkey, "from_cache": cached},
    }
    if cpu is not None:
        yh = CC.unpack_y(wl, y)
        res, t_cpu, workers = cpu
        done = [fwd_sample[j] for j in sorted(res)]
        errs = []
        for j in sorted(res):
            i = fwd_sample[j]
            s = wl.seqs[i]
            ps = wl.sets[s.param_set]
            du_i = s.u.astype(np.float32).astype(np.float64) @ ps.D.T
            st, sr = yh[i] - du_i, res[j] - du_i
            errs.append(float(np.linalg.norm(st - sr) / np.linalg.norm(sr)))
        steps_cpu = sum(wl.seqs[i].L for i in done)
        out["cpu_baseline"] = {"value": round(steps_cpu / t_cpu, 1), "unit": "output steps/s", "cores": workers,
                               "kind": "oracle",
                               "sample": f"{len(done)} of {len(wl.seqs)} sequences in full (every 17th by "
                                         f"length), oracle.trapezoid + oracle.recursion, numpy FP64, one "
                                         f"sequence per worker process with one BLAS thread, {workers} "
                                         f"workers, {t_cpu:.2f} s wall"}
        rel = {"Cx_max": float(f"{max(errs):.3e}")}
        gres, _, _ = cpu_bwd
        uoff = np.cumsum([0] + [s.L * wl.sets[s.param_set].p for s in wl.seqs])
        berr = {}
        for j, i in enumerate(bwd_sample):
            g = gres[j]
            s = wl.seqs[i]
            e = {"du": float(np.linalg.norm(du_h[uoff[i]:uoff[i + 1]] - g["u"].reshape(-1)) /
                             np.linalg.norm(g["u"]))}
            for jj, k in enumerate("ABCD"):
                e[f"d{k}"] = float(np.linalg.norm(grads[s.param_set][jj] - g[k]) / np.linalg.norm(g[k]))
            for k, v in e.items():
                berr[k] = max(berr.get(k, 0.0), v)
        rel["backward_max"] = {k: float(f"{v:.3e}") for k, v in berr.items()}
        out["rel_err_vs_fp64"] = {"bf16": rel}
        out["rel_err_sample"] = f"forward: sequences {done}; backward: sequences {bwd_sample}"
    plan.close()
    plan_b.close()
    print(json.dumps(out), flush=True)




def bench_plr(args):
    """The batched workload (16 x L=16384, m=256 HiPPO, p=q=8, N=13) in FP32 and
    FP64, each applied with dense stages and with partitioned low-rank powers
    (§5) where they halve the matrix-core steps: apply times (HIP graph
    replays), the PLR stage launches' roofline (compulsory bytes: a read of the
    stage input rows, of their partners and a write, per launch), the ranks
    behind them, and the error of both against the FP64 oracle on two sampled
    sequences."""
    import numpy as np
    import torch
    from paper_2411_17729_amd import binding as B
    from paper_2411_17729_amd import cascade as CC
    from paper_2411_17729_amd import workloads as W
    wl = W.batched(seed=args.seed)
    sample = [0, len(wl.seqs) - 1]
    refs = None
    if not args.no_cpu:
        ps0 = wl.sets[0]
        jobs = [(ps0.A, ps0.B, ps0.C, ps0.D, wl.seqs[i].delta, wl.seqs[i].u) for i in sample]
        res, _, _ = cpu_oracle_leg(_oracle_recursion_job, jobs, 1e9, len(jobs))
        refs = [res[j] for j in range(len(jobs))]
    _gpu_init()
    s0, ps = wl.seqs[0], wl.sets[0]
    wname = f"hippo_m{ps.m}_p{ps.p}_q{ps.q}_B{len(wl.seqs)}_L{s0.L}_N{s0.N}"
    K, Wm = args.steps, args.warmup
    out = {"metric": METRIC, "unit": "output steps/s", "n_gpus": 1, "steps": K, "warmup": Wm,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
           "config": {"workload": wname + "_plr", "sequences": len(wl.seqs), "L": s0.L, "m": ps.m,
                      "p": ps.p, "q": ps.q, "N": s0.N, "seed": args.seed}}
    legs = {}
    for dt, digits in (("f32", 7), ("f64", 12)):
        tdt = torch.float64 if dt == "f64" else torch.float32
        u = CC.pack_u(wl, dtype=tdt)
        steps = K if dt == "f32" else max(2, K // 5)
        leg = {"plr_digits": digits}
        ys = {}
        for name, dg in (("dense", 0), ("plr", digits)):
            plan = CC.plan_for_workload(wl, compute=dt, plr_digits=dg)
            y = torch.empty(plan.layout.y_numel, dtype=tdt, device="cuda")
            stream = torch.cuda.Stream()
            torch.cuda.synchronize()
            g = plan.graph_apply(u, y, stream)
            ms = _timed(lambda: CC.CascadePlan.graph_launch(g, stream), steps, Wm, stream)
            CC.CascadePlan.graph_destroy(g)
            info = plan.info()
            ent = {"ms_per_step": round(ms, 4), "value": round(wl.total_steps / (ms * 1e-3), 1)}
            if dg:
                plan.timing_read(B.TIMING_PLR)
                plan.timing(True)
                for _ in range(min(steps, 10)):
                    plan.apply(u, out=y)
                torch.cuda.synchronize()
                plan.timing(False)
                n_l, k_ms = plan.timing_read(B.TIMING_PLR)
                used = [k for k in range(s0.N + 1) if plan.plr_ranks(0, k)[1]]
                ent["plr_stages"] = used
                ent["ranks_op0"] = {k: max(plan.plr_ranks(0, k)[0]) for k in used}
                if n_l > 0:
                    per_apply = n_l / min(steps, 10)
                    avg = k_ms / n_l
                    rows = sum(max(0, s.L - (1 << k)) for s in wl.seqs for k in used)
                    es = 8 if dt == "f64" else 4
                    nbytes = sum(s.L for s in wl.seqs) * ps.m * es * 3 * len(used) / per_apply
                    gbps = nbytes / (avg * 1e-3) / 1e9
                    flops = info["plr_flops"] / per_apply
                    peak_tf = PEAK["f64_TFLOPs"] if dt == "f64" else PEAK["f32_TFLOPs"]
                    tf = flops / (avg * 1e-3) / 1e12
                    ent["roofline"] = {
                        "bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK["hbm_GBps"], "unit": "GB/s",
                        "frac": round(gbps / PEAK["hbm_GBps"], 4), "traffic": None, "kernel": "k_stage_plr",
                        "launches_timed": n_l, "avg_launch_ms": round(avg, 5),
                        "algorithmic_bytes_per_launch": round(nbytes),
                        "plr_flops_per_launch": round(flops), "plr_TFLOPs": round(tf, 2),
                        "plr_flops_frac_of_peak": round(tf / peak_tf, 4),
                        "dense_flops_of_the_same_rows": round(info["plr_dense_flops"] / per_apply),
                        "rows_per_apply": rows}
            ys[name] = CC.unpack_y(wl, y)
            leg[name] = ent
            plan.close()
        leg["speedup_plr_vs_dense"] = round(leg["dense"]["ms_per_step"] / leg["plr"]["ms_per_step"], 3)
        if refs is not None:
            leg["rel_err_vs_fp64"] = {
                name: float(f"{max(float(np.linalg.norm(yy[i] - r) / np.linalg.norm(r)) for i, r in zip(sample, refs)):.3e}")
                for name, yy in ys.items()}
        legs[dt] = leg
    out["dtype"] = "f32"
    out["value"] = legs["f32"]["plr"]["value"]
    out["ms_per_step"] = legs["f32"]["plr"]["ms_per_step"]
    out["roofline"] = legs["f32"]["plr"].get("roofline")
    out["legs"] = legs
    out["rel_err_sample"] = f"sequences {sample}, oracle.trapezoid + oracle.recursion (FP64)"
    _copy_probe(args, out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
