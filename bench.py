#!/usr/bin/env python
"""Throughput of the fast cascade on one MI355X.

Workload: 16 sequences x L = 16384 of one shared HiPPO-LegS model (m = 256,
p = q = 8, B, C, D ~ N(0, 1/m)), one step size per sequence (log-uniform in
[1e-3, 1e-1]), N = 13 (degree 16383), u ~ N(0, 1), all seeded and synthetic.

A step is one full forward pass over the batch: all N+1 stage launches with
the fused Bbar u input and C x + D u output, inputs already in HBM. The
headline is the cascade with BF16 MFMA operands (FP32 accumulation, FP32
state); the FP32-MFMA cascade and the plain FP32 recursion on the same GPU
are measured beside it, each with its relative error against the FP64
oracle on a sample of sequences. Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype bf16|f32]
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
# stage kernel of each ssm_stage_kernel value: (name, source file)
STAGE_KERNELS = {1: ("k_stage", "kernels_stage.hip"), 2: ("k_stage_res", "kernels_stage_res.hip"),
                 3: ("k_stage_chain", "kernels_stage_chain.hip")}


def _args():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--dtype", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the other dtype and the recursion comparator")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU oracle sample")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the measurement, run one device-to-device copy of this many MiB "
                         "(a reference for hardware byte counters)")
    return ap.parse_args()


def _stage_traffic(workload, dtype, kernel):
    """HBM bytes per stage launch from committed rocprofv3 counter runs, if
    they were taken on the current source of this stage kernel."""
    name, src = STAGE_KERNELS[kernel]
    path = os.path.join(ROOT, "profiles", f"stage_traffic_{workload}_{dtype}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2411_17729_amd", "csrc", src), "rb")
                         .read()).hexdigest()
    if rec.get("kernel") != name or rec.get("kernel_sha256") != sha:
        return None
    return rec.get("traffic_bytes_per_launch")


def main():
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_17729_amd import binding as B
    from paper_2411_17729_amd import cascade as CC
    from paper_2411_17729_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    B.load()

    wl = W.batched(seed=args.seed)
    s0 = wl.seqs[0]
    ps = wl.sets[0]
    wname = f"hippo_m{ps.m}_p{ps.p}_q{ps.q}_B{len(wl.seqs)}_L{s0.L}_N{s0.N}"
    total_steps = wl.total_steps
    u32 = CC.pack_u(wl, dtype=torch.float32)
    K, Wm = args.steps, args.warmup

    def run(plan, fn_name, steps, warm, timing_kind=None):
        fn = getattr(plan, fn_name)
        y = torch.empty(plan.layout.y_numel, dtype=plan.state_dtype, device="cuda")
        for _ in range(warm):
            fn(u32, out=y)
        torch.cuda.synchronize()
        if timing_kind is not None:
            plan.timing_read(timing_kind)  # clear warm-up records
            plan.timing(True)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(steps):
            fn(u32, out=y)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        kern = None
        if timing_kind is not None:
            plan.timing(False)
            kern = plan.timing_read(timing_kind)
        return y, ms / steps, kern

    def roofline(plan, kern, dtype, steps):
        info = plan.info()
        n_launch, k_ms = kern
        avg_ms = k_ms / max(n_launch, 1)
        per_launch_bytes = info["stage_bytes"] / info["stage_launches"]
        per_launch_flops = info["stage_flops"] / info["stage_launches"]
        gbps = per_launch_bytes / (avg_ms * 1e-3) / 1e9
        tflops = per_launch_flops / (avg_ms * 1e-3) / 1e12
        peak_tf = PEAK["bf16_TFLOPs"] if dtype == "bf16" else PEAK["f32_TFLOPs"]
        intensity = info["stage_flops"] / info["stage_bytes"]
        ridge = peak_tf * 1e12 / (PEAK["hbm_GBps"] * 1e9)
        bound = "mfma" if intensity > ridge else "hbm"
        kid = info["stage_kernel"]
        if kid == 3 and dtype == "f32" and ps.m > 128:
            kid = 2  # FP32 m > 128: the chain walk does not apply, the resident kernel runs
        traffic = _stage_traffic(wname, dtype, kid)
        if bound == "hbm":
            rf = {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK["hbm_GBps"],
                  "unit": "GB/s", "frac": round(gbps / PEAK["hbm_GBps"], 4)}
        else:
            rf = {"bound": "mfma", "achieved": round(tflops, 2), "peak": peak_tf,
                  "unit": "TFLOP/s", "frac": round(tflops / peak_tf, 4)}
        rf["traffic"] = traffic
        rf.update({"kernel": STAGE_KERNELS[kid][0], "launches_timed": n_launch, "avg_launch_ms": round(avg_ms, 5),
                   "algorithmic_bytes_per_launch": round(per_launch_bytes),
                   "algorithmic_flops_per_launch": round(per_launch_flops),
                   "mfma_util": round(tflops / peak_tf, 4), "hbm_GBps": round(gbps, 1)})
        return rf

    # ---------------- headline: the cascade in the chosen dtype ----------------
    plan = CC.plan_for_workload(wl, compute=args.dtype)
    y_main, ms_main, kern = run(plan, "apply", K, Wm, timing_kind=B.TIMING_STAGE)
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
    }
    ys = {args.dtype: CC.unpack_y(wl, y_main)}

    # ---------------- comparators on the same GPU ----------------
    if not args.no_compare:
        other = "f32" if args.dtype == "bf16" else "bf16"
        plan_o = CC.plan_for_workload(wl, compute=other)
        y_o, ms_o, kern_o = run(plan_o, "apply", K, Wm, timing_kind=B.TIMING_STAGE)
        ys[other] = CC.unpack_y(wl, y_o)
        out[f"cascade_{other}"] = {"value": round(total_steps / (ms_o * 1e-3), 1),
                                    "ms_per_step": round(ms_o, 4),
                                    "roofline": roofline(plan_o, kern_o, other, K)}
        plan_r = plan_o if other == "f32" else plan
        rsteps = max(2, K // 10)
        y_r, ms_r, _ = run(plan_r, "recursion", rsteps, 1)
        ys["recursion_f32"] = CC.unpack_y(wl, y_r)
        out["recursion_f32"] = {"value": round(total_steps / (ms_r * 1e-3), 1),
                                "ms_per_step": round(ms_r, 4), "steps": rsteps}
        out["speedup_vs_recursion"] = round(ms_r / ms_main, 2)

    # ---------------- CPU oracle: baseline timing and FP64 reference ----------------
    if not args.no_cpu:
        import oracle as O
        from threadpoolctl import threadpool_limits

        t_start = time.perf_counter()
        done = []
        refs = {}
        with threadpool_limits(limits=1):
            for i, s in enumerate(wl.seqs):
                Abar, Bbar = O.trapezoid(ps.A, ps.B, s.delta)
                yref, _ = O.recursion(Abar, Bbar, ps.C, ps.D, s.u.astype(np.float32).astype(np.float64))
                refs[i] = yref
                done.append(i)
                if time.perf_counter() - t_start >= args.cpu_seconds:
                    break
        t_cpu = time.perf_counter() - t_start
        steps_cpu = sum(wl.seqs[i].L for i in done)
        out["cpu_baseline"] = {
            "value": round(steps_cpu / t_cpu, 1), "unit": "output steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{len(done)} of {len(wl.seqs)} sequences in full (L={s0.L}), "
                      f"oracle.trapezoid + oracle.recursion, numpy FP64, 1 BLAS thread, {t_cpu:.1f} s"}
        rel = {}
        for name, yl in ys.items():
            ey = max(float(np.linalg.norm(yl[i] - refs[i]) / np.linalg.norm(refs[i])) for i in done)
            du = {i: wl.seqs[i].u.astype(np.float32).astype(np.float64) @ ps.D.T for i in done}
            ex = max(float(np.linalg.norm((yl[i] - du[i]) - (refs[i] - du[i])) /
                           np.linalg.norm(refs[i] - du[i])) for i in done)
            rel[name] = {"y": ey, "state": ex}
        out["rel_err_vs_fp64"] = {k: {kk: float(f"{vv:.3e}") for kk, vv in v.items()} for k, v in rel.items()}
        out["rel_err_sample"] = f"sequences {done}"

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = n * 4

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
