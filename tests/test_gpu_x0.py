"""Forward apply from a nonzero initial state x_{-1} (ssm_cascade_apply_x0)
against the FP64 oracle: the recursion from x0 where the cascade's window
covers the sequence, the truncated sum with the free response cut at
T = 2^(N+1) lags where it does not; BF16 plans with the input pass, stage
pairs and the six-stage output fold, FP32 and FP64 plans, ragged lengths and
sizes, and the error paths."""

import math

import numpy as np
import pytest
import torch

from oracle import ssm_oracle as O
from paper_2411_17729_amd import binding as B
from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err

pytestmark = pytest.mark.gpu


def _workload(seed, spec, zero_d=False):
    rng = np.random.default_rng(seed)
    sets, seqs = [], []
    for i, (m, p, q, L, N) in enumerate(spec):
        A, _ = W.hippo_legs(m)
        D = np.zeros((q, p)) if zero_d else rng.standard_normal((q, p)) / math.sqrt(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m), D))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    x0 = [rng.standard_normal(m) for (m, *_r) in spec]
    return W.Workload("x0", sets, seqs), x0


def _oracle(wl, x0, f64_u=False):
    out = []
    for s, x in zip(wl.seqs, x0):
        ps = wl.sets[s.param_set]
        Abar, Bbar = O.trapezoid(ps.A, ps.B, s.delta)
        u = s.u if f64_u else s.u.astype(np.float32).astype(np.float64)
        if (1 << (s.N + 1)) >= s.L:
            y, _ = O.recursion(Abar, Bbar, ps.C, ps.D, u, x0=x)
        else:
            y = O.truncated_sum(Abar, Bbar, ps.C, ps.D, u, s.N, x0=x)
        out.append(y)
    return out


def _run(wl, x0, compute, **kw):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute=compute, launch="per_stage", **kw)
    info = plan.info()
    dt = torch.float64 if compute == "f64" else torch.float32
    u = CC.pack_u(wl, dtype=dt)
    xt = torch.from_numpy(np.concatenate(x0)).to(dt).cuda()
    y = CC.unpack_y(wl, plan.apply(u, x0=xt))
    y_zero = CC.unpack_y(wl, plan.apply(u))
    torch.cuda.synchronize()
    plan.close()
    return y, y_zero, info


# (m, p, q, L, N): padded m 256 with the six-stage fold, m below its padded
# size, padded m 128, and a sequence longer than its window (L > 2^(N+1))
SPEC_BF16 = [(256, 8, 8, 3000, 11), (200, 8, 4, 2500, 11), (128, 4, 3, 1500, 10), (128, 4, 4, 1800, 9)]


@pytest.mark.parametrize("zero_d", [True, False])
def test_x0_bf16_plan(zero_d):
    wl, x0 = _workload(81, SPEC_BF16, zero_d=zero_d)
    y, y_zero, info = _run(wl, x0, "bf16")
    print("input stages", info["input_stages"], "fold", info["fold_stages"], "pairs", info["pair_launches"],
          flush=True)
    ref = _oracle(wl, x0)
    ref_zero = _oracle(wl, [np.zeros_like(x) for x in x0])
    for i in range(len(wl.seqs)):
        e = parity_err(y[i], ref[i])
        # the part x0 adds, on its own (the free response)
        ef = parity_err(np.asarray(y[i]) - np.asarray(y_zero[i]), ref[i] - ref_zero[i])
        print("seq", i, f"y {e:.2e} free response {ef:.2e}", flush=True)
        assert e <= 2e-2 and ef <= 2e-2, (i, e, ef)


def test_x0_f32_plan():
    spec = [(64, 2, 2, 1000, 9), (100, 3, 2, 1500, 9), (256, 4, 4, 700, 9)]
    wl, x0 = _workload(82, spec, zero_d=True)
    y, y_zero, info = _run(wl, x0, "f32")
    ref = _oracle(wl, x0)
    ref_zero = _oracle(wl, [np.zeros_like(x) for x in x0])
    for i in range(len(wl.seqs)):
        e = parity_err(y[i], ref[i])
        ef = parity_err(np.asarray(y[i]) - np.asarray(y_zero[i]), ref[i] - ref_zero[i])
        print("seq", i, f"y {e:.2e} free response {ef:.2e}", flush=True)
        assert e <= 1e-5 and ef <= 1e-5, (i, e, ef)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_x0_input_pass_runs_every_stage(compute):
    # sequences whose input pass folds every stage it runs and forms y itself
    # (kry = last + 1): short chunks at m = 64, p = 1 (2^6 p <= 64), a short
    # chunk at padded m 256 with p = 4, and a small N at a length far past the
    # window (N = 4: 2^5 = 32 lags, L = 1000); the free response must reach y
    # through the output map, since no stage runs after the input pass
    spec = [(64, 1, 1, 40, 11), (64, 1, 2, 64, 11), (256, 4, 4, 30, 11), (64, 1, 1, 1000, 4),
            (60, 1, 3, 17, 3)]
    wl, x0 = _workload(86, spec, zero_d=(compute == "f32"))
    y, y_zero, info = _run(wl, x0, compute)
    print("input stages", info["input_stages"], flush=True)
    assert info["input_stages"] >= 5
    ref = _oracle(wl, x0)
    ref_zero = _oracle(wl, [np.zeros_like(x) for x in x0])
    tol = 1e-5 if compute == "f32" else 2e-2
    for i in range(len(wl.seqs)):
        e = parity_err(y[i], ref[i])
        ef = parity_err(np.asarray(y[i]) - np.asarray(y_zero[i]), ref[i] - ref_zero[i])
        print("seq", i, f"y {e:.2e} free response {ef:.2e}", flush=True)
        assert e <= tol and ef <= tol, (i, e, ef)


def test_x0_f64_plan():
    spec = [(64, 1, 1, 512, 8), (48, 2, 1, 600, 8)]
    wl, x0 = _workload(83, spec)
    y, _, _ = _run(wl, x0, "f64")
    ref = _oracle(wl, x0, f64_u=True)
    for i in range(len(wl.seqs)):
        e = parity_err(y[i], ref[i])
        print("seq", i, f"y {e:.2e}", flush=True)
        assert e <= 1e-11, (i, e)


def test_x0_errors():
    from paper_2411_17729_amd import cascade as CC
    wl, x0 = _workload(84, [(64, 2, 2, 300, 8)])
    u = CC.pack_u(wl, dtype=torch.float32)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage")
    with pytest.raises(B.SSMError) as ei:  # one entry short
        B.ssm_cascade_apply_x0(plan.plan, u.data_ptr(), B.SSM_F32, u.numel(), u.data_ptr(), 63,
                               u.data_ptr(), u.numel(), None)
    assert ei.value.status == B.SSM_E_INVALID
    plan.close()
    plan = CC.plan_for_workload(wl, compute="bf16", launch="persistent")
    xt = torch.zeros(64, dtype=torch.float32, device="cuda")
    with pytest.raises(B.SSMError) as ei:
        plan.apply(u, x0=xt)
    assert ei.value.status == B.SSM_E_UNSUPPORTED
    plan.close()
    torch.cuda.synchronize()


def test_x0_bf16_state_rejected():
    from paper_2411_17729_amd import cascade as CC
    wl, x0 = _workload(85, [(256, 8, 8, 3000, 11)])
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", state_bf16=1)
    if plan.info()["state_dtype"] != B.SSM_BF16:
        plan.close()
        pytest.skip("the plan keeps an FP32 state")
    u = CC.pack_u(wl, dtype=torch.float32)
    xt = torch.zeros(256, dtype=torch.float32, device="cuda")
    with pytest.raises(B.SSMError) as ei:
        plan.apply(u, x0=xt)
    assert ei.value.status == B.SSM_E_UNSUPPORTED
    plan.close()
    torch.cuda.synchronize()
