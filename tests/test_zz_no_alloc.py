"""The allocation-free apply (ssm_cascade_apply_noalloc) through the C ABI.

It runs the same kernels as ssm_cascade_apply with the two state buffers
taken from the library's static device scratch, so its y must equal
ssm_cascade_apply's bit for bit. Two calls in a row, the second on a smaller
input, check that the scratch left behind by one call does not leak into the
next; the first is also held to the oracle's BF16 bound."""

import numpy as np
import pytest
import torch

from paper_2411_17729_amd import binding as B
from paper_2411_17729_amd import workloads as W
from tests.helpers import max_rel, oracle_outputs, state_part

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _same(a, b):
    return torch.equal(a.view(torch.int32), b.view(torch.int32)) if a.dtype == torch.float32 else \
        torch.equal(a.view(torch.int64), b.view(torch.int64))


def _noalloc(plan, u, y):
    B.ssm_cascade_apply_noalloc(plan.plan, u.data_ptr(), plan._u_code(u), u.numel(), y.data_ptr(), y.numel(),
                                torch.cuda.current_stream().cuda_stream)


def _pair(wl, compute, **kw):
    from paper_2411_17729_amd import cascade as CC
    ref = CC.plan_for_workload(wl, compute=compute, **kw)
    sta = CC.plan_for_workload(wl, compute=compute, static_state=1, **kw)
    return ref, sta


def test_noalloc_matches_apply_two_calls_second_smaller():
    from paper_2411_17729_amd import cascade as CC
    # call 1: the bench plan on two sequences (BF16 state, split input pass,
    # a stage pair, the six-stage output fold): 2 x 23.4 MiB of state
    wl1 = W.batched(seed=3, batch=2, m=256, L=12000, N=13, p=8, q=8)
    ref1, sta1 = _pair(wl1, "bf16", state_bf16=1)
    info = sta1.info()
    assert info["state_dtype"] == B.SSM_BF16 and info["fold_stages"] == 6 and info["pair_launches"] >= 1
    assert ref1._nbytes - sta1._nbytes >= 2 * 2 * 12000 * 256 * 4
    u1 = CC.pack_u(wl1, dtype=torch.float32)
    want1 = ref1.apply(u1)
    got1 = torch.full_like(want1, float("nan"))
    _noalloc(sta1, u1, got1)
    got1b = torch.full_like(want1, float("nan"))
    _noalloc(ref1, u1, got1b)  # an ordinary plan through the same entry point
    # call 2: smaller, another class and type (m = 100 padded to 128, FP32)
    wl2 = W.batched(seed=4, batch=1, m=100, L=1000, N=9, p=2, q=3)
    ref2, sta2 = _pair(wl2, "f32")
    u2 = CC.pack_u(wl2, dtype=torch.float32)
    want2 = ref2.apply(u2)
    got2 = torch.full_like(want2, float("nan"))
    _noalloc(sta2, u2, got2)
    torch.cuda.synchronize()
    print("noalloc call 1 (m=256 bf16, 2 x 12000) and call 2 (m=100 f32, 1000)", flush=True)
    assert _same(got1, want1) and _same(got1b, want1)
    assert _same(got2, want2)
    # and the first call against the oracle (BF16 bound on y and its state part)
    uq = [s.u.astype(np.float32).astype(np.float64) for s in wl1.seqs]
    ref = oracle_outputs(wl1, u_override=uq)
    got = CC.unpack_y(wl1, got1)
    assert max_rel(got, ref) <= 2e-2
    assert max_rel(state_part(wl1, got, uq), state_part(wl1, ref, uq)) <= 2e-2
    for p in (ref1, sta1, ref2, sta2):
        p.close()


def test_noalloc_fp64_plan():
    from paper_2411_17729_amd import cascade as CC
    wl = W.plain_fp64(seed=5, L=2048, N=10)
    ref, sta = _pair(wl, "f64")
    u = CC.pack_u(wl, dtype=torch.float64)
    want = ref.apply(u)
    got = torch.full_like(want, float("nan"))
    _noalloc(sta, u, got)
    torch.cuda.synchronize()
    assert _same(got, want)
    ref.close()
    sta.close()


def test_noalloc_limits_and_refusals():
    from paper_2411_17729_amd import cascade as CC
    # 2 x (65536 x 256 x 4 bytes) = 128 MiB of state: beyond the 64 MiB scratch
    wl = W.batched(seed=6, batch=1, m=256, L=65536, N=15, p=1, q=1)
    sta = CC.plan_for_workload(wl, compute="bf16", static_state=1)
    u = CC.pack_u(wl, dtype=torch.float32)
    y = torch.zeros(sta.layout.y_numel, dtype=torch.float32, device="cuda")
    with pytest.raises(B.SSMError) as ei:
        _noalloc(sta, u, y)
    assert ei.value.status == B.SSM_E_WORKSPACE and "static scratch" in str(ei.value)
    # a static_state plan has no state buffers for the other entry points
    with pytest.raises(B.SSMError) as ei:
        sta.apply(u, out=y)
    assert ei.value.status == B.SSM_E_NOT_PREPARED
    with pytest.raises(B.SSMError) as ei:
        sta.recursion(u, out=y)
    assert ei.value.status == B.SSM_E_NOT_PREPARED
    sta.close()
    # the backward keeps its state buffers in the workspace (sizing the
    # workspace already refuses)
    with pytest.raises(B.SSMError) as ei:
        CC.plan_for_workload(W.backward(seed=0, batch=1, L=512, N=8), compute="f32", with_backward=True,
                             static_state=1)
    assert "static_state" in str(ei.value)
    # the largest plan that fits: 2 x 32 MiB exactly
    wl = W.batched(seed=7, batch=1, m=256, L=32768, N=14, p=1, q=1)
    ref, sta = _pair(wl, "bf16")
    u = CC.pack_u(wl, dtype=torch.float32)
    want = ref.apply(u)
    got = torch.full_like(want, float("nan"))
    _noalloc(sta, u, got)
    torch.cuda.synchronize()
    assert 2 * 32768 * 256 * 4 == SCRATCH_BYTES
    assert _same(got, want)
    ref.close()
    sta.close()
