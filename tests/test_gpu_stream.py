"""A stream applied in chunks.

* Carried state (ssm_cascade_apply_state): each chunk starts from the state
  of the previous chunk's last row. With chunks of at most 2^(N+1) rows the
  cascade of a chunk is the recursion of eq. (1.2) from that state, so the
  chained outputs and the last state equal the FP64 recursion over the whole
  stream (checked in FP64, FP32 and BF16, ragged chunk lengths, several
  sequences of different sizes at once, and a chunk finished by the input
  pass alone). The recursion's growth is carried along too: on the stability
  operator (one eigenvalue 1 + 1e-5) the chained stream follows the
  recursion, not the truncated sum.
* Truncated operator H_N (the FIR of eq. (2.2)): a stream of 2^22 rows on the
  stability operator is applied in 64 chunks, each prefixed with the previous
  2^(N+1) - 1 inputs (no carried state), and equals the one-shot apply and
  the FP64 truncated sum; it stays under the FIR bound."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import binding as B
from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-2}


def _chunk_workload(sets, chunks, N, given=False):
    """One sequence per parameter set, each with its chunk of u."""
    seqs = [W.Sequence(i, d, int(u.shape[0]), N, u) for i, (d, u) in enumerate(chunks)]
    return W.Workload("chunk", sets, seqs, given=given)


def _stream(sets, deltas, us, bounds, N, compute, given=False):
    """Applies every stream chunk by chunk ([b0, b1) row ranges), carrying the
    states; returns per-sequence outputs and last states (FP64 numpy)."""
    from paper_2411_17729_amd import cascade as CC
    dt = torch.float64 if compute == "f64" else torch.float32
    ys = [[] for _ in sets]
    x = None
    for b0, b1 in bounds:
        wl = _chunk_workload(sets, [(d, u[b0:b1]) for d, u in zip(deltas, us)], N, given)
        plan = CC.plan_for_workload(wl, compute=compute, final_state=1)
        u_t = CC.pack_u(wl, dtype=dt)
        y, x = plan.apply_state(u_t, x0=x)
        for i, yi in enumerate(CC.unpack_y(wl, y)):
            ys[i].append(yi)
        x = x.clone()
        plan.close()
    torch.cuda.synchronize()
    xs = x.double().cpu().numpy()
    out_x, off = [], 0
    for ps in sets:
        out_x.append(xs[off: off + ps.m])
        off += ps.m
    return [np.concatenate(y) for y in ys], out_x


def _hippo_set(rng, m, p, q):
    A, b = W.hippo_legs(m)
    Bm = rng.standard_normal((m, p)) / np.sqrt(m)
    Bm[:, 0] = b / np.sqrt(m)
    return W.ParamSet(A, Bm, rng.standard_normal((q, m)) / np.sqrt(m), rng.standard_normal((q, p)))


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_chained_chunks_equal_the_recursion(compute):
    rng = np.random.default_rng(41)
    # padded sizes 32, 128 and 256; ragged chunk lengths up to 2^(N+1) = 2048
    sets = [_hippo_set(rng, 20, 2, 3), _hippo_set(rng, 100, 4, 2), _hippo_set(rng, 256, 8, 8)]
    deltas = [2e-2, 5e-3, 1e-2]
    total = 6000
    us = [rng.standard_normal((total, ps.p)) for ps in sets]
    if compute != "f64":
        us = [u.astype(np.float32).astype(np.float64) for u in us]
    cuts = [0, 1000, 2048, 2560, 4560, 6000]
    bounds = list(zip(cuts[:-1], cuts[1:]))
    ys, xl = _stream(sets, deltas, us, bounds, N=10, compute=compute)
    worst_y = worst_x = 0.0
    for ps, d, u, y, x in zip(sets, deltas, us, ys, xl):
        Abar, Bbar = O.trapezoid(ps.A, ps.B, d)
        ref, states = O.recursion(Abar, Bbar, ps.C, ps.D, u)
        worst_y = max(worst_y, parity_err(y, ref))
        worst_x = max(worst_x, float(np.linalg.norm(x - states[-1]) / np.linalg.norm(states[-1])))
    print(f"{compute}: chained y rel err {worst_y:.2e}, last state {worst_x:.2e}", flush=True)
    assert worst_y <= TOL[compute] and worst_x <= TOL[compute]


def test_chained_chunk_finished_by_the_input_pass():
    # chunks of 3 rows at m = 64, p = 1: the input pass (lags below 2^j) runs
    # every stage of a chunk and forms y, and must keep the state as well
    rng = np.random.default_rng(42)
    sets = [_hippo_set(rng, 64, 1, 1)]
    u = rng.standard_normal((30, 1)).astype(np.float32).astype(np.float64)
    bounds = [(i, i + 3) for i in range(0, 30, 3)]
    from paper_2411_17729_amd import cascade as CC
    wl = _chunk_workload(sets, [(1e-2, u[:3])], N=1)
    plan = CC.plan_for_workload(wl, compute="f32", final_state=1)
    assert plan.info()["input_stages"] >= 2  # the input pass holds both stages
    plan.close()
    ys, xl = _stream(sets, [1e-2], [u], bounds, N=1, compute="f32")
    Abar, Bbar = O.trapezoid(sets[0].A, sets[0].B, 1e-2)
    ref, states = O.recursion(Abar, Bbar, sets[0].C, sets[0].D, u)
    assert parity_err(ys[0], ref) <= 1e-5
    assert np.linalg.norm(xl[0] - states[-1]) <= 1e-5 * np.linalg.norm(states[-1])


def test_chained_stream_follows_the_recursion_on_the_stability_operator():
    # the carried state continues eq. (1.2) itself: 16 chunks of 4096 rows
    # (N = 11, a window of 4096) equal the recursion over 65536 rows, which
    # differs from the truncated sum of the same window
    wl = W.stability(seed=1, batch=1, m=128, L=1 << 16, N=11)
    ps = wl.sets[0]
    u = wl.seqs[0].u.astype(np.float32).astype(np.float64)
    bounds = [(i, i + 4096) for i in range(0, 1 << 16, 4096)]
    ys, xl = _stream([ps], [1.0], [u], bounds, N=11, compute="f32", given=True)
    ref, states = O.recursion(ps.A, ps.B, ps.C, ps.D, u)
    fir = O.truncated_sum_fft(ps.A, ps.B, ps.C, ps.D, u, 11)
    e = parity_err(ys[0], ref)
    e_fir = parity_err(fir, ref)
    print(f"chained vs recursion {e:.2e}; the truncated sum is {e_fir:.2e} away", flush=True)
    assert e <= 1e-5 and e_fir > 1e3 * e
    assert np.linalg.norm(xl[0] - states[-1]) <= 1e-5 * np.linalg.norm(states[-1])


def test_fir_stream_of_64_chunks_L4M():
    # H_N streamed without carried state: chunk k is rows [kC, (k + 1) C)
    # applied with the previous T - 1 rows in front (C = T = 2^16, N = 15)
    from paper_2411_17729_amd import cascade as CC
    wl = W.stability(seed=0, batch=2, L=1 << 22, N=15)
    ps = wl.sets[0]
    T = 1 << 16
    Cn = T
    us = [s.u.astype(np.float32).astype(np.float64) for s in wl.seqs]
    # one-shot apply for comparison
    plan = CC.plan_for_workload(wl, compute="f32")
    one = CC.unpack_y(wl, plan.apply(CC.pack_u(wl, dtype=torch.float32)))
    plan.close()
    plans = {}
    outs = [[] for _ in us]
    for k in range((1 << 22) // Cn):
        b0 = max(0, k * Cn - (T - 1))
        b1 = (k + 1) * Cn
        cw = W.Workload("fir_chunk", wl.sets, [W.Sequence(0, 1.0, b1 - b0, 15, u[b0:b1]) for u in us], given=True)
        if b1 - b0 not in plans:
            plans[b1 - b0] = CC.plan_for_workload(cw, compute="f32")
        y = CC.unpack_y(cw, plans[b1 - b0].apply(CC.pack_u(cw, dtype=torch.float32)))
        for i in range(len(us)):
            outs[i].append(y[i][-Cn:])
    torch.cuda.synchronize()
    for p_ in plans.values():
        p_.close()
    h = O.impulse_response(ps.A, ps.B, ps.C, T)[:, 0, 0]
    fir_bound = float(np.sum(np.abs(h)) + abs(ps.D[0, 0]))
    for u, o, y1 in zip(us, outs, one):
        ys = np.concatenate(o)
        ref = O.truncated_sum_fft(ps.A, ps.B, ps.C, ps.D, u, 15)
        Du = u @ ps.D.T
        e = parity_err(ys - Du, ref - Du)
        e1 = parity_err(ys, y1)
        print(f"64 chunks: state part rel err {e:.2e} vs FP64, {e1:.2e} vs one shot", flush=True)
        assert e <= 1e-5 and e1 <= 1e-5
        assert np.max(np.abs(ys)) <= fir_bound * float(np.max(np.abs(u)))


def test_apply_state_errors():
    from paper_2411_17729_amd import cascade as CC
    rng = np.random.default_rng(43)
    sets = [_hippo_set(rng, 64, 1, 1)]
    wl = _chunk_workload(sets, [(1e-2, rng.standard_normal((100, 1)))], N=6)
    u = CC.pack_u(wl, dtype=torch.float32)
    plain = CC.plan_for_workload(wl, compute="f32")
    with pytest.raises(B.SSMError) as ei:  # the plan does not keep final states
        plain.apply_state(u)
    assert ei.value.status == B.SSM_E_NOT_PREPARED
    y, _ = CC.plan_for_workload(wl, compute="f32", final_state=1).apply_state(u)
    with pytest.raises(B.SSMError) as ei:  # wrong x_last size
        CC.plan_for_workload(wl, compute="f32", final_state=1).apply_state(
            u, x_last=torch.empty(63, device="cuda"))
    assert ei.value.status == B.SSM_E_INVALID
    # without x_last it is the apply from x0 (here zero): same y as the plain plan
    fs = CC.plan_for_workload(wl, compute="f32", final_state=1)
    yp = plain.apply(u)
    ya = torch.empty_like(yp)
    B.ssm_cascade_apply_state(fs.plan, u.data_ptr(), B.SSM_F32, u.numel(), None, 0, ya.data_ptr(), ya.numel(),
                              None, 0, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.allclose(ya, yp, rtol=1e-6, atol=1e-6)
    # a persistent plan cannot keep final states
    with pytest.raises(B.SSMError):
        CC.plan_for_workload(wl, compute="f32", final_state=1, launch="persistent")
