"""Stability workload: a structured diagonal-plus-rank-2 Abar (m = 128) whose
eigenvalues lie in [0.99, 0.99999] except one at 1 + 1e-5.

* L = 65536 = 2^(N+1), N = 15: the cascade and the recursion are the same
  map; the FP32 cascade stays within 1e-5 of the FP64 truncated sum, and the
  FP32 recursion's error is reported next to it (it is larger).
* L = 2^22 with the same N (the window covers 65536 lags): the cascade is the
  bounded degree-65535 FIR and stays within 1e-5 of the FP64 truncated sum,
  while the plain recursion grows by (1 + 1e-5)^L ~ 1e18."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err

pytestmark = pytest.mark.gpu


def _run(wl, which):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute="f32")
    u = CC.pack_u(wl, dtype=torch.float32)
    y = plan.apply(u) if which == "cascade" else plan.recursion(u)
    torch.cuda.synchronize()
    out = CC.unpack_y(wl, y)
    plan.close()
    return out


def test_stability_L65536_fp32():
    wl = W.stability(seed=0)
    ps = wl.sets[0]
    yc = _run(wl, "cascade")
    yr = _run(wl, "recursion")
    ec, er = [], []
    for s, c, r in zip(wl.seqs, yc, yr):
        u = s.u.astype(np.float32).astype(np.float64)
        ref = O.truncated_sum_fft(ps.A, ps.B, ps.C, ps.D, u, s.N)
        Du = u @ ps.D.T
        ec.append(parity_err(c - Du, ref - Du))
        er.append(parity_err(r - Du, ref - Du))
    print("cascade state rel err", [f"{e:.2e}" for e in ec], "recursion", [f"{e:.2e}" for e in er],
          flush=True)
    assert max(ec) <= 1e-5
    assert max(ec) < max(er)


def test_stability_streamed_L4M_fp32():
    wl = W.stability(seed=0, batch=2, L=1 << 22, N=15)
    ps = wl.sets[0]
    T = 1 << 16
    h = O.impulse_response(ps.A, ps.B, ps.C, T)[:, 0, 0]
    fir_bound = float(np.sum(np.abs(h)) + abs(ps.D[0, 0]))
    yc = _run(wl, "cascade")
    yr = _run(wl, "recursion")
    for s, c, r in zip(wl.seqs, yc, yr):
        u = s.u.astype(np.float32).astype(np.float64)
        ref = O.truncated_sum_fft(ps.A, ps.B, ps.C, ps.D, u, s.N)
        Du = u @ ps.D.T
        e = parity_err(c - Du, ref - Du)
        umax = float(np.max(np.abs(u)))
        print(f"L=2^22 cascade rel err {e:.2e}, max|y| {np.max(np.abs(c)):.3e} "
              f"(FIR bound {fir_bound * umax:.3e}), recursion max|y| {np.max(np.abs(r)):.3e}",
              flush=True)
        assert e <= 1e-5
        assert np.max(np.abs(c)) <= fir_bound * umax
        assert np.max(np.abs(r[-1000:])) > 1e12 * np.max(np.abs(c))
