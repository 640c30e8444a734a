"""The backward from an initial state (ssm_cascade_backward_x0) against the
FP64 oracle: dL/dx_{-1} and the parameter gradients with x_{-1} != 0
(backpropagation in time, or brute force where the window truncates), with
sequences sharing an operator, ragged size classes and the three compute
types. Tolerances as for the other gradients: FP64 1e-10, FP32 1e-5, BF16
2e-2 (relative Frobenius error per result)."""

import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err, rel_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-2}


def _ragged_workload(seed):
    rng = np.random.default_rng(seed)
    sets, seqs = [], []
    for i, (m, p, q) in enumerate([(24, 2, 3), (100, 3, 2)]):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m), rng.standard_normal((q, p))))
    # set 1 twice with one delta (one operator, two sequences), once with another
    for ps_i, d, L, N in [(0, 2e-2, 300, 8), (1, 5e-3, 257, 8), (1, 5e-3, 130, 7), (1, 1e-2, 200, 7)]:
        seqs.append(W.Sequence(ps_i, d, L, N, rng.standard_normal((L, sets[ps_i].p))))
    return W.Workload("ragged_x0", sets, seqs)


def _run(wl, compute, x0s, with_x0=True):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute=compute, with_backward=True)
    sd = plan.state_dtype
    rng = np.random.default_rng(5)
    dys = [rng.standard_normal((s.L, wl.sets[s.param_set].q)) for s in wl.seqs]
    if compute != "f64":
        dys = [d.astype(np.float32).astype(np.float64) for d in dys]
        x0s = [x.astype(np.float32).astype(np.float64) for x in x0s]
    u = CC.pack_u(wl, dtype=sd)
    dy = torch.as_tensor(np.concatenate([d.reshape(-1) for d in dys]), device="cuda").to(sd)
    x0 = torch.as_tensor(np.concatenate(x0s), device="cuda").to(sd) if with_x0 else None
    du, g, dx0 = plan.backward(u, dy, x0=x0, want_dx0=True)
    torch.cuda.synchronize()
    uf = u.double().cpu().numpy()
    us, dul, off = [], [], 0
    duf = du.double().cpu().numpy()
    for s in wl.seqs:
        p = wl.sets[s.param_set].p
        us.append(uf[off: off + s.L * p].reshape(s.L, p))
        dul.append(duf[off: off + s.L * p].reshape(s.L, p))
        off += s.L * p
    dxl, off = [], 0
    dxf = dx0.double().cpu().numpy()
    for s in wl.seqs:
        m = wl.sets[s.param_set].m
        dxl.append(dxf[off: off + m])
        off += m
    gs = [[t.cpu().numpy() for t in parts] for parts in g]
    plan.close()
    return us, dys, x0s, dul, gs, dxl


def _oracle(wl, us, dys, x0s):
    acc = [dict(A=0.0, B=0.0, C=0.0, D=0.0) for _ in wl.sets]
    dus, dxs = [], []
    for s, u, dy, x0 in zip(wl.seqs, us, dys, x0s):
        ps = wl.sets[s.param_set]
        if wl.given:
            if (1 << (s.N + 1)) >= s.L:
                g = O.grads_recursion(ps.A, ps.B, ps.C, ps.D, u, dy, x0)
            else:
                g = O.grads_truncated_bruteforce(ps.A, ps.B, ps.C, ps.D, u, dy, s.N, x0)
            g = dict(u=g["u"], A=g["Abar"], B=g["Bbar"], C=g["C"], D=g["D"], x0=g["x0"])
        else:
            g = O.grads_full(ps.A, ps.B, ps.C, ps.D, s.delta, u, dy, s.N, x0=x0)
        for k in "ABCD":
            acc[s.param_set][k] = acc[s.param_set][k] + g[k]
        dus.append(g["u"])
        dxs.append(g["x0"])
    return acc, dus, dxs


def _check(wl, compute, x0s, tol=None, with_x0=True):
    us, dys, x0s, dul, gs, dxl = _run(wl, compute, x0s, with_x0)
    ref, dus, dxs = _oracle(wl, us, dys, x0s if with_x0 else [np.zeros_like(x) for x in x0s])
    tol = TOL[compute] if tol is None else tol
    errs = {"u": max(parity_err(a, b) for a, b in zip(dul, dus)),
            "x0": max(rel_err(a, b) for a, b in zip(dxl, dxs))}
    for si in range(len(wl.sets)):
        for j, k in enumerate("ABCD"):
            errs[f"{k}{si}"] = parity_err(gs[si][j], ref[si][k])
    print(wl.name, compute, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_backward_from_initial_state_ragged(compute):
    wl = _ragged_workload(11)
    rng = np.random.default_rng(12)
    x0s = [rng.standard_normal(wl.sets[s.param_set].m) for s in wl.seqs]
    _check(wl, compute, x0s)


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_backward_from_initial_state_truncated_window(compute):
    # 2^(N+1) < L: the free response stops at T lags; brute-force oracle
    wl = W.random_small(seed=13, m=5, p=2, q=2, L=23, N=2, n_seq=2, contraction=0.95)
    rng = np.random.default_rng(14)
    x0s = [rng.standard_normal(5) for _ in wl.seqs]
    _check(wl, compute, x0s)


def test_dx0_without_an_initial_state():
    # dx0 alone (x0 = NULL): the gradient at x_{-1} = 0, and the parameter
    # gradients of the plain backward
    wl = _ragged_workload(15)
    rng = np.random.default_rng(16)
    x0s = [rng.standard_normal(wl.sets[s.param_set].m) for s in wl.seqs]
    _check(wl, "f64", x0s, with_x0=False)
