"""Parity of the HIP adjoint cascade with the CPU FP64 oracle gradients
(backpropagation in time, or brute force when the window truncates), with
central finite differences through the FP64 GPU path, and invariance under
the checkpoint interval. Tolerances on the relative Frobenius error of each
gradient: FP64 1e-10, FP32 1e-5, BF16 2e-2."""

import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-5, "bf16": 2e-2}


def _oracle_grads(wl, dys, us, disc="trapezoid"):
    """Per-set sums of the oracle gradients and per-sequence du (``disc``: the
    discretization of a workload that is not given)."""
    nS = len(wl.sets)
    acc = [dict(A=0.0, B=0.0, C=0.0, D=0.0) for _ in range(nS)]
    dus = []
    for s, dy, u in zip(wl.seqs, dys, us):
        ps = wl.sets[s.param_set]
        if wl.given:
            T = 1 << (s.N + 1)
            if T >= s.L:
                g = O.grads_recursion(ps.A, ps.B, ps.C, ps.D, u, dy)
            else:
                g = O.grads_truncated_bruteforce(ps.A, ps.B, ps.C, ps.D, u, dy, s.N)
            g = dict(u=g["u"], A=g["Abar"], B=g["Bbar"], C=g["C"], D=g["D"])
        else:
            g = O.grads_full(ps.A, ps.B, ps.C, ps.D, s.delta, u, dy, s.N, disc=disc)
        for k in "ABCD":
            acc[s.param_set][k] = acc[s.param_set][k] + g[k]
        dus.append(g["u"])
    return acc, dus


def _gpu_grads(wl, compute, dys, ckpt_every=0, u_dtype=None, **plan_kw):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute=compute, with_backward=True, ckpt_every=ckpt_every,
                                **plan_kw)
    sd = plan.state_dtype
    u = CC.pack_u(wl, dtype=u_dtype or sd)
    dy = torch.as_tensor(np.concatenate([d.reshape(-1) for d in dys]), device="cuda").to(sd)
    du, g = plan.backward(u, dy)
    torch.cuda.synchronize()
    us, off = [], 0
    uf = u.double().cpu().numpy()
    for s in wl.seqs:
        p = wl.sets[s.param_set].p
        us.append(uf[off: off + s.L * p].reshape(s.L, p))
        off += s.L * p
    dul, off = [], 0
    duf = du.double().cpu().numpy()
    for s in wl.seqs:
        p = wl.sets[s.param_set].p
        dul.append(duf[off: off + s.L * p].reshape(s.L, p))
        off += s.L * p
    gs = [[t.cpu().numpy() for t in parts] for parts in g]
    return dul, gs, us, plan


def _compare(wl, compute, ckpt_every=0, tol=None, u_dtype=None, disc="trapezoid", **plan_kw):
    rng = np.random.default_rng(123)
    dys = wl.dy if wl.dy is not None else [rng.standard_normal((s.L, wl.sets[s.param_set].q)) for s in wl.seqs]
    if compute != "f64":
        dys = [d.astype(np.float32).astype(np.float64) for d in dys]
    if disc != "trapezoid":
        plan_kw["disc"] = disc
    dul, gs, us, _ = _gpu_grads(wl, compute, dys, ckpt_every, u_dtype, **plan_kw)
    ref, dus = _oracle_grads(wl, dys, us, disc)
    tol = TOL[compute] if tol is None else tol
    errs = {"u": max(parity_err(a, b) for a, b in zip(dul, dus))}
    for si in range(len(wl.sets)):
        if not any(s.param_set == si for s in wl.seqs):
            continue
        for j, k in enumerate("ABCD"):
            errs[f"{k}{si}"] = max(errs.get(f"{k}{si}", 0.0), parity_err(gs[si][j], ref[si][k]))
    print(wl.name, compute, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    return errs


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_backward_hippo_small(compute):
    wl = W.backward(seed=1, batch=3, m=24, L=300, N=8, p=2, q=3, delta=2e-2)
    _compare(wl, compute)


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_backward_given_truncated_window(compute):
    # 2^(N+1) < L: the gradient of the truncated map, by brute force
    wl = W.random_small(seed=2, m=5, p=2, q=2, L=23, N=2, n_seq=2, contraction=0.95)
    _compare(wl, compute)


@pytest.mark.parametrize("ckpt", [1, 2, 3, 0])
def test_backward_checkpoint_interval(ckpt):
    wl = W.backward(seed=4, batch=2, m=40, L=700, N=9, p=3, q=2, delta=1e-2)
    _compare(wl, "f64", ckpt_every=ckpt)


@pytest.mark.parametrize("compute,ckpt", [("f32", 1), ("f32", 3), ("bf16", 1), ("bf16", 4)])
def test_backward_input_pass_stage_inputs(compute, ckpt):
    # m = 128, p = 4: the stage inputs x^(1) .. x^(5) come from the resident
    # input pass (also when a checkpoint segment recomputes them)
    wl = W.backward(seed=6, batch=2, m=128, L=1500, N=10, p=4, q=4)
    _compare(wl, compute, ckpt_every=ckpt)


def test_backward_checkpointing_is_exact():
    # recomputing stage inputs from checkpoints reproduces them bit for bit
    from paper_2411_17729_amd import cascade as CC
    wl = W.backward(seed=5, batch=2, m=128, L=2000, N=10, p=4, q=4)
    dys = [d.astype(np.float32).astype(np.float64) for d in wl.dy]
    res = []
    for ck in (1, 4):
        dul, gs, _, _ = _gpu_grads(wl, "f32", dys, ckpt_every=ck)
        res.append((dul, gs))
    for a, b in zip(res[0][0], res[1][0]):
        assert np.array_equal(a, b)
    for pa, pb in zip(res[0][1], res[1][1]):
        for a, b in zip(pa, pb):
            assert np.array_equal(a, b)


def test_backward_ragged_classes():
    # sequences in several size classes, different N, a delta per sequence
    rng = np.random.default_rng(9)
    sets, seqs = [], []
    for i, (m, p, q, L, N) in enumerate([(7, 1, 2, 50, 5), (40, 3, 1, 257, 8), (70, 2, 2, 130, 7),
                                         (130, 4, 3, 96, 6), (200, 2, 2, 65, 6)]):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m), rng.standard_normal((q, p))))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    # a second sequence of set 1 with another delta (two operators of one set)
    seqs.append(W.Sequence(1, 3e-3, 100, 6, rng.standard_normal((100, 3))))
    wl = W.Workload("ragged_small", sets, seqs)
    _compare(wl, "f32")
    _compare(wl, "f64")
    # every operator padded to 256 (the padding is exact; gradients are cropped to m)
    _compare(wl, "f32", min_padded_m=256)


def test_backward_full_size_fp32():
    # 8 sequences x L = 8192, HiPPO m = 128, p = q = 4, delta = 5e-3, N = 12
    wl = W.backward(seed=0)
    _compare(wl, "f32")


def test_backward_bf16_m256():
    # BF16 operands at padded m 256 (the bench's state size), two sequences
    # sharing one HiPPO model, p = q = 8
    wl = W.backward(seed=8, batch=2, m=256, L=4096, N=11, p=8, q=8, delta=1e-2)
    _compare(wl, "bf16")


def test_backward_ragged_256_bf16_sampled():
    # the ragged batch of 256 sequences (every sequence its own HiPPO model of
    # m in {64, 128, 256}, L log-uniform in [512, 65536], N = ceil(log2 L) - 1),
    # BF16, the gradients of the whole batch in one backward call, checked
    # against the oracle on the longest and shortest sequences and a
    # mid-length one of each other size class
    wl = W.ragged(seed=0)
    dys = [d.astype(np.float32).astype(np.float64) for d in wl.dy]
    dul, gs, us, plan = _gpu_grads(wl, "bf16", dys)
    assert plan.info()["launch"] == 2
    Ls = [s.L for s in wl.seqs]
    ms = [wl.sets[s.param_set].m for s in wl.seqs]
    sample = {int(np.argmax(Ls)), int(np.argmin(Ls))}
    for m in (64, 128, 256):
        idx = sorted((i for i in range(len(Ls)) if ms[i] == m), key=lambda i: Ls[i])
        if not any(ms[i] == m for i in sample):
            sample.add(idx[len(idx) // 2])
    for i in sorted(sample):
        s = wl.seqs[i]
        ps = wl.sets[s.param_set]
        g = O.grads_full(ps.A, ps.B, ps.C, ps.D, s.delta, us[i], dys[i], s.N)
        errs = {"u": parity_err(dul[i], g["u"])}
        for j, k in enumerate("ABCD"):
            errs[k] = parity_err(gs[s.param_set][j], g[k])
        print("seq", i, "L", s.L, "m", ps.m, {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
        bad = {k: v for k, v in errs.items() if not v <= TOL["bf16"]}
        assert not bad, (i, bad)


def test_finite_differences_fp64_gpu():
    # central differences (h = 1e-6) of <dy, y> through the FP64 GPU forward
    from paper_2411_17729_amd import cascade as CC
    wl = W.backward(seed=6, batch=2, m=32, L=400, N=8, p=2, q=2, delta=1e-2)
    ps = wl.sets[0]
    dys = wl.dy
    dul, gs, us, _ = _gpu_grads(wl, "f64", dys)
    dyt = np.concatenate([d.reshape(-1) for d in dys])
    rng = np.random.default_rng(0)

    def f(A, B, C, D):
        w2 = W.Workload("fd", [W.ParamSet(A, B, C, D)], wl.seqs)
        plan = CC.plan_for_workload(w2, compute="f64")
        y = plan.apply(CC.pack_u(w2, dtype=torch.float64)).cpu().numpy()
        return float(np.dot(dyt, y))

    h = 1e-6
    base = dict(A=ps.A, B=ps.B, C=ps.C, D=ps.D)
    for j, name in enumerate("ABCD"):
        V = rng.standard_normal(base[name].shape)
        plus = dict(base)
        minus = dict(base)
        plus[name] = base[name] + h * V
        minus[name] = base[name] - h * V
        fd = (f(**plus) - f(**minus)) / (2 * h)
        an = float(np.sum(gs[0][j] * V))
        print(name, fd, an, flush=True)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, fd, an)


def test_autograd_function():
    from paper_2411_17729_amd import cascade as CC
    wl = W.backward(seed=7, batch=2, m=16, L=100, N=6, p=2, q=2, delta=1e-2)
    ps = wl.sets[0]
    layout = CC.make_layout(wl.seqs, [(ps.m, ps.p, ps.q)])
    params = [torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True)
              for x in (ps.A, ps.B, ps.C, ps.D)]
    u = CC.pack_u(wl, dtype=torch.float64).requires_grad_(True)
    y = CC.ssm_cascade(u, [params], layout, compute="f64")
    dy = torch.as_tensor(np.concatenate([d.reshape(-1) for d in wl.dy]), device="cuda")
    (y * dy).sum().backward()
    ref, dus = _oracle_grads(wl, wl.dy, [s.u for s in wl.seqs])
    assert parity_err(u.grad.cpu().numpy(), np.concatenate([d.reshape(-1) for d in dus])) < 1e-10
    for t, k in zip(params, "ABCD"):
        assert parity_err(t.grad.cpu().numpy(), ref[0][k]) < 1e-10, k
