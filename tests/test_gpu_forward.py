"""Parity of the HIP forward path (prepare, cascade, recursion) with the CPU
FP64 oracle, through the C ABI. Tolerances (relative Frobenius error per
sequence): FP64 1e-12, FP32 1e-5, BF16 2e-2, on y and on its state part
y - D u."""

import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import workloads as W
from tests.helpers import max_rel, oracle_outputs, parity_err, state_part

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def _run(wl, compute, u_dtype=None, recursion=False, **plan_kw):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute=compute, **plan_kw)
    if u_dtype is None:
        u_dtype = torch.float64 if compute == "f64" else torch.float32
    u = CC.pack_u(wl, dtype=u_dtype)
    y = plan.recursion(u) if recursion else plan.apply(u)
    torch.cuda.synchronize()
    # the u values the GPU actually saw (bf16 inputs are quantised)
    uq = []
    flat = u.double().cpu().numpy()
    off = 0
    for s in wl.seqs:
        p = wl.sets[s.param_set].p
        uq.append(flat[off: off + s.L * p].reshape(s.L, p))
        off += s.L * p
    return CC.unpack_y(wl, y), uq, plan


def _check(wl, compute, u_dtype=None, tol=None, recursion=False, **plan_kw):
    got, uq, plan = _run(wl, compute, u_dtype, recursion, **plan_kw)
    ref = oracle_outputs(wl, u_override=uq, method="recursion" if recursion else "auto")
    tol = TOL[compute] if tol is None else tol
    e_y = max_rel(got, ref)
    e_x = max_rel(state_part(wl, got, uq), state_part(wl, ref, uq))
    print(f"{wl.name} {compute} rel_y={e_y:.3e} rel_state={e_x:.3e}", flush=True)
    assert e_y <= tol and e_x <= tol, (e_y, e_x)
    return e_y, e_x, plan


def test_powers_and_bbar_fp64_worked_example():
    # §4 example: HiPPO m=100, delta=5e-4; a length that exercises P_0..P_15
    from paper_2411_17729_amd import cascade as CC
    m, delta, N = 100, 5e-4, 15
    A, b = W.hippo_legs(m)
    C = np.ones((1, m)) / m
    D = np.zeros((1, 1))
    seq = W.Sequence(0, delta, (1 << 15) + 1, N, None)
    layout = CC.make_layout([seq], [(m, 1, 1)])
    plan = CC.CascadePlan(layout, [(A, b[:, None], C, D)], compute="f64")
    Abar, Bbar = O.trapezoid(A, b, delta)
    P = O.powers(Abar, N)
    for k in range(N + 1):
        g = plan.power(0, k).cpu().numpy()
        err = np.max(np.abs(g - P[k])) / max(np.max(np.abs(P[k])), 1e-300)
        assert err < 1e-12, (k, err)
    # the paper's printed eigenvalue powers
    g15 = plan.power(0, 15).cpu().numpy()
    assert abs(g15[0, 0] / 5.87548e-15 - 1) < 2e-5
    gB = plan.bbar(0, m, 1).cpu().numpy()
    assert np.max(np.abs(gB - Bbar)) < 1e-13 * np.max(np.abs(Bbar))


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_plain_hippo_m64_L4096(compute):
    wl = W.plain_fp64(seed=0)
    _check(wl, compute)


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_small_shapes_and_truncation(compute):
    # m spanning every padded size, ragged L (1, 2, 3, tails), N below log2 L
    rng = np.random.default_rng(1)
    sets, seqs = [], []
    shapes = [(1, 1, 1), (5, 2, 3), (32, 4, 4), (33, 1, 2), (64, 8, 8), (100, 3, 1),
              (128, 4, 4), (200, 2, 5), (256, 8, 8)]
    Ls = [1, 2, 3, 17, 300, 1000, 129, 257, 64]
    Ns = [0, 0, 1, 3, 4, 9, 2, 8, 6]
    for i, ((m, p, q), L, N) in enumerate(zip(shapes, Ls, Ns)):
        A = rng.standard_normal((m, m))
        A *= 0.97 / max(np.linalg.norm(A, 2), 1e-12)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m),
                               rng.standard_normal((q, p)) * 0.1))
        seqs.append(W.Sequence(i, 0.0, L, N, rng.standard_normal((L, p))))
    wl = W.Workload("mixed_small", sets, seqs, given=True)
    _check(wl, compute)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_hippo_batched_shared_params(compute):
    # shared HiPPO parameters with one delta per sequence; several tiles + tail
    wl = W.batched(seed=3, batch=4, m=256, L=3000, N=11, p=8, q=8)
    _check(wl, compute)


def test_hippo_batched_full_size_fp32():
    # 16 sequences x L=16384, m=256, p=q=8, N=13, checked in full against the
    # FP64 recursion (2^(N+1) = L, so the window covers every sequence)
    wl = W.batched(seed=0)
    _check(wl, "f32")


def test_hippo_batched_full_size_bf16():
    # BF16 operands with the state kept in FP32 between passes (the bench's
    # second line), FP32 u, all 16 sequences in full
    wl = W.batched(seed=0)
    _check(wl, "bf16", state_bf16=0)


def test_hippo_batched_headline_plan():
    # the exact plan the headline bench line times: BF16 operands, the state
    # in BF16 between passes, the split input pass folding stages 0-5, one
    # stage pair (6, 7) and the six-stage output fold (8-13), on all 16
    # sequences of 16384 rows against the FP64 recursion (with the per-row
    # bound of parity_err)
    from paper_2411_17729_amd import binding as B
    wl = W.batched(seed=0)
    e_y, e_x, plan = _check(wl, "bf16", state_bf16=1)
    info = plan.info()
    assert info["state_dtype"] == B.SSM_BF16
    assert info["fold_stages"] == 6 and info["input_stages"] == 6
    assert info["pair_launches"] == 1 and info["fold_launches"] == 1
    assert info["stage_launches"] == 2  # the pair and the fold (the input pass is not a stage launch)


def test_hippo_batched_full_size_bf16_input():
    wl = W.batched(seed=0, batch=4)
    _check(wl, "bf16", u_dtype=torch.bfloat16)


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_recursion_matches_oracle(compute):
    wl = W.batched(seed=5, batch=3, m=128, L=700, N=9, p=4, q=4)
    _check(wl, compute, recursion=True, tol=1e-12 if compute == "f64" else 1e-4)


@pytest.mark.parametrize("m,p,L", [(20, 20, 300), (64, 1, 1000), (200, 200, 129), (256, 8, 2500)])
def test_recursion_fp32_sizes(m, p, L):
    # every padded size of the FP32 recursion kernel, the widest input (p = m:
    # the shortest chunks of Bbar u), chunk tails, one and several sequences
    wl = W.batched(seed=9, batch=2, m=m, L=L, N=max(1, math.ceil(math.log2(L)) - 1), p=p, q=3)
    _check(wl, "f32", recursion=True, tol=1e-4)


def test_stability_given_small():
    # discrete diagonal-plus-rank-2 Abar with one eigenvalue 1 + 1e-5
    wl = W.stability(seed=0, batch=2, m=128, L=4096, N=11)
    _check(wl, "f32")


def test_apply_is_deterministic():
    from paper_2411_17729_amd import cascade as CC
    wl = W.batched(seed=7, batch=2, m=128, L=2048, N=10, p=4, q=4)
    plan = CC.plan_for_workload(wl, compute="bf16")
    u = CC.pack_u(wl)
    y1 = plan.apply(u).clone()
    y2 = plan.apply(u)
    torch.cuda.synchronize()
    assert torch.equal(y1, y2)
