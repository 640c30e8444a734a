"""The chain-walking stage kernel: against the FP64 oracle, against the
resident kernel, across segment lengths (bitwise: every block sees the same
operands in the same order whatever the segmentation), and in the adjoint
direction through the backward pass."""

import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err

pytestmark = pytest.mark.gpu

# (m, p, q, L, N): padded sizes 64, 128 and 256; L not a multiple of 16 or of
# the shifts; stages whose shift exceeds half of L; a sequence shorter than 16;
# a window 2^(N+1) = 512 shorter than the sequence (truncated sum)
SPEC = [(256, 8, 8, 3001, 11), (128, 4, 2, 1999, 10), (64, 2, 3, 777, 9), (100, 3, 1, 500, 8),
        (200, 1, 5, 33, 5), (48, 2, 2, 15, 3), (256, 8, 8, 4096, 11), (64, 2, 2, 2500, 8)]


def _workload(seed=21, zero_d=True):
    rng = np.random.default_rng(seed)
    sets, seqs = [], []
    for i, (m, p, q, L, N) in enumerate(SPEC):
        A, _ = W.hippo_legs(m)
        D = np.zeros((q, p)) if zero_d else rng.standard_normal((q, p)) / math.sqrt(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m), D))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    return W.Workload("chain", sets, seqs)


def _oracle(wl):
    out = []
    for s in wl.seqs:
        ps = wl.sets[s.param_set]
        Abar, Bbar = O.trapezoid(ps.A, ps.B, s.delta)
        u = s.u.astype(np.float32).astype(np.float64)
        if (1 << (s.N + 1)) >= s.L:
            y, _ = O.recursion(Abar, Bbar, ps.C, ps.D, u)
        else:
            y = O.truncated_sum(Abar, Bbar, ps.C, ps.D, u, s.N)
        out.append(y)
    return out


def _apply(wl, compute, **kw):
    # (the chain kernels run every stage: no output fold)
    from paper_2411_17729_amd import cascade as CC
    kw.setdefault("fold_stages", -1)
    plan = CC.plan_for_workload(wl, compute=compute, launch="per_stage", **kw)
    info = plan.info()
    u = CC.pack_u(wl, dtype=torch.float32)
    y = plan.apply(u).clone()
    torch.cuda.synchronize()
    plan.close()
    return y, info


@pytest.mark.parametrize("compute", ["f32", "bf16"])
@pytest.mark.parametrize("input_stages", [0, -1])
def test_chain_matches_oracle(compute, input_stages):
    # D = 0 (y is the state part alone, so its error is not hidden under D u)
    # and D != 0 (the epilogue's D u term)
    from paper_2411_17729_amd import cascade as CC
    tol = 1e-5 if compute == "f32" else 2e-2
    for zero_d in (True, False):
        wl = _workload(zero_d=zero_d)
        y, info = _apply(wl, compute, stage_kernel="chain", input_stages=input_stages)
        assert info["stage_kernel"] == 3
        got = CC.unpack_y(wl, y)
        ref = _oracle(wl)
        for i in range(len(wl.seqs)):
            e = parity_err(got[i], ref[i])
            print(compute, input_stages, "D=0" if zero_d else "D!=0", "seq", i, f"{e:.2e}",
                  flush=True)
            assert e <= tol, (i, zero_d, e)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_chain_segment_lengths_bitwise(compute):
    wl = _workload(seed=22)
    ys = [_apply(wl, compute, stage_kernel="chain", chain_blocks=t)[0] for t in (1, 3, 8, 64)]
    for y in ys[1:]:
        assert torch.equal(ys[0], y)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_chain_matches_resident(compute):
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(seed=23)
    yc, ic = _apply(wl, compute, stage_kernel="chain")
    yr, ir = _apply(wl, compute, stage_kernel="resident")
    assert (ic["stage_kernel"], ir["stage_kernel"]) == (3, 2)
    tol = 2e-6 if compute == "f32" else 1e-2
    for a, b in zip(CC.unpack_y(wl, yc), CC.unpack_y(wl, yr)):
        assert parity_err(a, b) <= tol


@pytest.mark.parametrize("compute", ["f32", "bf16"])
@pytest.mark.parametrize("stage_kernel", ["chain", "resident"])
def test_backward_per_stage_kernels(compute, stage_kernel):
    # the adjoint walks the columns the other way (reversed shifts)
    from tests.test_gpu_backward import _compare
    wl = W.backward(seed=24, batch=3, m=128, L=1500, N=10, p=4, q=4, delta=5e-3)
    _compare(wl, compute, launch="per_stage", stage_kernel=stage_kernel)


def _ragged_res(seed, compute, one_fold=False):
    # uneven L (33 .. 5000) and m over the classes the resident persistent launch
    # takes; p <= m/4 so both launch modes fold the same stages
    rng = np.random.default_rng(seed)
    spec = [(64, 4, 2, 5000, 12), (100, 2, 3, 1777, 10), (128, 8, 4, 3001, 11), (48, 4, 1, 33, 5),
            (60, 4, 4, 700, 6), (64, 16, 2, 1500, 10)]  # the last folds 2 stages: stages 2, 3 by rows
    if compute == "bf16":
        spec += [(256, 8, 8, 4100, 12), (200, 4, 2, 999, 9)]
    if one_fold:  # one stage folded into the input pass (the persistent launch only):
        # 2p = padded m, and sequences of length 1 and 2
        spec += [(64, 32, 2, 1000, 9), (64, 2, 2, 2, 1), (128, 4, 4, 1, 0)]
    sets, seqs = [], []
    for i, (m, p, q, L, N) in enumerate(spec):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m),
                               rng.standard_normal((q, p)) / math.sqrt(m)))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    return W.Workload("ragged_res", sets, seqs)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_resident_persistent_matches_per_stage(compute):
    # one persistent launch of input-pass, resident and chain items against the
    # per-stage launches of the same code: every row sees the same operands in
    # the same order, so the outputs agree bit for bit
    from paper_2411_17729_amd import cascade as CC
    wl = _ragged_res(31, compute)
    u = CC.pack_u(wl, dtype=torch.float32)
    pers = CC.plan_for_workload(wl, compute=compute, launch="persistent")
    info = pers.info()
    assert info["launch"] == 2 and info["stage_kernel"] == 3 and info["input_stages"] >= 4
    per = CC.plan_for_workload(wl, compute=compute, launch="per_stage", pair_stages=1, input_split=1,
                               fold_stages=-1)
    ya = pers.apply(u).clone()
    yb = per.apply(u).clone()
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
    got = CC.unpack_y(wl, ya)
    ref = _oracle(wl)
    tol = 1e-5 if compute == "f32" else 2e-2
    for i in range(len(wl.seqs)):
        e = parity_err(got[i], ref[i])
        assert e <= tol, (i, e)


def test_resident_persistent_one_folded_stage():
    # operators with 2p = padded m, or sequences of one or two steps, fold a
    # single stage into the input pass
    from paper_2411_17729_amd import cascade as CC
    wl = _ragged_res(32, "bf16", one_fold=True)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="persistent")
    assert plan.info()["stage_kernel"] == 3
    got = CC.unpack_y(wl, plan.apply(CC.pack_u(wl, dtype=torch.float32)))
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        assert parity_err(got[i], ref[i]) <= 2e-2, i


def test_resident_persistent_graph_replays():
    from paper_2411_17729_amd import cascade as CC
    wl = _ragged_res(33, "bf16")
    plan = CC.plan_for_workload(wl, compute="bf16")
    assert plan.info()["launch"] == 2 and plan.info()["stage_kernel"] == 3
    stream = torch.cuda.Stream()
    u = CC.pack_u(wl, dtype=torch.float32)
    y = torch.empty(plan.layout.y_numel, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g = plan.graph_apply(u, y, stream)
    try:
        for rep in range(3):
            with torch.cuda.stream(stream):
                u.mul_(0.5 + rep)  # eager work between replays
            CC.CascadePlan.graph_launch(g, stream)
            stream.synchronize()
            ref = plan.apply(u)
            torch.cuda.synchronize()
            assert torch.equal(y, ref), rep
    finally:
        CC.CascadePlan.graph_destroy(g)


def test_lower_triangular_powers_are_marked():
    """Prepare marks operators whose Abar is lower triangular (every HiPPO
    operator; none of a dense random one); the FP32 chain kernel then skips the
    zero blocks of their powers, with the same results as the oracle."""
    from paper_2411_17729_amd import cascade as CC
    wl = W.batched(seed=2, batch=2, m=128, L=3000, N=10, p=4, q=4)
    plan = CC.plan_for_workload(wl, compute="f32", launch="per_stage")
    info = plan.info()
    assert info["lower_ops"] == info["n_ops"] == 2
    y = CC.unpack_y(wl, plan.apply(CC.pack_u(wl, dtype=torch.float32)))
    torch.cuda.synchronize()
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        assert parity_err(y[i], ref[i]) <= 1e-5, i
    dense = W.random_small(seed=1, m=64, p=2, q=2, L=500, N=7, n_seq=1, contraction=0.9)
    assert CC.plan_for_workload(dense, compute="f32").info()["lower_ops"] == 0


@pytest.mark.parametrize("mix", [False, True])
def test_fp32_split_halves(mix):
    """FP32 at padded m 256: two workgroups share each chain unit, holding the
    interleaved halves of P_k's rows. With every operator of the class lower
    triangular the launches leave out the zero blocks (forward and adjoint);
    a dense operator in the class (mix) turns that off for the whole class.
    Forward against the FP64 oracle, gradients against the oracle's."""
    from paper_2411_17729_amd import cascade as CC
    from tests.test_gpu_backward import _compare
    rng = np.random.default_rng(31)
    sets, seqs = [], []
    for i, (m, p, q, L, N) in enumerate([(256, 4, 4, 3001, 11), (200, 2, 3, 1500, 10)]):
        if mix and i == 1:  # stable, dense: Abar has entries above the diagonal
            A = rng.standard_normal((m, m)) / math.sqrt(m) - 1.5 * np.eye(m)
        else:
            A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m),
                               rng.standard_normal((q, p)) / math.sqrt(m)))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    wl = W.Workload("split_halves", sets, seqs)
    y, info = _apply(wl, "f32")
    assert info["n_ops"] == 2 and info["lower_ops"] == (1 if mix else 2)
    for a, b in zip(CC.unpack_y(wl, y), _oracle(wl)):
        assert parity_err(a, b) <= 1e-5
    _compare(wl, "f32", launch="per_stage", stage_kernel="chain")


@pytest.mark.parametrize("pq", [(16, 16), (3, 17)])
def test_fp32_m256_output_widths(pq):
    """FP32 at padded m 256: the last stage runs lean and a separate pass forms
    y = C x + D u (du = Bbar^T g + D^T dy) while p and q are at most 16 (the
    widest case here); with q = 17 the tiled stage kernel forms it instead.
    Forward against the FP64 oracle, gradients against the oracle's."""
    from paper_2411_17729_amd import cascade as CC
    from tests.test_gpu_backward import _compare
    p, q = pq
    rng = np.random.default_rng(37)
    sets, seqs = [], []
    for i, (m, L, N) in enumerate([(256, 700, 9), (230, 333, 8)]):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m),
                               rng.standard_normal((q, p)) / math.sqrt(m)))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    wl = W.Workload("output_widths", sets, seqs)
    y, info = _apply(wl, "f32")
    for a, b in zip(CC.unpack_y(wl, y), _oracle(wl)):
        assert parity_err(a, b) <= 1e-5
    _compare(wl, "f32", launch="per_stage", stage_kernel="chain")
