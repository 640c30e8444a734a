"""Stage pairs: two consecutive lean stages of the forward cascade in one pass
(w_l = y_l + P_{k+1} y_{l-2^{k+1}}, y_l = x_l + P_k x_{l-2^k}). Against the
FP64 oracle, against the same plan with pairs off, across segment lengths
(bitwise: a block's partners are rebuilt from the same rows in the same
order whatever the segmentation) and under graph replay."""

import math

import numpy as np
import pytest
import torch

from paper_2411_17729_amd import workloads as W
from tests.helpers import parity_err
from tests.test_gpu_chain import _oracle

pytestmark = pytest.mark.gpu

# (m, p, q, L, N): padded m 256 (three sequences; the split input pass folds
# stages 0-5, pairs (6,7) (8,9) and the tail pair (10,11), which forms y) and
# 128 (last stages 9 and 10: the pair (6,7), then single stages); L not a
# multiple of 16; columns shorter than a segment (segments run on into the
# next column); a class of 64 that has no pairs
SPEC = [(256, 8, 8, 4096, 11), (256, 8, 8, 3001, 11), (256, 8, 4, 2500, 11),
        (100, 4, 2, 1999, 10), (128, 4, 3, 1000, 10), (64, 2, 2, 777, 9)]


def _workload(seed, zero_d=False, spec=SPEC):
    rng = np.random.default_rng(seed)
    sets, seqs = [], []
    for i, (m, p, q, L, N) in enumerate(spec):
        A, _ = W.hippo_legs(m)
        D = np.zeros((q, p)) if zero_d else rng.standard_normal((q, p)) / math.sqrt(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m),
                               rng.standard_normal((q, m)) / math.sqrt(m), D))
        seqs.append(W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, N, rng.standard_normal((L, p))))
    return W.Workload("pairs", sets, seqs)


def _apply(wl, **kw):
    # (the pairs run to the last stage: no output fold)
    from paper_2411_17729_amd import cascade as CC
    kw.setdefault("fold_stages", -1)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", **kw)
    info = plan.info()
    y = plan.apply(CC.pack_u(wl, dtype=torch.float32)).clone()
    torch.cuda.synchronize()
    plan.close()
    return y, info


@pytest.mark.parametrize("zero_d", [True, False])
def test_pair_matches_oracle(zero_d):
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(41, zero_d=zero_d)
    y, info = _apply(wl)
    print("pair launches", info["pair_launches"], "stage launches", info["stage_launches"], flush=True)
    assert info["stage_kernel"] == 3 and info["pair_launches"] == 4 and info["input_stages"] == 6
    got = CC.unpack_y(wl, y)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(got[i], ref[i])
        print("seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)


def _paired_vs_unpaired(wl, tail_seqs, **kw):
    # Every state row of a pair sees the operands of two chain launches (the
    # FP32 stage input rounded to BF16, the same entries in the same operand
    # slots of the same MFMA steps, accumulated onto the same FP32 row), so
    # outputs formed by the chain kernel agree bit for bit. A tail pair forms
    # C w = C y + (C P_{k+1}) y_prev2 with the product C P_{k+1} rounded once to
    # BF16 (the unpaired path rounds P_{k+1} and multiplies by C in FP32), so
    # its outputs differ by one BF16 rounding of that term.
    from paper_2411_17729_amd import cascade as CC
    yp, ip = _apply(wl, **kw)
    yu, iu = _apply(wl, pair_stages=1, **kw)
    assert iu["pair_launches"] == 0
    assert iu["stage_launches"] == ip["stage_launches"] + ip["pair_launches"]
    for i, (a, b) in enumerate(zip(CC.unpack_y(wl, yp), CC.unpack_y(wl, yu))):
        e = parity_err(a, b)
        print("seq", i, f"{e:.2e}", flush=True)
        if i in tail_seqs:
            assert e <= 2e-3, (i, e)
        else:
            assert np.array_equal(a, b), i
    return yp, ip


def test_pair_matches_unpaired():
    wl = _workload(42)
    _, ip = _paired_vs_unpaired(wl, tail_seqs={0, 1, 2})
    assert ip["pair_launches"] == 4


def test_pair_segment_lengths_bitwise():
    wl = _workload(43)
    ys = [_apply(wl, pair_blocks=t)[0] for t in (4, 5, 13, 64, 256)]
    for y in ys[1:]:
        assert torch.equal(ys[0], y)


def test_pair_graph_replays():
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(44)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", fold_stages=-1)
    assert plan.info()["pair_launches"] == 4
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


def test_pair_from_stage4():
    # four folded stages: the first pair is (4, 5), whose columns are single
    # 16-row blocks apart; bitwise equal to the unpaired plan and within the
    # BF16 bound of the oracle
    from paper_2411_17729_amd import cascade as CC
    spec = [(256, 16, 4, 3000, 11), (256, 16, 8, 2049, 11), (128, 8, 2, 1777, 10), (100, 8, 3, 1500, 10)]
    wl = _workload(45, spec=spec)
    yp, ip = _paired_vs_unpaired(wl, tail_seqs={0, 1}, input_stages=4)
    # padded m 256: pairs from 4 to the tail pair (10, 11); 128: from 4 to (8, 9)
    assert ip["input_stages"] == 4 and ip["pair_launches"] == 7
    got = CC.unpack_y(wl, yp)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(got[i], ref[i])
        print("seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)


# The split input pass: K_j rows in registers, up to 2^j p = 2 m columns; one
# p per class. (m, p, q, L, N): L not a multiple of 16 and shorter than a unit
# of rows, m below the padded size; p = 8 and 4 (j = 6: 2^j p = 512 and 256)
# or p = 16 and 8 (j = 5: 512 and 256, 16-byte operands in both classes)
SPLIT_SPECS = {
    6: [(256, 8, 8, 5000, 13), (200, 8, 4, 3001, 11), (256, 8, 2, 777, 10),
        (128, 4, 2, 2500, 11), (100, 4, 3, 999, 9), (128, 4, 4, 1100, 8)],
    5: [(256, 16, 4, 2000, 11), (256, 16, 2, 999, 10), (128, 8, 2, 1500, 10), (120, 8, 4, 700, 9)],
}


@pytest.mark.parametrize("j", [6, 5])
@pytest.mark.parametrize("u_dtype", ["f32", "bf16"])
@pytest.mark.parametrize("zero_d", [True, False])
def test_split_input_matches_oracle(j, u_dtype, zero_d):
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(46, zero_d=zero_d, spec=SPLIT_SPECS[j])
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", fold_stages=-1)
    info = plan.info()
    # j: the largest with 2^j p <= 2 padded m (the resident pass: 2^j p <= m)
    assert info["input_stages"] == j, info["input_stages"]
    dt = torch.float32 if u_dtype == "f32" else torch.bfloat16
    u = CC.pack_u(wl, dtype=dt)
    got = CC.unpack_y(wl, plan.apply(u))
    torch.cuda.synchronize()
    plan.close()
    if u_dtype == "bf16":  # the oracle sees the inputs the GPU sees
        flat = u.double().cpu().numpy()
        off = 0
        for s_ in wl.seqs:
            n = s_.L * wl.sets[s_.param_set].B.shape[1]
            s_.u = flat[off: off + n].reshape(s_.L, -1)
            off += n
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(got[i], ref[i])
        print(u_dtype, "D=0" if zero_d else "D!=0", "seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)


def test_split_input_matches_resident_input():
    # the same j folded by the resident pass (K_j in LDS) and the split pass:
    # the same BF16 operands, summed in another order, so the outputs agree to
    # far below the BF16 error
    from paper_2411_17729_amd import cascade as CC
    spec = [(256, 8, 8, 4000, 12), (128, 4, 4, 3001, 11)]
    wl = _workload(47, spec=spec)
    ys, isp = _apply(wl, input_stages=5)
    yr, ire = _apply(wl, input_stages=5, input_split=1)
    assert isp["input_stages"] == ire["input_stages"] == 5
    for i, (a, b) in enumerate(zip(CC.unpack_y(wl, ys), CC.unpack_y(wl, yr))):
        e = parity_err(a, b)
        print("seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-3, (i, e)


@pytest.mark.parametrize("case", ["short", "mixed_p"])
def test_split_input_falls_back(case):
    # a sequence whose last stage comes before the split pass's j, or a class
    # whose operators differ in p, keeps its class on the resident input pass
    from paper_2411_17729_amd import cascade as CC
    spec = {"short": [(256, 8, 8, 3000, 11), (256, 8, 4, 40, 11)],  # L = 40: last stage 5 < 6
            "mixed_p": [(256, 8, 8, 3000, 11), (256, 16, 4, 2000, 11)]}[case]
    wl = _workload(48, spec=spec)
    y, info = _apply(wl)
    assert info["input_stages"] == 5
    got = CC.unpack_y(wl, y)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        assert parity_err(got[i], ref[i]) <= 2e-2, i


@pytest.mark.parametrize("case", ["q16_p64", "bf16_u", "q17"])
def test_tail_pair_edges(case):
    # the tail pair at its limits: 16 outputs and 64 inputs (segments of 8
    # blocks to fit the staged inputs), BF16 inputs, and 17 outputs, where the
    # last two stages run unpaired
    from paper_2411_17729_amd import cascade as CC
    spec = {"q16_p64": [(256, 64, 16, 3000, 11), (250, 64, 16, 2100, 11)],
            "bf16_u": [(256, 8, 8, 3000, 11), (256, 8, 3, 2500, 11)],
            "q17": [(256, 8, 17, 3000, 11), (256, 8, 4, 2500, 11)]}[case]
    wl = _workload(49, spec=spec)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", fold_stages=-1)
    info = plan.info()
    dt = torch.bfloat16 if case == "bf16_u" else torch.float32
    u = CC.pack_u(wl, dtype=dt)
    got = CC.unpack_y(wl, plan.apply(u))
    torch.cuda.synchronize()
    plan.close()
    npair = {"q16_p64": 4, "bf16_u": 3, "q17": 2}[case]  # j = 3, 6, 6
    assert info["pair_launches"] == npair, info["pair_launches"]
    if case == "bf16_u":
        flat = u.double().cpu().numpy()
        off = 0
        for s_ in wl.seqs:
            n = s_.L * wl.sets[s_.param_set].B.shape[1]
            s_.u = flat[off: off + n].reshape(s_.L, -1)
            off += n
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(got[i], ref[i])
        print(case, "seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)
