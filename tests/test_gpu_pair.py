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
from tests.helpers import rel_err
from tests.test_gpu_chain import _oracle

pytestmark = pytest.mark.gpu

# (m, p, q, L, N): padded m 256 (three sequences, pairs (5,6) (7,8) (9,10),
# tail 11) and 128 (last stages 9 and 10: pairs below 9, then single stages);
# L not a multiple of 16; columns of stage 9 shorter than a segment (segments
# run on into the next column); a class of 64 that has no pairs
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
    from paper_2411_17729_amd import cascade as CC
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
    assert info["stage_kernel"] == 3 and info["pair_launches"] == 5
    got = CC.unpack_y(wl, y)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = rel_err(got[i], ref[i])
        print("seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)


def test_pair_matches_unpaired():
    # every output of a pair sees the operands of two chain launches (the FP32
    # stage input rounded to BF16, the same entries in the same operand slots
    # of the same MFMA steps, accumulated onto the same FP32 row), so the two
    # plans agree bit for bit
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(42)
    yp, ip = _apply(wl)
    yu, iu = _apply(wl, pair_stages=1)
    assert ip["pair_launches"] == 5 and iu["pair_launches"] == 0
    assert iu["stage_launches"] == ip["stage_launches"] + 5
    for i, (a, b) in enumerate(zip(CC.unpack_y(wl, yp), CC.unpack_y(wl, yu))):
        print("seq", i, f"{rel_err(a, b):.2e}", flush=True)
    assert torch.equal(yp, yu)


def test_pair_segment_lengths_bitwise():
    wl = _workload(43)
    ys = [_apply(wl, pair_blocks=t)[0] for t in (4, 5, 13, 64, 256)]
    for y in ys[1:]:
        assert torch.equal(ys[0], y)


def test_pair_graph_replays():
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(44)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage")
    assert plan.info()["pair_launches"] == 5
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
    # 2^5 p > padded m folds four stages: the first pair is (4, 5), whose
    # columns are single 16-row blocks apart; bitwise equal to the unpaired
    # plan and within the BF16 bound of the oracle
    from paper_2411_17729_amd import cascade as CC
    spec = [(256, 16, 4, 3000, 11), (256, 16, 8, 2049, 11), (128, 8, 2, 1777, 10), (100, 8, 3, 1500, 10)]
    wl = _workload(45, spec=spec)
    yp, ip = _apply(wl)
    yu, iu = _apply(wl, pair_stages=1)
    assert ip["input_stages"] == 4 and ip["pair_launches"] == 6 and iu["pair_launches"] == 0
    assert torch.equal(yp, yu)
    got = CC.unpack_y(wl, yp)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = rel_err(got[i], ref[i])
        print("seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)
