"""BF16 state between the passes of the forward apply (split input pass, stage
pairs, tail pair): against the FP64 oracle at the BF16 bound, against the FP32
state plan, the fallback to FP32 state where some pass could not keep it,
bitwise across segment lengths, and under graph replay."""

import numpy as np
import pytest
import torch

from paper_2411_17729_amd import binding as B
from tests.helpers import parity_err
from tests.test_gpu_chain import _oracle
from tests.test_gpu_pair import _apply, _workload

pytestmark = pytest.mark.gpu

# (m, p, q, L, N): padded m 256, p = 8 (the split input pass folds stages 0-5,
# then the pairs (6, 7), (8, 9) and the tail pair (10, 11)) and padded m 128,
# p = 4 (stages 0-5 folded, (6, 7) and the tail pair (8, 9)); L not a
# multiple of 16, m below the padded size
SPEC = [(256, 8, 8, 4096, 11), (256, 8, 8, 3001, 11), (200, 8, 4, 2500, 11),
        (128, 4, 3, 1500, 9), (100, 4, 2, 1999, 9)]


def _bf16_inputs(wl, u):
    # the oracle sees the inputs the GPU sees
    flat = u.double().cpu().numpy()
    off = 0
    for s_ in wl.seqs:
        n = s_.L * wl.sets[s_.param_set].B.shape[1]
        s_.u = flat[off: off + n].reshape(s_.L, -1)
        off += n


@pytest.mark.parametrize("u_dtype", ["f32", "bf16"])
@pytest.mark.parametrize("zero_d", [True, False])
def test_bf16_state_matches_oracle(u_dtype, zero_d):
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(61, zero_d=zero_d, spec=SPEC)
    dt = torch.float32 if u_dtype == "f32" else torch.bfloat16
    u = CC.pack_u(wl, dtype=dt)
    outs = {}
    for sb in (1, 0):
        plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", state_bf16=sb, fold_stages=-1)
        info = plan.info()
        assert info["state_dtype"] == (B.SSM_BF16 if sb else B.SSM_F32)
        assert info["input_stages"] == 6 and info["pair_launches"] == 5
        outs[sb] = CC.unpack_y(wl, plan.apply(u))
        torch.cuda.synchronize()
        plan.close()
    if u_dtype == "bf16":
        _bf16_inputs(wl, u)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(outs[1][i], ref[i])
        e32 = parity_err(outs[0][i], ref[i])
        d = parity_err(outs[1][i], outs[0][i])
        print(u_dtype, "D=0" if zero_d else "D!=0", "seq", i,
              f"bf16 state {e:.2e}  fp32 state {e32:.2e}  between {d:.2e}", flush=True)
        assert e <= 2e-2, (i, e)
        # one more BF16 rounding of the state per pass: well inside the bound
        assert d <= 1e-2, (i, d)


def test_bf16_state_falls_back():
    # stage 12 of the first class runs unpaired: the plan keeps FP32 state and
    # gives what the default plan gives
    from paper_2411_17729_amd import cascade as CC
    spec = [(256, 8, 8, 5000, 12), (256, 8, 4, 4200, 12), (128, 4, 3, 1500, 9)]
    wl = _workload(62, spec=spec)
    yb, ib = _apply(wl, state_bf16=1)
    y0, i0 = _apply(wl)
    assert ib["state_dtype"] == B.SSM_F32 and i0["state_dtype"] == B.SSM_F32
    assert torch.equal(yb, y0)


def test_bf16_state_segment_lengths_bitwise():
    wl = _workload(63, spec=SPEC)
    ys = []
    for t in (4, 7, 64, 256):
        y, info = _apply(wl, state_bf16=1, pair_blocks=t)
        assert info["state_dtype"] == B.SSM_BF16
        ys.append(y)
    for y in ys[1:]:
        assert torch.equal(ys[0], y)


def test_bf16_state_graph_replays():
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(64, spec=SPEC)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", state_bf16=1, fold_stages=-1)
    assert plan.info()["state_dtype"] == B.SSM_BF16
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
    plan.close()


def test_autotuner_gates_bf16_state(tmp_path):
    # the tuner times BF16-state candidates only where the plan can keep the
    # state in BF16, and keeps one only within its tolerance of the same plan
    # with FP32 state
    from paper_2411_17729_amd import tune
    wl = _workload(65, spec=SPEC)
    path = str(tmp_path / "cache.json")
    best = tune.best_tuning(wl, compute="bf16", path=path, allow_bf16_state=True)
    (key, rec), = tune.load_cache(path).items()
    assert key.endswith("/bf16state")
    b16 = [c for c in rec["candidates"] if c["state_bf16"]]
    assert b16 and all("rel_diff" in c or "rejected" in c for c in b16)
    for c in b16:
        print("bf16-state candidate", c, flush=True)
        if "rel_diff" in c:
            assert ("ms" in c) == (c["rel_diff"] <= 5e-3)
    assert rec["ms"] == min(c["ms"] for c in rec["candidates"] if "ms" in c)
    assert best["state_bf16"] == rec["choice"]["state_bf16"]
    # a tolerance no BF16-state plan can meet leaves FP32 state
    best0, _, table0 = tune.tune(wl, "bf16", allow_bf16_state=True, tol=0.0)
    assert best0["state_bf16"] == 0
    assert all("rejected" in c for c in table0 if c["state_bf16"])
