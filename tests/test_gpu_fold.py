"""Output pass with the last stages folded in: y_l = sum_{j < 2^s} G_j x_{l - j 2^k0}
+ D u_l, G_j = C Abar^(j 2^k0). Against the FP64 oracle at the BF16 bound,
against the same plan with every stage run (pairs and the tail pair), for
each fold depth, with BF16 state, under graph replay, at the limits of q and p
and with the accounting of plan_info."""

import math

import numpy as np
import pytest
import torch

from paper_2411_17729_amd import binding as B
from tests.helpers import parity_err
from tests.test_gpu_chain import _oracle
from tests.test_gpu_pair import _workload

pytestmark = pytest.mark.gpu

# (m, p, q, L, N): padded m 256 (input pass to stage 5, then q <= 8: the fold
# of 6..11, 64 lags of 64 rows in two ranges) and 128 (input pass to stage 5,
# the fold of 6..9); L not a multiple of 16, m below the padded size
SPEC = [(256, 8, 8, 4096, 11), (256, 8, 8, 3001, 11), (200, 8, 4, 2500, 11),
        (128, 4, 3, 1500, 9), (100, 4, 2, 1999, 9)]


def _run(wl, u_dtype="f32", **kw):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage", **kw)
    info = plan.info()
    dt = torch.float32 if u_dtype == "f32" else torch.bfloat16
    u = CC.pack_u(wl, dtype=dt)
    y = CC.unpack_y(wl, plan.apply(u))
    torch.cuda.synchronize()
    plan.close()
    return y, info, u


def _bf16_inputs(wl, u):
    flat = u.double().cpu().numpy()
    off = 0
    for s_ in wl.seqs:
        n = s_.L * wl.sets[s_.param_set].B.shape[1]
        s_.u = flat[off: off + n].reshape(s_.L, -1)
        off += n


@pytest.mark.parametrize("u_dtype", ["f32", "bf16"])
@pytest.mark.parametrize("zero_d", [True, False])
def test_fold_matches_oracle(u_dtype, zero_d):
    wl = _workload(71, zero_d=zero_d, spec=SPEC)
    y, info, u = _run(wl, u_dtype)
    yu, iu, _ = _run(wl, u_dtype, fold_stages=-1)
    print("fold stages", info["fold_stages"], "launches", info["fold_launches"], "pairs",
          info["pair_launches"], flush=True)
    assert info["fold_stages"] == 6 and info["fold_launches"] == 2 and info["pair_launches"] == 0
    assert iu["fold_launches"] == 0 and iu["pair_launches"] == 5
    if u_dtype == "bf16":
        _bf16_inputs(wl, u)
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e, eu, d = parity_err(y[i], ref[i]), parity_err(yu[i], ref[i]), parity_err(y[i], yu[i])
        print(u_dtype, "D=0" if zero_d else "D!=0", "seq", i,
              f"fold {e:.2e}  stages {eu:.2e}  between {d:.2e}", flush=True)
        assert e <= 2e-2, (i, e)
        # the two differ by the BF16 roundings of the stages the fold replaces
        assert d <= 5e-3, (i, d)


# fold depths: (spec, tuning, expected (fold_stages, fold k0 of the class))
DEPTHS = {
    # padded m 256, last stage 13, input pass to 5: q <= 8 takes s = 6 at k0 =
    # 8 after the pair (6, 7); s = 4 at k0 = 10 after the pairs (6, 7), (8, 9);
    # s = 2 at k0 = 12 after three pairs; q = 9 stops at s = 4
    "s6": ([(256, 8, 8, 9000, 13), (230, 8, 5, 8500, 13)], {}, 6),
    "s4": ([(256, 8, 8, 9000, 13), (230, 8, 5, 8500, 13)], {"fold_stages": 4}, 4),
    "s4_q9": ([(256, 8, 9, 9000, 13), (230, 8, 5, 8500, 13)], {}, 4),
    "s2": ([(256, 8, 8, 9000, 13), (230, 8, 5, 8500, 13)], {"fold_stages": 2}, 2),
    # padded m 128, last stage 10: s = 5 at k0 = 6, 32 lags of 64 rows
    "s5": ([(128, 4, 3, 2000, 10), (90, 4, 16, 1100, 10)], {}, 5),
    # pairs off: s = 3 at k0 = 10 after single stages 6..9
    "s3_no_pairs": ([(256, 8, 8, 5000, 12), (256, 8, 2, 4800, 12)], {"fold_stages": 3, "pair_stages": 1}, 3),
    # s = 6 at k0 = 6 straight after the input pass; columns of 33 to 47
    # blocks (the range from lag 32 reads the 1 to 15 blocks that reach it)
    "s6_short": ([(256, 8, 8, 3001, 11), (256, 8, 1, 2100, 11), (200, 8, 7, 2500, 11)], {}, 6),
}


@pytest.mark.parametrize("case", sorted(DEPTHS))
def test_fold_depths(case):
    spec, kw, s = DEPTHS[case]
    wl = _workload(72, spec=spec)
    y, info, _ = _run(wl, **kw)
    assert info["fold_stages"] == s, info["fold_stages"]
    assert info["fold_launches"] == 1
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(y[i], ref[i])
        print(case, "seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)


def test_fold_bf16_state():
    wl = _workload(73, spec=SPEC)
    yb, ib, _ = _run(wl, state_bf16=1)
    yf, if_, _ = _run(wl)
    assert ib["state_dtype"] == B.SSM_BF16 and ib["fold_launches"] == 2
    assert if_["state_dtype"] == B.SSM_F32
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e, d = parity_err(yb[i], ref[i]), parity_err(yb[i], yf[i])
        print("seq", i, f"bf16 state {e:.2e} between {d:.2e}", flush=True)
        assert e <= 2e-2 and d <= 1e-2, (i, e, d)


@pytest.mark.parametrize("p", [8, 64])
def test_fold_six_long_memory(p):
    # small step (long memory): G_j for j >= 32 of the six-stage fold (lags
    # 2048 .. 4032 at k0 = 6) are far from zero, and with D = 0 the rows they
    # reach (l >= 2048) carry only the state part, checked on their own
    from paper_2411_17729_amd import workloads as W
    rng = np.random.default_rng(75)
    m, q, L, N = 256, 8, 3000, 11
    A, _ = W.hippo_legs(m)
    ps = W.ParamSet(A, rng.standard_normal((m, p)) / math.sqrt(m), rng.standard_normal((q, m)) / math.sqrt(m),
                    np.zeros((q, p)))
    wl = W.Workload("fold6", [ps], [W.Sequence(0, 1e-3, L, N, rng.standard_normal((L, p)))])
    y, info, _ = _run(wl)
    assert info["fold_stages"] == 6 and info["fold_launches"] == 1
    ref = _oracle(wl)[0]
    late = parity_err(y[0][2048:], ref[2048:])
    print("p", p, "rel", f"{parity_err(y[0], ref):.2e}", "rows from 2048", f"{late:.2e}", flush=True)
    assert late <= 2e-2 and parity_err(y[0], ref) <= 2e-2


@pytest.mark.parametrize("case", ["q16_p64", "q1_p1", "q8_p64", "p65"])
def test_fold_limits(case):
    # q = 16 and p = 64 (the largest the fold takes), q = p = 1 and q = 8, p = 64
    # (six stages), and p = 65, where the class keeps its tail pair
    spec = {"q16_p64": [(256, 64, 16, 3000, 11), (250, 64, 16, 2100, 11)],
            "q1_p1": [(256, 1, 1, 3000, 11), (256, 1, 1, 2050, 11)],
            "q8_p64": [(256, 64, 8, 3000, 11), (256, 64, 8, 2050, 11)],
            "p65": [(256, 65, 4, 3000, 11), (256, 65, 4, 2500, 11)]}[case]
    wl = _workload(74, spec=spec)
    y, info, _ = _run(wl)
    assert info["fold_launches"] == (0 if case == "p65" else 1), info["fold_launches"]
    ref = _oracle(wl)
    for i in range(len(wl.seqs)):
        e = parity_err(y[i], ref[i])
        print(case, "seq", i, f"{e:.2e}", flush=True)
        assert e <= 2e-2, (i, e)


def test_fold_graph_replays():
    from paper_2411_17729_amd import cascade as CC
    wl = _workload(75, spec=SPEC)
    plan = CC.plan_for_workload(wl, compute="bf16", launch="per_stage")
    assert plan.info()["fold_launches"] == 2
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


def test_fold_plan_accounting():
    # one read of every state row and one write of y; 2 q m flops per row and
    # lag, with min(2^s, l / 2^k0 + 1) lags at row l
    wl = _workload(76, spec=SPEC)
    _, info, _ = _run(wl)
    nbytes = flops = 0.0
    for s_ in wl.seqs:
        m, q = wl.sets[s_.param_set].m, wl.sets[s_.param_set].C.shape[0]
        k0, nl = 6, 64 if m > 128 else 16  # six stages at padded m 256 (q <= 8), four at 128
        nbytes += s_.L * (4 * m + 4 * q)
        lags = np.minimum(nl, np.arange(s_.L) // (1 << k0) + 1)
        flops += 2.0 * q * m * float(lags.sum())
    assert math.isclose(info["fold_bytes"], nbytes, rel_tol=1e-12)
    assert math.isclose(info["fold_flops"], flops, rel_tol=1e-12)


def test_fold_depth_within_the_narrow_kernel():
    # p = q = 1 at m = 256: the resident input pass folds stages 0-7, so with
    # N = 14 a six-stage fold would leave stage 8 unpaired; the planner must
    # then pick a depth the four-column kernel takes (at most 4 at m = 256),
    # not five
    from paper_2411_17729_amd import workloads as W
    wl = W.batched(seed=8, batch=1, m=256, L=20000, N=14, p=1, q=1)
    y, info, u = _run(wl)
    print("fold stages", info["fold_stages"], "input stages", info["input_stages"], flush=True)
    assert info["input_stages"] == 8 and 2 <= info["fold_stages"] <= 4
    ref = _oracle(wl)
    e = max(parity_err(g, r) for g, r in zip(y, ref))
    assert e <= 2e-2, e


# The six-stage fold with BF16 state over a range of input widths. (m, p, q,
# L, N, u type), each a plan with the split input pass, so that the state can
# be BF16: odd L, p = 16, p = 4 in BF16 (16-byte pieces of u straddle rows),
# q not a multiple of 4 (scalar y stores), and p = 32.
STREAM_SPEC = [(256, 16, 8, 8191, 12, "f32"), (256, 16, 3, 8191, 12, "bf16"), (256, 4, 5, 20001, 14, "bf16"),
               (256, 8, 5, 12001, 13, "f32"), (250, 32, 8, 4001, 11, "f32")]


@pytest.mark.parametrize("spec", STREAM_SPEC, ids=lambda s: "m{}_p{}_q{}_L{}_N{}_{}".format(*s))
def test_fold_bf16_state_input_widths(spec):
    from paper_2411_17729_amd import workloads as W
    m, p, q, L, N, ut = spec
    wl = W.batched(seed=81 + p, batch=2, m=m, L=L, N=N, p=p, q=q)
    y, info, u = _run(wl, ut, state_bf16=1)
    print("spec", spec, "fold", info["fold_stages"], "state", info["state_dtype"], flush=True)
    assert info["fold_stages"] == 6 and info["state_dtype"] == B.SSM_BF16
    if ut == "bf16":
        _bf16_inputs(wl, u)
    ref = _oracle(wl)
    e = max(parity_err(g, r) for g, r in zip(y, ref))
    Dref = [r - s.u.astype(np.float32).astype(np.float64) @ wl.sets[0].D.T for r, s in zip(ref, wl.seqs)]
    Dgot = [g - s.u.astype(np.float32).astype(np.float64) @ wl.sets[0].D.T for g, s in zip(y, wl.seqs)]
    e_x = max(parity_err(g, r) for g, r in zip(Dgot, Dref))
    print("rel err y", e, "state part", e_x, flush=True)
    assert e <= 2e-2 and e_x <= 2e-2, (e, e_x)
    # D u row by row near the end of each sequence (the inputs' last pieces)
    for g_, r_ in zip(y, ref):
        assert np.allclose(g_[-40:], r_[-40:], rtol=0, atol=2e-2 * np.abs(r_).max())
