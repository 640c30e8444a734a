"""Partitioned low-rank powers (§5) on the GPU, through the C ABI: the ranks
the prepare-time compression finds against the oracle's SVD ranks, and the
forward apply with PLR stages against the FP64 oracle within the floating-point
tolerance plus the a-priori bound of the truncation (each stage's power off by
at most 2 D 10^-digits in the 2-norm, carried through the stage recurrence).
"""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import workloads as W
from tests.helpers import oracle_outputs, parity_err

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
LEVELS = {64: 2, 128: 3, 256: 4}


def _pad(m):
    return 64 if m <= 64 else 128 if m <= 128 else 256


def _bound(wl, seq, eps):
    """Column-wise bound on |y_plr - y| when every stage's power is off by at
    most eps in the 2-norm: e_k <= (1 + ||P_k||) e_{k-1} + eps max_l ||v_l^(k)||,
    then ||C|| e (all stages counted, a superset of those run in PLR form)."""
    ps = wl.sets[seq.param_set]
    Abar, Bbar = (ps.A, ps.B) if wl.given else O.trapezoid(ps.A, ps.B, seq.delta)
    P = O.powers(Abar, seq.N)
    _, st = O.cascade(Abar, Bbar, ps.C, np.zeros_like(ps.D), seq.u, seq.N, return_stages=True)
    e = 0.0
    for k in range(seq.N + 1):
        e = (1 + np.linalg.norm(P[k], 2)) * e + eps * np.linalg.norm(st[k], axis=0).max()
    return np.linalg.norm(ps.C, 2) * e


def _run(wl, compute, digits, **kw):
    from paper_2411_17729_amd import cascade as CC
    plan = CC.plan_for_workload(wl, compute=compute, plr_digits=digits, **kw)
    dt = torch.float64 if compute == "f64" else torch.float32
    y = plan.apply(CC.pack_u(wl, dtype=dt))
    torch.cuda.synchronize()
    return plan, CC.unpack_y(wl, y)


def _check(wl, compute, digits, **kw):
    plan, got = _run(wl, compute, digits, **kw)
    info = plan.info()
    ref = oracle_outputs(wl)
    worst = 0.0
    for i, s in enumerate(wl.seqs):
        eps = 2 * LEVELS[_pad(wl.sets[s.param_set].m)] * 10.0 ** (-digits)
        rms = np.sqrt(np.mean(np.sum(ref[i] ** 2, axis=1)))
        allowed = TOL[compute] + _bound(wl, s, eps) / rms
        e = parity_err(got[i], ref[i])
        print(f"seq {i} m={wl.sets[s.param_set].m} L={s.L} err={e:.3e} allowed={allowed:.3e}", flush=True)
        assert e <= allowed, (i, e, allowed)
        worst = max(worst, e)
    return plan, info, got, worst


def _batched(seed, m, L, N, batch=3, pq=4):
    return W.batched(seed=seed, batch=batch, m=m, L=L, N=N, p=pq, q=pq)


@pytest.mark.parametrize("m,delta", [(256, 1e-2), (100, 3e-3)])
def test_plr_ranks_against_the_oracle(m, delta):
    """The compression's ranks are never below the SVD's (Eckart-Young), equal
    them where the powers are exactly low rank (rank 2^k for k <= 2), and mark
    blocks beyond the cap; stage 0 has rank-1 lower blocks (§5)."""
    from paper_2411_17729_amd import cascade as CC
    A, b = W.hippo_legs(m)
    rng = np.random.default_rng(4)
    C = rng.standard_normal((2, m)) / m
    D = np.zeros((2, 1))
    N, digits = 7, 10
    seq = W.Sequence(0, delta, 1024, N, None)
    layout = CC.make_layout([seq], [(m, 1, 2)])
    plan = CC.CascadePlan(layout, [(A, b[:, None], C, D)], compute="f64", plr_digits=digits)
    Abar, _ = O.trapezoid(A, b, delta)
    P = O.powers(Abar, N)
    tol = 10.0 ** (-digits)
    for k in range(N):  # stage N forms y densely
        ranks, _ = plan.plr_ranks(0, k)
        lo = O.plr_ranks(O.plr_compress(P[k], tol * 1.01, leaf=16))
        ex = O.plr_ranks(O.plr_compress(P[k], tol, leaf=16))
        for d, nodes in enumerate(lo, start=1):
            for g, pair in enumerate(nodes):
                for side in range(2):
                    r = ranks[2 * ((1 << (d - 1)) - 1) + 2 * g + side]
                    want = pair[side]
                    if want > 32:
                        assert r == 33, (k, d, g, side, r, want)
                        continue
                    assert r >= want, (k, d, g, side, r, want)
                    if k <= 2:
                        assert r == ex[d - 1][g][side], (k, d, g, side, r)
                    if k == 0:
                        assert r == (0 if side == 1 or 2 * g * (_pad(m) >> d) + (_pad(m) >> d) >= m else 1)


@pytest.mark.parametrize("compute,digits", [("f64", 12), ("f32", 7)])
def test_plr_forward_matches_the_oracle(compute, digits):
    wl = _batched(11, 256, 3000, 10)
    plan, info, got, worst = _check(wl, compute, digits, input_stages=-1)
    assert info["plr_stages"] > 0
    assert 0 < info["plr_flops"] < 0.5 * info["plr_dense_flops"]
    assert worst <= TOL[compute]  # the truncation is far below the type's tolerance


def test_plr_coarse_tolerance_stays_within_the_bound():
    """At 10^-3 the truncation is visible in the output (FP64 plan), and still
    within the bound."""
    from paper_2411_17729_amd import cascade as CC
    wl = _batched(5, 128, 2500, 9, batch=2)
    plan, info, got, worst = _check(wl, "f64", 3, input_stages=-1)
    assert info["plr_stages"] > 0
    dense = CC.plan_for_workload(wl, compute="f64", input_stages=-1)
    yd = CC.unpack_y(wl, dense.apply(CC.pack_u(wl, dtype=torch.float64)))
    torch.cuda.synchronize()
    diff = max(np.abs(g - d).max() for g, d in zip(got, yd))
    assert diff > 1e-9


def test_plr_ragged_classes_fp32():
    """Sequences of padded sizes 64, 128 and 256 with uneven lengths (tails of
    partial units, 2^k beyond some lengths): every class picks its own PLR
    stages (padded 64 none: its dense product is already cheaper)."""
    rng = np.random.default_rng(21)
    sets, seqs = [], []
    for i, (m, L) in enumerate([(64, 700), (128, 1500), (200, 333), (256, 2048), (100, 1111)]):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, 3)) / m, rng.standard_normal((2, m)) / m,
                               rng.standard_normal((2, 3)) / m))
        s = W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, 9, None)
        s.u = rng.standard_normal((L, 3))
        seqs.append(s)
    wl = W.Workload("plr_ragged", sets, seqs)
    plan, info, got, worst = _check(wl, "f32", 7, input_stages=-1)
    assert info["plr_stages"] > 0
    assert worst <= TOL["f32"]


def test_plr_general_matrix_keeps_dense_stages():
    """A random orthogonal Abar: every power is orthogonal, so its off-diagonal
    blocks keep ranks far above the cap at every stage; no stage runs in PLR
    form and the output is the dense plan's, bit for bit."""
    from paper_2411_17729_amd import cascade as CC
    rng = np.random.default_rng(3)
    m, p, q, L = 128, 2, 2, 900
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    ps = W.ParamSet(Q, rng.standard_normal((m, p)), rng.standard_normal((q, m)), rng.standard_normal((q, p)))
    seqs = []
    for _ in range(2):
        s = W.Sequence(0, 0.1, L, 8, None)
        s.u = rng.standard_normal((L, p))
        seqs.append(s)
    wl = W.Workload("orthogonal_m128", [ps], seqs, given=True)
    plan = CC.plan_for_workload(wl, compute="f32", plr_digits=6)
    assert plan.info()["plr_stages"] == 0
    ranks, used = plan.plr_ranks(0, 6)  # stages 0..5 are in the input pass
    assert not used and max(ranks) == 33
    u = CC.pack_u(wl, dtype=torch.float32)
    y1 = plan.apply(u)
    y0 = CC.plan_for_workload(wl, compute="f32").apply(u)
    torch.cuda.synchronize()
    assert torch.equal(y1, y0)


def test_plr_graph_replays():
    from paper_2411_17729_amd import cascade as CC
    wl = _batched(8, 128, 1200, 8, batch=2)
    plan = CC.plan_for_workload(wl, compute="f32", plr_digits=7, input_stages=-1)
    assert plan.info()["plr_stages"] > 0
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


def test_plr_two_sided_forms():
    """Abar = diag(lambda) + a rank-1 term: off-diagonal blocks on both sides
    of the diagonal (rank 1 at stage 0, at most 2^k later), so the stage runs
    the general path (Z of each block formed when its row range opens)."""
    rng = np.random.default_rng(12)
    m, p, q, L = 256, 2, 2, 1500  # (at padded 128 a rank-1 pair of blocks per node does not pay)
    a, b = rng.standard_normal(m), rng.standard_normal(m)
    A = np.diag(rng.uniform(0.5, 0.95, m)) + 0.05 * np.outer(a, b) / (np.linalg.norm(a) * np.linalg.norm(b))
    ps = W.ParamSet(A, rng.standard_normal((m, p)) / m, rng.standard_normal((q, m)) / m,
                    rng.standard_normal((q, p)) / m)
    seqs = []
    for _ in range(2):
        s_ = W.Sequence(0, 0.1, L, 9, None)
        s_.u = rng.standard_normal((L, p))
        seqs.append(s_)
    wl = W.Workload("two_sided_m256", [ps], seqs, given=True)
    plan, info, got, worst = _check(wl, "f32", 7, input_stages=-1)
    assert info["plr_stages"] > 0
    ranks, used = plan.plr_ranks(0, 0)
    assert used and ranks[1] == 1 and ranks[0] == 1  # level 1: lower and upper blocks of rank 1
    assert worst <= TOL["f32"]



def test_plr_from_an_initial_state():
    """apply_x0 on a plan with PLR stages: the free response enters before the
    stages, so the PLR stages carry it like any other state."""
    from paper_2411_17729_amd import cascade as CC
    rng = np.random.default_rng(31)
    sets, seqs, x0 = [], [], []
    for i, (m, L) in enumerate([(256, 2000), (200, 1300), (128, 1700)]):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, 2)) / m, rng.standard_normal((2, m)) / m,
                               np.zeros((2, 2))))
        s_ = W.Sequence(i, float(10 ** rng.uniform(-3, -1)), L, 10, None)
        s_.u = rng.standard_normal((L, 2))
        seqs.append(s_)
        x0.append(rng.standard_normal(m))
    wl = W.Workload("plr_x0", sets, seqs)
    plan = CC.plan_for_workload(wl, compute="f32", plr_digits=7, input_stages=-1, launch="per_stage")
    assert plan.info()["plr_stages"] > 0
    u = CC.pack_u(wl, dtype=torch.float32)
    xt = torch.from_numpy(np.concatenate(x0)).float().cuda()
    y = CC.unpack_y(wl, plan.apply(u, x0=xt))
    torch.cuda.synchronize()
    for i, (s_, x) in enumerate(zip(wl.seqs, x0)):
        ps = wl.sets[s_.param_set]
        Abar, Bbar = O.trapezoid(ps.A, ps.B, s_.delta)
        ref, _ = O.recursion(Abar, Bbar, ps.C, ps.D, s_.u.astype(np.float32).astype(np.float64), x0=x)
        e = parity_err(y[i], ref)
        print("seq", i, f"{e:.3e}", flush=True)
        assert e <= TOL["f32"], (i, e)


def test_plr_with_the_final_state():
    """A plan that keeps the final state (stream chunks) with PLR stages: y and
    the last row's state against the oracle's recursion."""
    from paper_2411_17729_amd import cascade as CC
    wl = _batched(14, 256, 1500, 10, batch=2)
    plan = CC.plan_for_workload(wl, compute="f32", plr_digits=7, input_stages=-1, final_state=1)
    assert plan.info()["plr_stages"] > 0
    u = CC.pack_u(wl, dtype=torch.float32)
    y, xl = plan.apply_state(u)
    torch.cuda.synchronize()
    y = CC.unpack_y(wl, y)
    xl = xl.double().cpu().numpy().reshape(len(wl.seqs), -1)
    for i, s_ in enumerate(wl.seqs):
        ps = wl.sets[s_.param_set]
        Abar, Bbar = O.trapezoid(ps.A, ps.B, s_.delta)
        ref, xs = O.recursion(Abar, Bbar, ps.C, ps.D, s_.u.astype(np.float32).astype(np.float64))
        last = np.asarray(xs)[-1]  # the state after row L - 1
        assert parity_err(y[i], ref) <= TOL["f32"]
        assert np.linalg.norm(xl[i] - last) / np.linalg.norm(last) <= TOL["f32"]


def test_plr_full_size_fp32_sampled():
    """The bench workload (16 x L = 16384, m = 256, p = q = 8, N = 13) in FP32
    with PLR stages at d = 7, two sequences against the oracle."""
    from paper_2411_17729_amd import cascade as CC
    wl = W.batched(seed=0)
    plan = CC.plan_for_workload(wl, compute="f32", plr_digits=7)
    assert plan.info()["plr_stages"] > 0
    y = CC.unpack_y(wl, plan.apply(CC.pack_u(wl, dtype=torch.float32)))
    torch.cuda.synchronize()
    for i in (0, 15):
        s_ = wl.seqs[i]
        ps = wl.sets[s_.param_set]
        Abar, Bbar = O.trapezoid(ps.A, ps.B, s_.delta)
        ref, _ = O.recursion(Abar, Bbar, ps.C, ps.D, s_.u.astype(np.float32).astype(np.float64))
        e = parity_err(y[i], ref)
        print("seq", i, f"{e:.3e}", flush=True)
        assert e <= TOL["f32"], (i, e)
