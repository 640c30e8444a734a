"""The exponential discretization (Abar = exp(delta A) of §5, Bbar the
zero-order hold) on the GPU, through the C ABI: Abar, Bbar and the powers
against the FP64 oracle, the cascade on them against the oracle's recursion
or truncated sum at the FP64, FP32 and BF16 bounds, the host-side refusal of
a non-finite norm, and the gradients through it against the oracle's and
against central finite differences of the FP64 GPU forward."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import binding as B
from paper_2411_17729_amd import workloads as W
from tests.helpers import max_rel, oracle_outputs, state_part

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def _plan(wl, compute, **kw):
    from paper_2411_17729_amd import cascade as CC
    return CC.plan_for_workload(wl, compute=compute, disc="zoh", **kw)


def _rel_max(g, r):
    return float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))


# (label, A, B, delta): HiPPO-LegS at the bench, worked-example and c1 steps,
# a random stable matrix with p = 3, and one with a large norm (many squarings)
def _cases():
    rng = np.random.default_rng(11)
    out = []
    for m, delta in ((256, 1e-3), (256, 1e-1), (100, 5e-4), (64, 1e-2)):
        A, b = W.hippo_legs(m)
        out.append((f"hippo_m{m}_d{delta:g}", A, b[:, None], delta))
    S = rng.standard_normal((100, 100)) / 10.0
    out.append(("random_m100_p3", S - 1.5 * np.eye(100), rng.standard_normal((100, 3)), 0.05))
    A, b = W.hippo_legs(128)
    out.append(("hippo_m128_d5", A, np.concatenate([b[:, None], rng.standard_normal((128, 3))], 1), 5.0))
    return out


@pytest.mark.parametrize("case", range(6))
def test_zoh_abar_bbar_and_powers(case):
    from paper_2411_17729_amd import cascade as CC
    label, A, Bm, delta = _cases()[case]
    m, p = Bm.shape
    N = 6
    C = np.ones((1, m)) / m
    D = np.zeros((1, p))
    seq = W.Sequence(0, delta, 200, N, None)
    layout = CC.make_layout([seq], [(m, p, 1)])
    plan = CC.CascadePlan(layout, [(A, Bm, C, D)], compute="f64", disc="zoh")
    Abar, Bbar = O.zoh(A, Bm, delta)
    P = O.powers(Abar, N)
    ea = _rel_max(plan.power(0, 0).cpu().numpy(), Abar)
    eb = _rel_max(plan.bbar(0, m, p).cpu().numpy(), Bbar)
    ep = [_rel_max(plan.power(0, k).cpu().numpy(), P[k]) for k in range(N + 1)]
    # FP64 on both sides, by different methods (Taylor steps and s squarings
    # here, scipy's Pade approximant with its own scaling there). A rounding
    # error before t remaining squarings grows up to 2^t times (first order),
    # so the bound scales with 2^s, s the squarings of the scaling to norm 1/2;
    # Abar^(2^k) adds another factor 2^k.
    E = np.zeros((m + p, m + p))
    E[:m, :m], E[:m, m:] = delta * A, delta * Bm
    nrm = max(np.abs(E).sum(0).max(), np.abs(E).sum(1).max())
    sq = max(0, int(np.ceil(np.log2(nrm / 0.5))))
    tol = max(2.0 ** sq, 64.0) * 2 * np.finfo(float).eps
    print(f"{label}: s {sq} tol {tol:.1e}  Abar {ea:.2e} Bbar {eb:.2e} powers {max(ep):.2e}", flush=True)
    assert ea < tol and eb < tol, (ea, eb, tol)
    assert all(e < (1 << k) * tol for k, e in enumerate(ep)), (ep, tol)


@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_zoh_plain_hippo_m64_L4096(compute):
    from paper_2411_17729_amd import cascade as CC
    wl = W.plain_fp64(seed=0)
    plan = _plan(wl, compute)
    u = CC.pack_u(wl, dtype=torch.float64 if compute == "f64" else torch.float32)
    got = CC.unpack_y(wl, plan.apply(u))
    torch.cuda.synchronize()
    ref = oracle_outputs(wl, disc="zoh")
    e_y = max_rel(got, ref)
    e_x = max_rel(state_part(wl, got), state_part(wl, ref))
    print(f"zoh plain {compute}: y {e_y:.2e} state {e_x:.2e}", flush=True)
    assert e_y <= TOL[compute] and e_x <= TOL[compute], (e_y, e_x)


@pytest.mark.parametrize("compute", ["f32", "bf16"])
def test_zoh_batched_per_sequence_delta(compute):
    # one operator per step size: the discretization runs for each
    from paper_2411_17729_amd import cascade as CC
    wl = W.batched(seed=3, batch=4, L=2048, N=10, m=128, p=4, q=4)
    plan = _plan(wl, compute)
    u = CC.pack_u(wl, dtype=torch.float32)
    got = CC.unpack_y(wl, plan.apply(u))
    torch.cuda.synchronize()
    ref = oracle_outputs(wl, disc="zoh")
    e_y = max_rel(got, ref)
    e_x = max_rel(state_part(wl, got), state_part(wl, ref))
    print(f"zoh batched {compute}: y {e_y:.2e} state {e_x:.2e}", flush=True)
    assert e_y <= TOL[compute] and e_x <= TOL[compute], (e_y, e_x)


def test_zoh_differs_from_trapezoid():
    # the two discretizations give different operators (a plan that ignored
    # the choice would pass the tests above only by accident)
    from paper_2411_17729_amd import cascade as CC
    wl = W.plain_fp64(seed=0)
    pz = _plan(wl, "f64")
    pt = CC.plan_for_workload(wl, compute="f64")
    d = _rel_max(pz.power(0, 0).cpu().numpy(), pt.power(0, 0).cpu().numpy())
    assert d > 1e-8, d


def test_zoh_rejects_nonfinite():
    from paper_2411_17729_amd import cascade as CC
    m, p = 8, 1
    A = -np.eye(m)
    A[2, 3] = np.nan
    seq = W.Sequence(0, 0.1, 64, 3, None)
    layout = CC.make_layout([seq], [(m, p, 1)])
    with pytest.raises(B.SSMError) as ei:
        CC.CascadePlan(layout, [(A, np.ones((m, p)), np.ones((1, m)), np.zeros((1, p)))], compute="f32",
                       disc="zoh")
    assert ei.value.status == B.SSM_E_NUMERIC and "non-finite" in str(ei.value)


# ---- the backward through the exponential ----------------------------------

@pytest.mark.parametrize("compute", ["f64", "f32", "bf16"])
def test_zoh_backward_matches_oracle(compute):
    from tests.test_gpu_backward import _compare
    wl = W.backward(seed=1, batch=3, m=24, L=300, N=8, p=2, q=3, delta=2e-2)
    _compare(wl, compute, disc="zoh")


def test_zoh_backward_per_sequence_delta_and_classes():
    # operators of two size classes, one step size per sequence, a large step
    # (several squarings in the adjoint)
    from tests.test_gpu_backward import _compare
    rng = np.random.default_rng(21)
    sets, seqs = [], []
    for i, (m, p, q, L, N, d) in enumerate([(40, 3, 2, 257, 8, 1e-2), (40, 3, 2, 200, 7, 0.3),
                                            (130, 4, 3, 96, 6, 5e-3)]):
        A, _ = W.hippo_legs(m)
        sets.append(W.ParamSet(A, rng.standard_normal((m, p)) / m, rng.standard_normal((q, m)) / m,
                               rng.standard_normal((q, p))))
        s = W.Sequence(i, d, L, N, None)
        s.u = rng.standard_normal((L, p))
        seqs.append(s)
    dy = [rng.standard_normal((s.L, sets[s.param_set].q)) for s in seqs]
    wl = W.Workload("zoh_ragged", sets, seqs, dy=dy)
    _compare(wl, "f64", disc="zoh")


def test_zoh_backward_finite_differences_fp64_gpu():
    # central differences (h = 1e-6) of <dy, y> through the FP64 GPU forward
    # with the exponential discretization
    from paper_2411_17729_amd import cascade as CC
    from tests.test_gpu_backward import _gpu_grads
    wl = W.backward(seed=6, batch=2, m=32, L=400, N=8, p=2, q=2, delta=5e-2)
    ps = wl.sets[0]
    _, gs, _, _ = _gpu_grads(wl, "f64", wl.dy, disc="zoh")
    dyt = np.concatenate([d.reshape(-1) for d in wl.dy])
    rng = np.random.default_rng(0)

    def f(A, Bm):
        w2 = W.Workload("fd", [W.ParamSet(A, Bm, ps.C, ps.D)], wl.seqs)
        plan = CC.plan_for_workload(w2, compute="f64", disc="zoh")
        y = plan.apply(CC.pack_u(w2, dtype=torch.float64)).cpu().numpy()
        return float(np.dot(dyt, y))

    h = 1e-6
    for j, (name, X) in enumerate((("A", ps.A), ("B", ps.B))):
        V = rng.standard_normal(X.shape)
        args_p = [ps.A, ps.B]
        args_m = [ps.A, ps.B]
        args_p[j] = X + h * V
        args_m[j] = X - h * V
        fd = (f(*args_p) - f(*args_m)) / (2 * h)
        an = float(np.sum(gs[0][j] * V))
        print(name, fd, an, flush=True)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, fd, an)
