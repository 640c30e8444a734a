"""Automatic N (N = -e in a descriptor: tolerance 10^-e on the Frobenius norm
of the first power the polynomial leaves out, capped where the window covers
the sequence): the N the library picks equal the oracle's, for the worked
example of §4 and for a batch of HiPPO sequences with their own step sizes,
lengths and tolerances, and the outputs equal the oracle's truncated sums
with those N (FP64 plans)."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import binding as B
from paper_2411_17729_amd import workloads as W
from tests.helpers import max_rel, oracle_outputs

pytestmark = pytest.mark.gpu


def _plan(wl, Ns, compute="f64"):
    from paper_2411_17729_amd import cascade as CC
    for s, n in zip(wl.seqs, Ns):
        s.N = n
    return CC.plan_for_workload(wl, compute=compute)


def test_auto_n_worked_example():
    # §4: HiPPO m = 100, delta = 5e-4; |P_15|_F ~ 1.0e-9 and |P_14|_F ~ 7.8e-3
    A, b = W.hippo_legs(100)
    rng = np.random.default_rng(3)
    ps = W.ParamSet(A, b[:, None], rng.standard_normal((1, 100)) / 10, np.zeros((1, 1)))
    L = 1 << 16
    u = rng.standard_normal((L, 1))
    wl = W.Workload("worked", [ps], [W.Sequence(0, 5e-4, L, -8, u), W.Sequence(0, 5e-4, L, -14, u.copy())])
    plan = _plan(wl, [-8, -14])
    got = plan.stages()
    Ab, _ = O.trapezoid(A, b[:, None], 5e-4)
    assert got == [O.auto_stages(Ab, L, 1e-8), O.auto_stages(Ab, L, 1e-14)] == [14, 15]
    for s, n in zip(wl.seqs, got):
        s.N = n
    from paper_2411_17729_amd import cascade as CC
    y = CC.unpack_y(wl, plan.apply(CC.pack_u(wl, dtype=torch.float64)))
    torch.cuda.synchronize()
    Ab, Bb = O.trapezoid(A, b[:, None], 5e-4)
    ref = [O.truncated_sum_fft(Ab, Bb, ps.C, ps.D, s.u, s.N) for s in wl.seqs]
    assert max_rel(y, ref) <= 1e-10


def test_auto_n_batch_matches_the_oracle():
    rng = np.random.default_rng(5)
    wl = W.batched(seed=6, batch=5, m=64, L=3000, N=11, p=2, q=2)
    Ls = [3000, 1025, 700, 4096, 9]
    tols = [-4, -8, -12, -6, -10]
    for s, L in zip(wl.seqs, Ls):
        s.L = L
        s.u = rng.standard_normal((L, 2))
    plan = _plan(wl, tols)
    got = plan.stages()
    want = []
    for s, e in zip(wl.seqs, tols):
        Ab, _ = O.trapezoid(wl.sets[0].A, wl.sets[0].B, s.delta)
        want.append(O.auto_stages(Ab, s.L, 10.0 ** e))
    print("chosen N", got, "oracle", want, flush=True)
    assert got == want
    for s, n in zip(wl.seqs, got):
        s.N = n
    from paper_2411_17729_amd import cascade as CC
    y = CC.unpack_y(wl, plan.apply(CC.pack_u(wl, dtype=torch.float64)))
    torch.cuda.synchronize()
    assert max_rel(y, oracle_outputs(wl)) <= 1e-10
    # the workspace sized for the caps holds the plan of the chosen N
    lay = plan.layout
    descs = [B.ssm_seq_desc(m=d.m, p=d.p, q=d.q, N=n, L=d.L, delta=d.delta, param_set=d.param_set, reserved=0,
                            u_offset=d.u_offset, y_offset=d.y_offset) for d, n in zip(lay.descs, got)]
    chosen = B.ssm_cascade_workspace_bytes(descs, B.SSM_DISC_TRAPEZOID, B.SSM_F64, 0)
    auto = B.ssm_cascade_workspace_bytes(lay.descs, B.SSM_DISC_TRAPEZOID, B.SSM_F64, 0)
    assert auto >= chosen
