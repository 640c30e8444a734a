"""The FP64 precomputation on the GPU (trapezoid of §1 and the powers) for
lower-triangular A (blockwise triangular inverse: the HiPPO matrices of §4)
and for general A (Gauss-Jordan), at every padded size, against the oracle's
discretization and numpy's matrix powers; and the refusal of a singular
I - delta/2 A on both paths."""

import numpy as np
import pytest
import torch

import oracle as O
from paper_2411_17729_amd import binding as B
from paper_2411_17729_amd import workloads as W

pytestmark = pytest.mark.gpu


def _prepared(A, Bm, delta, N=4):
    from paper_2411_17729_amd import cascade as CC
    m, p = Bm.shape
    C = np.ones((1, m)) / m
    D = np.zeros((1, p))
    seq = W.Sequence(0, delta, 1 << (N + 1), N, None)
    layout = CC.make_layout([seq], [(m, p, 1)])
    return CC.CascadePlan(layout, [(A, Bm, C, D)], compute="f64")


def _check(A, Bm, delta, N=4, tol=1e-12):
    plan = _prepared(A, Bm, delta, N)
    Ab, Bb = O.trapezoid(A, Bm, delta)
    m = A.shape[0]
    P = np.linalg.matrix_power
    for k in range(N + 1):
        got = plan.power(0, k).cpu().numpy()
        want = P(Ab, 1 << k)
        assert np.linalg.norm(got - want) <= tol * max(1.0, np.linalg.norm(want)), k
    got_b = plan.bbar(0, m, Bm.shape[1]).cpu().numpy()
    assert np.linalg.norm(got_b - Bb) <= tol * np.linalg.norm(Bb)
    plan.close()


@pytest.mark.parametrize("m", [20, 64, 100, 200, 256])
def test_lower_triangular_hippo_and_random(m):
    A, b = W.hippo_legs(m)
    rng = np.random.default_rng(m)
    _check(A, np.c_[b, rng.standard_normal(m)], 1e-2)
    # a random lower-triangular A with a well-conditioned I - delta/2 A
    R = np.tril(rng.standard_normal((m, m))) / np.sqrt(m)
    np.fill_diagonal(R, -np.abs(np.diag(R)) - 1.0)
    _check(R, rng.standard_normal((m, 2)), 5e-2)


@pytest.mark.parametrize("m", [33, 128, 256])
def test_general_and_upper_triangular(m):
    rng = np.random.default_rng(100 + m)
    A = rng.standard_normal((m, m)) / np.sqrt(m) - 0.5 * np.eye(m)
    _check(A, rng.standard_normal((m, 3)), 5e-2)
    _check(np.triu(A), rng.standard_normal((m, 1)), 5e-2)  # not lower: Gauss-Jordan


@pytest.mark.parametrize("lower", [True, False])
def test_singular_system_is_refused(lower):
    # I - delta/2 A with a zero diagonal entry (A_33 = 2 / delta)
    m, delta = 40, 0.1
    A = -np.eye(m)
    A[3, 3] = 2.0 / delta
    if not lower:
        A[0, m - 1] = 0.3
    with pytest.raises(B.SSMError) as ei:
        _prepared(A, np.ones((m, 1)), delta)
    assert ei.value.status == B.SSM_E_NUMERIC
