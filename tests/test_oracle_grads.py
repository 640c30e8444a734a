"""Pins for the oracle's derivatives: central finite differences in FP64 on the
forward oracle (which is itself pinned in test_oracle_pins.py), plus the
dot-product (transpose) test. CPU only."""

import numpy as np
import pytest

import oracle as O
from paper_2411_17729_amd import workloads as W


def _loss(A, B, C, D, delta, u, dy, N):
    Abar, Bbar = O.trapezoid(A, B, delta)
    return float(np.sum(dy * O.truncated_sum(Abar, Bbar, C, D, u, N)))


def _fd_dir(f, X, V, h=1e-6):
    return (f(X + h * V) - f(X - h * V)) / (2 * h)


@pytest.mark.parametrize("L,N", [(24, 4), (24, 2), (9, 0)])
def test_grads_full_match_central_differences(L, N):
    rng = np.random.default_rng(L + 10 * N)
    m, p, q, delta = 5, 2, 3, 0.3
    A = rng.standard_normal((m, m)) / np.sqrt(m) - 1.2 * np.eye(m)
    B, C, D = rng.standard_normal((m, p)), rng.standard_normal((q, m)), rng.standard_normal((q, p))
    u, dy = rng.standard_normal((L, p)), rng.standard_normal((L, q))
    g = O.grads_full(A, B, C, D, delta, u, dy, N)
    args = dict(A=A, B=B, C=C, D=D, u=u)
    for name, X in args.items():
        for trial in range(3):
            V = rng.standard_normal(X.shape)

            def f(Xv, name=name):
                a = dict(args)
                a[name] = Xv
                return _loss(a["A"], a["B"], a["C"], a["D"], delta, a["u"], dy, N)

            fd = _fd_dir(f, X, V)
            an = float(np.sum(g[name] * V))
            assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (name, fd, an)


def test_bptt_equals_bruteforce_when_window_covers_sequence():
    wl = W.random_small(seed=4, m=4, p=2, q=2, L=15, N=3)
    ps, s = wl.sets[0], wl.seqs[0]
    # with and without an initial state (then also its gradient)
    for x0 in (None, np.random.default_rng(5).standard_normal(4)):
        a = O.grads_recursion(ps.A, ps.B, ps.C, ps.D, s.u, wl.dy[0], x0)
        b = O.grads_truncated_bruteforce(ps.A, ps.B, ps.C, ps.D, s.u, wl.dy[0], 3, x0)
        for k in a:
            if a[k] is None:
                assert x0 is None and b[k] is None, k
                continue
            assert np.allclose(a[k], b[k], rtol=1e-12, atol=1e-12), k


def test_truncated_grads_differ_from_bptt_when_truncating():
    wl = W.random_small(seed=4, m=4, p=2, q=2, L=40, N=2, contraction=0.99)
    ps, s = wl.sets[0], wl.seqs[0]
    a = O.grads_recursion(ps.A, ps.B, ps.C, ps.D, s.u, wl.dy[0])
    b = O.grads_truncated_bruteforce(ps.A, ps.B, ps.C, ps.D, s.u, wl.dy[0], 2)
    assert np.max(np.abs(a["Abar"] - b["Abar"])) > 1e-3


def test_dot_product_transpose_identity():
    # <dy, J du> = <J^T dy, du> for the linear map u -> y
    wl = W.random_small(seed=8, m=5, p=2, q=3, L=30, N=3)
    ps, s = wl.sets[0], wl.seqs[0]
    rng = np.random.default_rng(1)
    du = rng.standard_normal(s.u.shape)
    Jdu = O.cascade(ps.A, ps.B, ps.C, ps.D, du, 3)
    g = O.grads_truncated_bruteforce(ps.A, ps.B, ps.C, ps.D, s.u, wl.dy[0], 3)
    assert abs(np.sum(wl.dy[0] * Jdu) - np.sum(g["u"] * du)) < 1e-10


def test_trapezoid_adjoint_central_differences():
    rng = np.random.default_rng(2)
    m, p, delta = 6, 2, 0.05
    A, _ = W.hippo_legs(m)
    B = rng.standard_normal((m, p))
    gAbar, gBbar = rng.standard_normal((m, m)), rng.standard_normal((m, p))
    gA, gB = O.trapezoid_adjoint(A, B, delta, gAbar, gBbar)

    def f(Av, Bv):
        Ab, Bb = O.trapezoid(Av, Bv, delta)
        return float(np.sum(gAbar * Ab) + np.sum(gBbar * Bb))

    for _ in range(3):
        VA, VB = rng.standard_normal((m, m)), rng.standard_normal((m, p))
        fdA = _fd_dir(lambda X: f(X, B), A, VA)
        fdB = _fd_dir(lambda X: f(A, X), B, VB)
        assert abs(fdA - np.sum(gA * VA)) < 1e-8 * max(1, abs(fdA))
        assert abs(fdB - np.sum(gB * VB)) < 1e-8 * max(1, abs(fdB))
