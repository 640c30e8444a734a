"""Pins of the oracle's exponential discretization (the choice Abar = exp(delta A)
of §5, with Bbar read as the zero-order hold) and of its adjoint, against
closed forms, exact identities of the exponential and finite differences, and
planted mistakes that each must fail a pin. CPU only."""

import math

import numpy as np
import pytest

import oracle as O
from paper_2411_17729_amd import workloads as W


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


# ---- closed forms --------------------------------------------------------

def _diagonal_case(zoh):
    # diagonal A: exp acts entrywise; Bbar_i = (e^{delta l_i} - 1) / l_i B_i, and delta B_i at l_i = 0
    lam = np.array([-3.0, -0.5, 0.0, 0.25])
    B = np.arange(1.0, 9.0).reshape(4, 2)
    delta = 0.3
    Ab, Bb = zoh(np.diag(lam), B, delta)
    e = np.exp(delta * lam)
    w = np.array([(x - 1.0) / l if l != 0 else delta for x, l in zip(e, lam)])
    return _rel(Ab, np.diag(e)) < 1e-14 and _rel(Bb, w[:, None] * B) < 1e-14


def _jordan_case(zoh):
    # nilpotent A (a 3x3 Jordan block times a): the series ends after three terms
    a, delta = 1.7, 0.4
    A = a * np.diag([1.0, 1.0], k=1)
    B = np.array([[1.0, -2.0], [0.5, 3.0], [2.0, 1.0]])
    Ab, Bb = zoh(A, B, delta)
    X = delta * A
    ref_A = np.eye(3) + X + X @ X / 2.0
    ref_B = delta * (np.eye(3) + X / 2.0 + X @ X / 6.0) @ B
    return _rel(Ab, ref_A) < 1e-14 and _rel(Bb, ref_B) < 1e-14


def _rotation_case(zoh):
    # the generator of plane rotations: exp(delta A) rotates by omega delta, and
    # int_0^delta exp(sA) ds = A^{-1} (exp(delta A) - I) since A is invertible
    om, delta = 2.5, 0.7
    A = np.array([[0.0, -om], [om, 0.0]])
    B = np.array([[1.0], [2.0]])
    Ab, Bb = zoh(A, B, delta)
    c, s = math.cos(om * delta), math.sin(om * delta)
    R = np.array([[c, -s], [s, c]])
    # A^{-1} = [[0, 1/om], [-1/om, 0]]
    Ainv = np.array([[0.0, 1.0 / om], [-1.0 / om, 0.0]])
    return _rel(Ab, R) < 1e-14 and _rel(Bb, Ainv @ (R - np.eye(2)) @ B) < 1e-14


def _semigroup_case(zoh):
    # two holds of delta are one hold of 2 delta: Abar_{2d} = Abar_d^2 and
    # Bbar_{2d} = Abar_d Bbar_d + Bbar_d
    rng = np.random.default_rng(3)
    A, b = W.hippo_legs(12)
    B = np.concatenate([b[:, None], rng.standard_normal((12, 2))], axis=1)
    d = 0.02
    A1, B1 = zoh(A, B, d)
    A2, B2 = zoh(A, B, 2 * d)
    return _rel(A2, A1 @ A1) < 1e-12 and _rel(B2, A1 @ B1 + B1) < 1e-12


def _hippo_diagonal_case(zoh):
    # HiPPO-LegS is lower triangular, so exp(delta A) is too and its diagonal is
    # exp(delta A_nn) = exp(-delta (n + 1)) (eq. (4.1), 1-based)
    A, b = W.hippo_legs(40)
    delta = 5e-3
    Ab, _ = zoh(A, b, delta)
    n = np.arange(1, 41, dtype=float)
    return (np.max(np.abs(np.triu(Ab, 1))) == 0.0
            and np.max(np.abs(np.diag(Ab) - np.exp(-delta * (n + 1))) / np.exp(-delta * (n + 1))) < 1e-13)


CASES = {"diagonal": _diagonal_case, "jordan": _jordan_case, "rotation": _rotation_case,
         "semigroup": _semigroup_case, "hippo_diagonal": _hippo_diagonal_case}


@pytest.mark.parametrize("case", sorted(CASES))
def test_zoh_pins(case):
    assert CASES[case](O.zoh)


def test_zoh_agrees_with_trapezoid_to_third_order():
    # the trapezoidal Abar is the (1,1) Pade approximant of exp(delta A), and its
    # Bbar = delta (I - delta/2 A)^{-1} B matches delta (I + delta A/2 + delta^2 A^2/6 ...) B
    # to second order: both differences shrink by 8 when delta halves
    rng = np.random.default_rng(4)
    A = rng.standard_normal((6, 6))
    B = rng.standard_normal((6, 2))
    errs = []
    for d in (0.02, 0.01, 0.005):
        Az, Bz = O.zoh(A, B, d)
        At, Bt = O.trapezoid(A, B, d)
        errs.append((np.linalg.norm(Az - At), np.linalg.norm(Bz - Bt)))
    for (a0, b0), (a1, b1) in zip(errs, errs[1:]):
        assert 7.5 < a0 / a1 < 8.5 and 7.5 < b0 / b1 < 8.5, errs


def test_zoh_bbar_is_the_hold_integral():
    # Bbar = int_0^delta exp(sA) ds B by Gauss-Legendre quadrature of the
    # integrand (each exp(sA) by the eigendecomposition of a symmetric A)
    rng = np.random.default_rng(5)
    S = rng.standard_normal((5, 5))
    A = -(S @ S.T) / 5.0
    B = rng.standard_normal((5, 2))
    delta = 0.8
    w, V = np.linalg.eigh(A)
    xs, ws = np.polynomial.legendre.leggauss(30)
    integral = np.zeros((5, 5))
    for x, wt in zip(xs, ws):
        s = 0.5 * delta * (x + 1.0)
        integral += 0.5 * delta * wt * (V * np.exp(s * w)) @ V.T
    Ab, Bb = O.zoh(A, B, delta)
    assert _rel(Ab, (V * np.exp(delta * w)) @ V.T) < 1e-13
    assert _rel(Bb, integral @ B) < 1e-13


# ---- the adjoint -----------------------------------------------------------

def _fd_dir(f, X, V, h=1e-6):
    return (f(X + h * V) - f(X - h * V)) / (2 * h)


def test_zoh_adjoint_central_differences():
    rng = np.random.default_rng(6)
    m, p, delta = 6, 2, 0.05
    A, _ = W.hippo_legs(m)
    B = rng.standard_normal((m, p))
    gAbar, gBbar = rng.standard_normal((m, m)), rng.standard_normal((m, p))
    gA, gB = O.zoh_adjoint(A, B, delta, gAbar, gBbar)

    def f(Av, Bv):
        Ab, Bb = O.zoh(Av, Bv, delta)
        return float(np.sum(gAbar * Ab) + np.sum(gBbar * Bb))

    for _ in range(3):
        VA, VB = rng.standard_normal((m, m)), rng.standard_normal((m, p))
        fdA = _fd_dir(lambda X: f(X, B), A, VA)
        fdB = _fd_dir(lambda X: f(A, X), B, VB)
        assert abs(fdA - np.sum(gA * VA)) < 1e-8 * max(1, abs(fdA))
        assert abs(fdB - np.sum(gB * VB)) < 1e-8 * max(1, abs(fdB))


def test_zoh_adjoint_diagonal_closed_form():
    # diagonal A, gradient on the diagonal of Abar only: d/dl e^{delta l} = delta e^{delta l}
    lam = np.array([-1.0, -0.3, 0.2])
    B = np.ones((3, 1))
    delta = 0.5
    g = np.array([0.7, -1.1, 2.0])
    gA, gB = O.zoh_adjoint(np.diag(lam), B, delta, np.diag(g), np.zeros((3, 1)))
    assert _rel(np.diag(gA), g * delta * np.exp(delta * lam)) < 1e-13
    assert np.max(np.abs(gB)) < 1e-15


def test_grads_full_zoh_central_differences():
    # end to end: sum(dy * y) of the cascade after the exponential discretization
    wl = W.random_small(seed=9, m=5, p=2, q=3, L=24, N=3, delta=0.1)
    ps, s = wl.sets[0], wl.seqs[0]
    dy = wl.dy[0]
    g = O.grads_full(ps.A, ps.B, ps.C, ps.D, s.delta, s.u, dy, N=3, disc="zoh")

    def f(A, B):
        Ab, Bb = O.zoh(A, B, s.delta)
        return float(np.sum(dy * O.cascade(Ab, Bb, ps.C, ps.D, s.u, 3)))

    rng = np.random.default_rng(7)
    for _ in range(2):
        VA, VB = rng.standard_normal(ps.A.shape), rng.standard_normal(ps.B.shape)
        fdA = _fd_dir(lambda X: f(X, ps.B), ps.A, VA)
        fdB = _fd_dir(lambda X: f(ps.A, X), ps.B, VB)
        assert abs(fdA - np.sum(g["A"] * VA)) < 1e-7 * max(1, abs(fdA))
        assert abs(fdB - np.sum(g["B"] * VB)) < 1e-7 * max(1, abs(fdB))


# ---- planted mistakes ------------------------------------------------------

def _mutant(bug):
    from scipy.linalg import expm

    def zoh(A, B, delta):
        A = np.asarray(A, float)
        B = np.asarray(B, float)
        if B.ndim == 1:
            B = B[:, None]
        m, p = A.shape[0], B.shape[1]
        E = np.zeros((m + p, m + p))
        E[:m, :m] = delta * (A.T if bug == "transposed" else A)
        E[:m, m:] = B if bug == "no_delta_on_b" else delta * B
        F = expm(E)
        Ab, Bb = F[:m, :m], F[:m, m:]
        if bug == "printed_literally":  # (delta A)^{-1}[exp(delta A) - I] delta A applied to B
            Bb = (Ab - np.eye(m)) @ B
        if bug == "half_step":
            Ab = expm(0.5 * delta * A)
        return Ab, Bb
    return zoh


def test_oracle_zoh_passes_pins():
    assert all(case(O.zoh) for case in CASES.values())


@pytest.mark.parametrize("bug", ["transposed", "no_delta_on_b", "printed_literally", "half_step"])
def test_zoh_mutant_is_caught(bug):
    assert not all(case(_mutant(bug)) for case in CASES.values())
