"""Pins for the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests touch a GPU. Each pin compares the oracle with something
other than itself: numbers printed in the paper (tests/golden), closed forms,
library routines (scipy.signal.lfilter, numpy.convolve, scipy.linalg.expm,
numpy.linalg.matrix_power), brute force on tiny inputs, and the Lemma of §2.
"""

import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest
import scipy.linalg
import scipy.signal

import oracle as O
from paper_2411_17729_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _bruteforce_truncated(Abar, Bbar, C, D, u, N):
    """y_l = sum_{j<=min(l,T-1)} C Abar^j Bbar u_{l-j} + D u_l with matrix_power."""
    T = 1 << (N + 1)
    L = u.shape[0]
    y = np.zeros((L, C.shape[0]))
    for l in range(L):
        y[l] = D @ u[l]
        for j in range(min(l, T - 1) + 1):
            y[l] += C @ np.linalg.matrix_power(Abar, j) @ Bbar @ u[l - j]
    return y


def _rand_system(rng, m, p, q, gamma=0.9):
    A = rng.standard_normal((m, m))
    A *= gamma / np.linalg.norm(A, 2)
    return A, rng.standard_normal((m, p)), rng.standard_normal((q, m)), rng.standard_normal((q, p))


# ---------------------------------------------------------------- §4 example
def test_worked_example_hippo_m100():
    g = json.load(open(os.path.join(GOLDEN, "hippo_m100_worked_example.json")))
    A, b = W.hippo_legs(g["m"], one_based=True)
    Abar, _ = O.trapezoid(A, b, g["delta"])
    d = np.diag(Abar)
    # the matrix stays lower triangular, so its diagonal holds the eigenvalues
    assert np.allclose(np.triu(Abar, 1), 0.0, atol=0.0)
    assert abs(d.max() - g["d_first"]) < 1e-15
    assert abs(d.min() - g["d_last"]) < 1e-15
    assert abs(d[0] - g["d_first"]) < 1e-15 and abs(d[-1] - g["d_last"]) < 1e-15
    P = O.powers(Abar, 15)
    assert abs(P[15][0, 0] / g["d_first_pow_2_15"] - 1.0) < g["d_first_pow_2_15_printed_rel_accuracy"]
    # exact value: the triangular matrix's first diagonal entry is (1 - delta)/(1 + delta)
    # (A_11 = -2), raised to 2^15 in 50-digit decimal arithmetic
    getcontext().prec = 50
    dex = (Decimal(1) - Decimal(repr(g["delta"]))) / (Decimal(1) + Decimal(repr(g["delta"])))
    assert abs(P[15][0, 0] / float(dex ** 32768) - 1.0) < 1e-10
    # the paper's N: the smallest N with d_first^(2^(N+1)) below 1e-14
    N = next(n for n in range(40) if d[0] ** (2 ** (n + 1)) < 1e-14)
    assert N == g["N"] and 2 ** (N + 1) - 1 == g["degree"] and N + 1 == g["matvecs"]
    # powers agree with an independent evaluation to the accuracy the paper quotes
    ref = np.linalg.matrix_power(Abar, 2 ** 10)
    assert np.max(np.abs(P[10] - ref)) < g["powers_accuracy"] * max(1.0, np.max(np.abs(ref)))


def test_worked_example_rejects_zero_based_hippo():
    g = json.load(open(os.path.join(GOLDEN, "hippo_m100_worked_example.json")))
    A, b = W.hippo_legs(g["m"], one_based=False)
    d = np.diag(O.trapezoid(A, b, g["delta"])[0])
    assert abs(d.max() - g["d_first"]) > 1e-6


def test_hippo_generator_by_hand():
    A, b = W.hippo_legs(3)
    s = math.sqrt
    ref = -np.array([[2.0, 0.0, 0.0], [s(5) * s(3), 3.0, 0.0], [s(7) * s(3), s(7) * s(5), 4.0]])
    assert np.allclose(A, ref, rtol=0, atol=1e-15)
    assert np.allclose(b, [s(3), s(5), s(7)], rtol=0, atol=1e-15)


# ---------------------------------------------------------- discretization
def test_trapezoid_diagonal_closed_form():
    a = np.array([-0.5, -3.0, -40.0, 0.2])
    bvec = np.array([1.0, -2.0, 0.5, 3.0])
    dt = 0.01
    Abar, Bbar = O.trapezoid(np.diag(a), bvec, dt)
    h = dt / 2
    assert np.allclose(Abar, np.diag((1 + h * a) / (1 - h * a)), rtol=1e-15, atol=1e-16)
    assert np.allclose(Bbar[:, 0], dt * bvec / (1 - h * a), rtol=1e-15, atol=1e-16)


def test_trapezoid_is_second_order_in_delta():
    # (I - hA)^{-1}(I + hA) is the (1,1) Pade approximant of exp(delta A):
    # its error is O(delta^3), so halving delta divides it by about 8.
    rng = np.random.default_rng(3)
    A = rng.standard_normal((5, 5)) - 2 * np.eye(5)
    errs = []
    for dt in (0.02, 0.01, 0.005):
        Abar, _ = O.trapezoid(A, np.ones((5, 1)), dt)
        errs.append(np.linalg.norm(Abar - scipy.linalg.expm(dt * A)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 7.0 < r1 < 9.0 and 7.0 < r2 < 9.0


def test_trapezoid_identity_and_contraction_for_hippo():
    # I + Abar = 2 (I - delta/2 A)^{-1}; for HiPPO A + A^T is negative definite,
    # so the Cayley transform is a strict contraction (spectral norm < 1).
    for m, dt in ((64, 1e-2), (100, 5e-4), (256, 1e-1)):
        A, b = W.hippo_legs(m)
        Abar, _ = O.trapezoid(A, b, dt)
        Mi = np.linalg.inv(np.eye(m) - 0.5 * dt * A)
        assert np.max(np.abs(np.eye(m) + Abar - 2 * Mi)) < 1e-12
        assert np.linalg.norm(Abar, 2) < 1.0


# --------------------------------------------------------- cascade algebra
@pytest.mark.parametrize("N", [0, 1, 2, 3, 4])
def test_telescoping_product(N):
    # prod_{k=0}^{N} (I + X^(2^k)) = sum_{j < 2^(N+1)} X^j  (the basis of eq. (2.2))
    rng = np.random.default_rng(N)
    X = rng.standard_normal((4, 4)) * 0.4
    P = O.powers(X, N)
    prod = np.eye(4)
    for k in range(N + 1):
        prod = prod @ (np.eye(4) + P[k])
    ref = sum(np.linalg.matrix_power(X, j) for j in range(2 ** (N + 1)))
    assert np.max(np.abs(prod - ref)) < 1e-12 * max(1, np.max(np.abs(ref)))


CASES = [
    # (m, p, q, L, N)
    (1, 1, 1, 1, 0), (2, 1, 1, 8, 2), (3, 2, 1, 17, 1), (4, 1, 2, 16, 3),
    (5, 2, 3, 33, 2), (6, 3, 2, 64, 5), (6, 2, 2, 40, 0), (3, 1, 1, 9, 6),
]


@pytest.mark.parametrize("m,p,q,L,N", CASES)
def test_cascade_equals_bruteforce_sum(m, p, q, L, N):
    rng = np.random.default_rng(100 * m + L + N)
    Abar, Bbar, C, D = _rand_system(rng, m, p, q, gamma=1.05)  # spectrum may pass 1
    u = rng.standard_normal((L, p))
    ref = _bruteforce_truncated(Abar, Bbar, C, D, u, N)
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(O.cascade(Abar, Bbar, C, D, u, N) - ref)) < 1e-12 * scale
    assert np.max(np.abs(O.truncated_sum(Abar, Bbar, C, D, u, N) - ref)) < 1e-12 * scale
    if (1 << (N + 1)) >= L:
        y, _ = O.recursion(Abar, Bbar, C, D, u)
        assert np.max(np.abs(y - ref)) < 1e-12 * scale


def test_stage_columns_on_impulse_m2_L8():
    # eqs. (3.2)-(3.4) by hand: with v^(0) = e_0 b (an impulse at l=0), after
    # stage n the column l is Abar^l b for l < 2^n and 0 beyond.
    Abar = np.array([[0.5, 0.25], [-0.125, 0.75]])
    b = np.array([[1.0], [2.0]])
    u = np.zeros((8, 1))
    u[0, 0] = 1.0
    _, st = O.cascade(Abar, b, np.eye(2), np.zeros((2, 1)), u, 2, return_stages=True)
    # explicit columns (exact binary fractions)
    A1 = Abar @ b            # [1.0, 1.375]
    A2 = Abar @ A1           # [0.84375, 0.90625]
    A3 = Abar @ A2
    assert np.allclose(A1[:, 0], [1.0, 1.375]) and np.allclose(A2[:, 0], [0.84375, 0.90625])
    exp = {1: [b, A1], 2: [b, A1, A2, A3]}
    for n, cols in exp.items():
        V = st[n]
        for l in range(8):
            want = cols[l][:, 0] if l < len(cols) else np.zeros(2)
            assert np.array_equal(V[:, l], want), (n, l)
    # stage 3 (shift 4) fills the remaining columns 4..7 with Abar^l b
    for l in range(8):
        assert np.allclose(st[3][:, l], (np.linalg.matrix_power(Abar, l) @ b)[:, 0], atol=1e-15)


def test_stage_columns_on_step_input():
    # constant input: after stage n, column l = sum_{j=0}^{min(l, 2^n-1)} Abar^j b
    rng = np.random.default_rng(7)
    Abar, b, _, _ = _rand_system(rng, 3, 1, 1, gamma=0.8)
    L = 20
    _, st = O.cascade(Abar, b, np.eye(3), np.zeros((3, 1)), np.ones((L, 1)), 4, return_stages=True)
    for n in range(6):
        for l in range(L):
            want = sum(np.linalg.matrix_power(Abar, j) @ b for j in range(min(l, 2 ** n - 1) + 1))
            assert np.allclose(st[n][:, l], want[:, 0], atol=1e-13)


# ------------------------------------------------------------ closed forms
def test_diagonal_geometric_closed_forms():
    lam = np.array([0.9, -0.7, 1.0, 0.999])
    b = np.array([1.0, 2.0, -1.0, 0.5])
    Abar = np.diag(lam)
    L, N = 50, 4  # T = 32 < L: truncation active
    T = 32
    eye = np.eye(4)
    Z = np.zeros((4, 1))
    # step response
    x = O.cascade(Abar, b[:, None], eye, Z, np.ones((L, 1)), N)
    for l in range(L):
        k = min(l, T - 1) + 1
        for i in range(4):
            want = b[i] * (k if lam[i] == 1.0 else (1 - lam[i] ** k) / (1 - lam[i]))
            assert abs(x[l, i] - want) < 1e-12 * max(1, abs(want))
    # geometric input mu^l, for l < T: b (mu^(l+1) - lam^(l+1)) / (mu - lam)
    mu = 0.95
    x = O.cascade(Abar, b[:, None], eye, Z, (mu ** np.arange(L))[:, None], N)
    for l in range(T):
        for i in range(4):
            want = b[i] * (mu ** (l + 1) - lam[i] ** (l + 1)) / (mu - lam[i])
            assert abs(x[l, i] - want) < 1e-12 * max(1, abs(want))


def test_scalar_case_matches_lfilter_and_convolve():
    lam, b, c, d = 0.97, 0.7, -1.3, 0.25
    rng = np.random.default_rng(11)
    L, N = 300, 6
    T = 1 << (N + 1)
    u = rng.standard_normal(L)
    y = O.cascade([[lam]], [[b]], [[c]], [[d]], u[:, None], N)[:, 0]
    # below T the cascade is the IIR filter y = c b /(1 - lam z^-1) + d
    iir = scipy.signal.lfilter([c * b], [1.0, -lam], u) + d * u
    assert np.max(np.abs(y[:T] - iir[:T])) < 1e-12
    assert np.max(np.abs(y[T:] - iir[T:])) > 1e-6  # truncation is visible afterwards
    # always the FIR with taps c lam^j b, j < T
    fir = np.convolve(u, c * b * lam ** np.arange(T))[:L] + d * u
    assert np.max(np.abs(y - fir)) < 1e-12


def test_markov_parameters():
    rng = np.random.default_rng(5)
    Abar, Bbar, C, D = _rand_system(rng, 4, 2, 3)
    L, N = 24, 3
    for col in range(2):
        u = np.zeros((L, 2))
        u[0, col] = 1.0
        y = O.cascade(Abar, Bbar, C, D, u, N)
        assert np.allclose(y[0], (D + C @ Bbar)[:, col], atol=1e-14)
        for j in range(1, L):
            want = (C @ np.linalg.matrix_power(Abar, j) @ Bbar)[:, col] if j < 16 else 0.0
            assert np.allclose(y[j], want, atol=1e-14)


# --------------------------------------------------- z-domain and the Lemma
def test_cascade_taps_are_the_coefficients_of_H_N():
    rng = np.random.default_rng(21)
    Abar, Bbar, C, D = _rand_system(rng, 3, 1, 2, gamma=0.95)
    N = 3
    T = 1 << (N + 1)
    u = np.zeros((T, 1))
    u[0, 0] = 1.0
    taps = O.cascade(Abar, Bbar, C, D, u, N)  # (T, q): D + h_0, h_1, ...
    for w in np.linspace(0.1, 3.0, 7):
        z = np.exp(1j * w)
        Hz = sum(taps[j][:, None] * z ** (-j) for j in range(T))
        assert np.allclose(Hz, O.transfer_truncated(Abar, Bbar, C, D, z, N), atol=1e-12)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_lemma_bound_on_unit_circle(N):
    rng = np.random.default_rng(40 + N)
    gamma = 0.9
    Abar, Bbar, C, D = _rand_system(rng, 5, 2, 2, gamma=gamma)
    bound = gamma ** (2 ** (N + 1)) / (1 - gamma) * np.linalg.norm(C, 2) * np.linalg.norm(Bbar, 2)
    worst = 0.0
    for w in np.linspace(0, 2 * np.pi, 97):
        z = np.exp(1j * w)
        diff = O.transfer(Abar, Bbar, C, D, z) - O.transfer_truncated(Abar, Bbar, C, D, z, N)
        worst = max(worst, np.linalg.norm(diff, 2))
    assert worst <= bound
    assert worst > 1e-14  # the truncation is visible at this N


# ------------------------------------------------------------- stability
def test_cascade_bounded_while_recursion_diverges():
    lam = np.array([0.5, 1.01])  # one eigenvalue past 1
    Abar = np.diag(lam)
    b = np.ones((2, 1))
    C = np.ones((1, 2))
    D = np.zeros((1, 1))
    N = 5
    T = 1 << (N + 1)
    rng = np.random.default_rng(0)
    L = 4000
    u = rng.uniform(-1, 1, (L, 1))
    fir_bound = sum(np.sum(np.abs(lam) ** j) for j in range(T)) * np.max(np.abs(u))
    y = O.cascade(Abar, b, C, D, u, N)
    assert np.max(np.abs(y)) <= fir_bound
    yr, _ = O.recursion(Abar, b, C, D, u)
    assert np.max(np.abs(yr)) > 1e6 * fir_bound


def test_stability_workload_spectrum():
    wl = W.stability(seed=0, batch=1, m=16, L=8, N=2)
    lam = np.sort(np.linalg.eigvals(wl.sets[0].A).real)
    assert np.allclose(lam, np.sort(wl.meta["eigenvalues"]), atol=1e-12)
    assert abs(lam.max() - (1 + 1e-5)) < 1e-12


# ------------------------------------------------------------- invariants
def test_linearity_causality_shift():
    rng = np.random.default_rng(9)
    Abar, Bbar, C, D = _rand_system(rng, 4, 2, 2)
    L, N = 40, 3
    u1, u2 = rng.standard_normal((L, 2)), rng.standard_normal((L, 2))
    f = lambda u: O.cascade(Abar, Bbar, C, D, u, N)
    assert np.allclose(f(2 * u1 - 3 * u2), 2 * f(u1) - 3 * f(u2), atol=1e-12)
    u3 = u1.copy()
    u3[25:] = rng.standard_normal((L - 25, 2))
    assert np.array_equal(f(u1)[:25], f(u3)[:25])
    s = 7
    us = np.zeros_like(u1)
    us[s:] = u1[: L - s]
    assert np.allclose(f(us)[s:], f(u1)[: L - s], atol=1e-12)


def test_effective_stages():
    assert O.effective_stages(5, 1) == 0
    assert O.effective_stages(5, 2) == 1
    assert O.effective_stages(5, 3) == 2
    assert O.effective_stages(11, 4096) == 12
    assert O.effective_stages(3, 4096) == 4


def test_fft_truncated_sum_matches_direct_sum():
    rng = np.random.default_rng(31)
    Abar, Bbar, C, D = _rand_system(rng, 4, 2, 3, gamma=1.02)
    u = rng.standard_normal((500, 2))
    for N in (2, 5, 9):
        a = O.truncated_sum(Abar, Bbar, C, D, u, N)
        b = O.truncated_sum_fft(Abar, Bbar, C, D, u, N)
        assert np.max(np.abs(a - b)) < 1e-10 * max(1.0, np.max(np.abs(a)))


def test_auto_stages_closed_forms_and_worked_example():
    # diagonal Abar: |Abar^(2^(n+1))|_F = sqrt(sum_i lam_i^(2^(n+2))) by hand
    lam = np.array([0.5, 0.25])
    A = np.diag(lam)
    # n = 0: 0.25^2 + ... ; the norms for n + 1 = 1..5 are
    # sqrt(0.5^(2^(k+1)) + 0.25^(2^(k+1))), k = n + 1
    norms = [np.sqrt(0.5 ** (2 ** (k + 1)) + 0.25 ** (2 ** (k + 1))) for k in range(1, 7)]
    for tol in (1e-2, 1e-6, 1e-12):
        want = next(n for n in range(6) if norms[n] <= tol)
        assert O.auto_stages(A, 1 << 20, tol) == want
    # the cap: the smallest N whose window 2^(N+1) covers L
    for L, cap in ((1, 0), (2, 0), (3, 1), (8, 2), (9, 3), (10, 3), (4096, 11), (4097, 12)):
        assert O.auto_stages(np.eye(2), L, 1e-300) == cap  # the identity never decays
    # §4 (m = 100, delta = 5e-4, 1-based HiPPO): |P_15|_F ~ 1.0e-9 and
    # |P_14|_F ~ 7.8e-3, so tolerances between give the paper's N = 14, and
    # 1e-14 needs one stage more (|P_16|_F ~ 5.9e-24)
    A4, b4 = W.hippo_legs(100)
    Ab, _ = O.trapezoid(A4, b4[:, None], 5e-4)
    assert O.auto_stages(Ab, 1 << 20, 1e-8) == 14
    assert O.auto_stages(Ab, 1 << 20, 1e-14) == 15
    assert O.auto_stages(Ab, (1 << 15) + 1, 1e-14) == 15  # at the cap
    assert O.auto_stages(Ab, 1 << 12, 1e-14) == 11        # the cap decides
