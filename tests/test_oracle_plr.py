"""Pins of the partitioned low-rank (PLR) oracle of §5 against what the paper
and linear algebra fix: the rank-1 off-diagonal blocks of the trapezoidal
HiPPO matrix (§5, eq. (4.2)), the rank growth of its powers bounded by the
product rule for off-diagonal blocks of lower-triangular matrices, exact
reconstruction at zero tolerance, planted ranks, the Eckart-Young optimality
of the truncation and its error bound, the block-by-block application against
the dense product, the flop count of a rank-1 form, and the cascade of §3 with
PLR powers against the dense cascade. Planted mistakes in copies of the
oracle's steps must each fail one of these pins.
"""

import numpy as np
import pytest

import oracle as O
from paper_2411_17729_amd import workloads as W


def _hippo_abar(m, delta):
    A, b = W.hippo_legs(m)
    Abar, _ = O.trapezoid(A, b, delta)
    return Abar


def _block(M, npad, d, g, side):
    s = npad >> d
    a = 2 * g * s
    Mp = np.zeros((npad, npad))
    Mp[: M.shape[0], : M.shape[0]] = M
    if side == 0:
        return Mp[a + s:a + 2 * s, a:a + s]
    return Mp[a:a + s, a + s:a + 2 * s]


@pytest.mark.parametrize("m", [64, 100, 256])
@pytest.mark.parametrize("delta", [1e-3, 1e-2, 1e-1])
def test_hippo_abar_offdiagonal_blocks_have_rank_one(m, delta):
    """§5: the matrix of eq. (4.2) has a PLR form with rank-1 off-diagonal
    blocks; it is lower triangular, so the upper blocks vanish. Blocks lying
    wholly in the zero padding have rank 0."""
    Abar = _hippo_abar(m, delta)
    T = O.plr_compress(Abar, 1e-12 * np.linalg.norm(Abar), leaf=16)
    for d, nodes in enumerate(O.plr_ranks(T), start=1):
        s = T["npad"] >> d
        for g, (r_low, r_up) in enumerate(nodes):
            rows0 = 2 * g * s + s  # first row of the lower block
            assert r_low == (1 if rows0 < m else 0), (d, g)
            assert r_up == 0, (d, g)


@pytest.mark.parametrize("m,delta", [(64, 1e-2), (256, 1e-3), (256, 1e-1), (128, 5e-3)])
def test_hippo_power_ranks_grow_at_most_by_the_product_rule(m, delta):
    """For lower-triangular F, G the lower block of F G over the split
    (I1, I2) is F21 G11 + F22 G21, so its rank is at most rank F21 + rank G21:
    the lower blocks of Abar^(2^k) have rank <= 2^k (and <= s). The bound is
    met at small k, so the truncation keeps every rank the powers really have."""
    P = O.powers(_hippo_abar(m, delta), 5)
    for k in range(6):
        T = O.plr_compress(P[k], 1e-11 * np.linalg.norm(P[k]), leaf=16)
        for d, nodes in enumerate(O.plr_ranks(T), start=1):
            s = T["npad"] >> d
            for r_low, r_up in nodes:
                assert r_up == 0
                assert r_low <= min(1 << k, s)
                if k <= 2:
                    assert r_low == min(1 << k, s)


@pytest.mark.parametrize("n,leaf", [(64, 16), (80, 16), (128, 8), (48, 16)])
def test_zero_tolerance_reconstructs_the_matrix(n, leaf):
    rng = np.random.default_rng(n + leaf)
    M = rng.standard_normal((n, n))
    T = O.plr_compress(M, 0.0, leaf=leaf)
    np.testing.assert_allclose(O.plr_dense(T), M, rtol=0, atol=1e-12)
    X = rng.standard_normal((n, 5))
    np.testing.assert_allclose(O.plr_apply(T, X), M @ X, rtol=0, atol=1e-11)


def _planted(npad, leaf, ranks, rng):
    M = np.zeros((npad, npad))
    for f in range(npad // leaf):
        M[f * leaf:(f + 1) * leaf, f * leaf:(f + 1) * leaf] = rng.standard_normal((leaf, leaf))
    D = len(ranks)
    for d in range(1, D + 1):
        s = npad >> d
        for g in range(1 << (d - 1)):
            a = 2 * g * s
            for side, r in enumerate(ranks[d - 1][g]):
                blk = rng.standard_normal((s, r)) @ rng.standard_normal((r, s))
                if side == 0:
                    M[a + s:a + 2 * s, a:a + s] = blk
                else:
                    M[a:a + s, a + s:a + 2 * s] = blk
    return M


def test_planted_ranks_are_found_block_by_block():
    rng = np.random.default_rng(7)
    npad, leaf = 128, 16
    ranks = [[(3, 0)], [(1, 4), (0, 2)], [(2, 2), (5, 1), (0, 0), (3, 6)]]
    M = _planted(npad, leaf, ranks, rng)
    T = O.plr_compress(M, 1e-9, leaf=leaf)
    assert [[tuple(x) for x in lv] for lv in O.plr_ranks(T)] == ranks
    np.testing.assert_allclose(O.plr_dense(T), M, rtol=0, atol=1e-9)


def test_truncation_is_minimal_and_within_the_bound():
    """Each block's Frobenius error is <= tol and one rank less would exceed
    it (Eckart-Young); the whole form is within 2 D tol in the 2-norm."""
    rng = np.random.default_rng(3)
    n = 128
    i = np.arange(n)
    M = np.exp(-np.abs(i[:, None] - i[None, :]) / 12.0) * (1 + 0.1 * rng.standard_normal((n, n)))
    tol = 1e-3 * np.linalg.norm(M)
    T = O.plr_compress(M, tol, leaf=16)
    for d, nodes in enumerate(T["levels"], start=1):
        for g, pair in enumerate(nodes):
            for side, (U, V) in enumerate(pair):
                B = _block(M, T["npad"], d, g, side)
                assert np.linalg.norm(B - U @ V.T) <= tol * (1 + 1e-12)
                r = U.shape[1]
                if r > 0:
                    sv = np.linalg.svd(B, compute_uv=False)
                    assert np.sqrt(np.sum(sv[r - 1:] ** 2)) > tol
    err = np.linalg.norm(M - O.plr_dense(T), 2)
    assert err <= O.plr_error_bound(T, tol)
    assert err > 0


def test_apply_matches_the_dense_form():
    rng = np.random.default_rng(11)
    A = _hippo_abar(100, 2e-2)
    P = O.powers(A, 6)
    for k in (0, 3, 6):
        T = O.plr_compress(P[k], 1e-6, leaf=16)
        X = rng.standard_normal((100, 9))
        np.testing.assert_allclose(O.plr_apply(T, X), O.plr_dense(T) @ X, rtol=0, atol=1e-12)
        x = X[:, 0]
        np.testing.assert_allclose(O.plr_apply(T, x), O.plr_dense(T) @ x, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m", [64, 256])
def test_rank_one_form_costs_m_log_m(m):
    """With rank-1 lower blocks and empty upper blocks one column costs
    2 (m leaf + m D) flops: m leaf for the diagonal leaves and, on each of the
    D levels, 2 s flops per node over m / (2 s) nodes."""
    T = O.plr_compress(_hippo_abar(m, 1e-2), 1e-12 * m, leaf=16)
    D = T["D"]
    assert O.plr_flops(T) == 2 * (m * 16 + m * D)


def test_cascade_with_exact_forms_equals_the_dense_cascade():
    rng = np.random.default_rng(5)
    m, p, q, L, N = 40, 2, 3, 300, 7
    A, _ = W.hippo_legs(m)
    Abar, Bbar = O.trapezoid(A, rng.standard_normal((m, p)), 0.03)
    C = rng.standard_normal((q, m))
    Dm = rng.standard_normal((q, p))
    u = rng.standard_normal((L, p))
    y = O.cascade(Abar, Bbar, C, Dm, u, N)
    y0 = O.cascade_plr(Abar, Bbar, C, Dm, u, N, 0.0, leaf=8)
    np.testing.assert_allclose(y0, y, rtol=0, atol=1e-11 * np.abs(y).max())
    # dense on some stages, PLR on the others: the same map
    y1 = O.cascade_plr(Abar, Bbar, C, Dm, u, N, 0.0, leaf=8, stages=[0, 2, 5])
    np.testing.assert_allclose(y1, y, rtol=0, atol=1e-11 * np.abs(y).max())


def _stage_error_bound(Abar, Bbar, C, u, N, eps):
    """Column-wise bound on |y_plr - y| from the stage recurrence
    e_k <= (1 + ||P_k||) e_{k-1} + eps_k max_l ||v_l^(k)||, times ||C||."""
    P = O.powers(Abar, N)
    _, st = O.cascade(Abar, Bbar, C, np.zeros((C.shape[0], u.shape[1])), u, N, return_stages=True)
    e = 0.0
    for k in range(N + 1):
        vmax = np.linalg.norm(st[k], axis=0).max()
        e = (1 + np.linalg.norm(P[k], 2)) * e + eps[k] * vmax
    return np.linalg.norm(C, 2) * e


def test_cascade_with_truncated_forms_stays_within_the_bound():
    rng = np.random.default_rng(9)
    m, p, q, L, N = 64, 2, 2, 400, 7
    A, _ = W.hippo_legs(m)
    Abar, Bbar = O.trapezoid(A, rng.standard_normal((m, p)), 0.05)
    C = rng.standard_normal((q, m))
    Dm = np.zeros((q, p))
    u = rng.standard_normal((L, p))
    tol = 1e-4
    y = O.cascade(Abar, Bbar, C, Dm, u, N)
    yp, forms = O.cascade_plr(Abar, Bbar, C, Dm, u, N, tol, leaf=16, return_stages=True)
    eps = [O.plr_error_bound(T, tol) for T in forms]
    col_err = np.linalg.norm(yp - y, axis=1).max()
    assert col_err <= _stage_error_bound(Abar, Bbar, C, u, N, eps)
    assert col_err > 1e-12  # the truncation is really in use


# ---- planted mistakes ----

def _apply_mutant(T, X, bug):
    npad, leaf, n = T["npad"], T["leaf"], T["n"]
    Xp = np.zeros((npad, X.shape[1]))
    Xp[:n] = X
    Y = np.zeros_like(Xp)
    for f, Lf in enumerate(T["leaves"]):
        Lm = Lf.T if bug == "leaf_transposed" else Lf
        Y[f * leaf:(f + 1) * leaf] += Lm @ Xp[f * leaf:(f + 1) * leaf]
    for d, nodes in enumerate(T["levels"], start=1):
        if bug == "drop_deepest_level" and d == T["D"]:
            continue
        s = npad >> d
        for g, ((Ul, Vl), (Uu, Vu)) in enumerate(nodes):
            a = 2 * g * s
            if bug == "sides_swapped":
                Y[a:a + s] += Ul @ (Vl.T @ Xp[a + s:a + 2 * s])
                Y[a + s:a + 2 * s] += Uu @ (Vu.T @ Xp[a:a + s])
            elif bug == "same_half":
                Y[a + s:a + 2 * s] += Ul @ (Vl.T @ Xp[a + s:a + 2 * s])
                Y[a:a + s] += Uu @ (Vu.T @ Xp[a:a + s])
            else:
                Y[a + s:a + 2 * s] += Ul @ (Vl.T @ Xp[a:a + s])
                Y[a:a + s] += Uu @ (Vu.T @ Xp[a + s:a + 2 * s])
    return Y[:n]


@pytest.mark.parametrize("bug", ["leaf_transposed", "drop_deepest_level", "sides_swapped", "same_half"])
def test_apply_mutants_fail_the_dense_pin(bug):
    rng = np.random.default_rng(2)
    M = rng.standard_normal((64, 64))
    T = O.plr_compress(M, 0.0, leaf=16)
    X = rng.standard_normal((64, 4))
    assert np.abs(_apply_mutant(T, X, "none") - M @ X).max() < 1e-11
    assert np.abs(_apply_mutant(T, X, bug) - M @ X).max() > 1e-3


def test_spectral_truncation_mutant_fails_the_frobenius_pin():
    """Keeping the singular values above tol (a 2-norm rule) instead of the
    Frobenius tail leaves blocks whose error exceeds tol."""
    rng = np.random.default_rng(4)
    s = 64
    B = rng.standard_normal((s, s)) @ np.diag(0.8 ** np.arange(s)) @ rng.standard_normal((s, s)) / s
    tol = 1e-3 * np.linalg.norm(B)
    U, sv, Vt = np.linalg.svd(B)
    r_bad = int(np.sum(sv > tol))
    err_bad = np.linalg.norm(B - (U[:, :r_bad] * sv[:r_bad]) @ Vt[:r_bad])
    assert err_bad > tol
    T = O.plr_compress(np.block([[np.zeros((s, s)), np.zeros((s, s))], [B, np.zeros((s, s))]]), tol, leaf=s)
    (Ul, Vl), _ = T["levels"][0][0]
    assert np.linalg.norm(B - Ul @ Vl.T) <= tol
    assert Ul.shape[1] > r_bad
