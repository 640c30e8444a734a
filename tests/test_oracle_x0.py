"""Pins for the oracle's initial state x_{-1} (eq. (1.2) with a nonzero
initial condition): chunking identities of the recursion, the closed form for a
diagonal Abar, the truncation at T = 2^(N+1) lags, and planted mistakes that
these pins catch."""

import numpy as np

from oracle import ssm_oracle as O


def _system(rng, m=5, p=2, q=3):
    A = rng.standard_normal((m, m)) / np.sqrt(m) * 0.9
    return A, rng.standard_normal((m, p)), rng.standard_normal((q, m)), rng.standard_normal((q, p))


def test_recursion_chunks_carry_the_state():
    # running u in two pieces, the second from the first's last state, is the
    # same as one run: x0 enters as the state before the first step
    rng = np.random.default_rng(1)
    A, B, C, D = _system(rng)
    u = rng.standard_normal((40, 2))
    x0 = rng.standard_normal(5)
    y, x = O.recursion(A, B, C, D, u, x0=x0)
    y1, x1 = O.recursion(A, B, C, D, u[:17], x0=x0)
    y2, x2 = O.recursion(A, B, C, D, u[17:], x0=x1[-1])
    np.testing.assert_allclose(np.vstack([y1, y2]), y, rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.vstack([x1, x2]), x, rtol=0, atol=1e-13)
    # and from zero, the first piece is the plain recursion
    y0, _ = O.recursion(A, B, C, D, u)
    yz, _ = O.recursion(A, B, C, D, u, x0=np.zeros(5))
    np.testing.assert_array_equal(y0, yz)


def test_diagonal_closed_form():
    # Abar = diag(lam), u = 0, C = I, D = 0: y_l = lam^(l+1) x0, for the
    # recursion and for the truncated sum while l < T
    lam = np.array([0.9, -0.5, 0.99, 0.3])
    x0 = np.array([1.0, 2.0, -1.0, 0.5])
    L = 12
    u = np.zeros((L, 1))
    Bz, Dz = np.zeros((4, 1)), np.zeros((4, 1))
    want = lam[None, :] ** (np.arange(L)[:, None] + 1) * x0[None, :]
    y, x = O.recursion(np.diag(lam), Bz, np.eye(4), Dz, u, x0=x0)
    np.testing.assert_allclose(y, want, rtol=1e-14, atol=0)
    np.testing.assert_allclose(x, want, rtol=1e-14, atol=0)
    yt = O.truncated_sum(np.diag(lam), Bz, np.eye(4), Dz, u, N=3, x0=x0)  # T = 16 > L
    np.testing.assert_allclose(yt, want, rtol=1e-14, atol=0)
    # planted mistake: x0 taken as x_0 (one power short) misses the closed form
    wrong = lam[None, :] ** np.arange(L)[:, None] * x0[None, :]
    assert np.abs(wrong - want).max() > 0.1


def test_truncation_of_the_free_response():
    # with L > T the polynomial keeps the lags l < T only: lam^(l+1) x0, then 0
    lam = np.array([0.8, -0.6])
    x0 = np.array([1.5, -2.0])
    N, L = 2, 13  # T = 8
    z = O.free_response(np.diag(lam), np.eye(2), x0, L, N)
    l = np.arange(L)[:, None]
    want = np.where(l < 8, lam[None, :] ** (l + 1) * x0[None, :], 0.0)
    np.testing.assert_allclose(z, want, rtol=1e-14, atol=0)


def test_truncated_sum_with_state_is_the_cascade_window():
    # T >= L: the truncated sum from x0 equals the recursion from x0; and the
    # same holds for any split of the window, the state carried (brute force)
    rng = np.random.default_rng(2)
    A, B, C, D = _system(rng, m=6, p=3, q=2)
    u = rng.standard_normal((30, 3))
    x0 = rng.standard_normal(6)
    y, _ = O.recursion(A, B, C, D, u, x0=x0)
    yt = O.truncated_sum(A, B, C, D, u, N=4, x0=x0)  # T = 32 >= 30
    np.testing.assert_allclose(yt, y, rtol=0, atol=1e-12)
    # brute force of x_l = A^(l+1) x0 + sum_j A^j B u_{l-j}
    for l in (0, 1, 7, 29):
        xl = np.linalg.matrix_power(A, l + 1) @ x0 + sum(np.linalg.matrix_power(A, j) @ B @ u[l - j]
                                                        for j in range(l + 1))
        np.testing.assert_allclose(C @ xl + D @ u[l], y[l], rtol=0, atol=1e-12)
    # planted mistake: the free response added with Bbar in front of x0
    # (x0 treated as an input) fails the brute force
    zb = O.free_response(A, C, B @ np.ones(3), 30, 4)
    assert np.abs(zb[0] - C @ A @ x0).max() > 1e-3


def _loss(A, B, C, D, u, dy, N, x0, truncated):
    if truncated:
        y = O.truncated_sum(A, B, C, D, u, N, x0=x0)
    else:
        y, _ = O.recursion(A, B, C, D, u, x0=x0)
    return float(np.sum(dy * y))


def _fd(f, X, h=1e-6):
    g = np.zeros_like(X)
    for idx in np.ndindex(X.shape):
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += h
        Xm[idx] -= h
        g[idx] = (f(Xp) - f(Xm)) / (2 * h)
    return g


def test_initial_state_gradients_by_finite_differences():
    # d sum(dy * y) / d(x0, Abar, C) with a nonzero initial state, for the
    # recursion (BPTT) and for the truncated sum with T < L (brute force):
    # central differences (h = 1e-6, FP64) of the forward oracles
    rng = np.random.default_rng(7)
    A, B, C, D = _system(rng, m=4, p=2, q=3)
    u = rng.standard_normal((11, 2))
    dy = rng.standard_normal((11, 3))
    x0 = rng.standard_normal(4)
    for N, truncated in ((None, False), (1, True)):  # T = 4 < L = 11
        g = O.grads_recursion(A, B, C, D, u, dy, x0) if not truncated else \
            O.grads_truncated_bruteforce(A, B, C, D, u, dy, N, x0)
        fx = _fd(lambda X: _loss(A, B, C, D, u, dy, N, X, truncated), x0)
        fa = _fd(lambda X: _loss(X, B, C, D, u, dy, N, x0, truncated), A)
        fc = _fd(lambda X: _loss(A, B, X, D, u, dy, N, x0, truncated), C)
        fb = _fd(lambda X: _loss(A, X, C, D, u, dy, N, x0, truncated), B)
        np.testing.assert_allclose(g["x0"], fx, rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(g["Abar"], fa, rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(g["C"], fc, rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(g["Bbar"], fb, rtol=1e-6, atol=1e-8)
        # planted mistakes: x0's gradient without the leading Abar^T, and
        # gAbar without the x0 term, both miss the differences
        lam0 = np.linalg.solve(A.T, g["x0"])
        assert np.abs(lam0 - fx).max() > 1e-3
        if not truncated:
            assert np.abs((g["Abar"] - np.outer(lam0, x0)) - fa).max() > 1e-3
    # with x0 = None the x0 entry is absent and the rest is unchanged
    g0 = O.grads_recursion(A, B, C, D, u, dy)
    gz = O.grads_recursion(A, B, C, D, u, dy, np.zeros(4))
    assert g0["x0"] is None
    np.testing.assert_allclose(g0["Abar"], gz["Abar"], rtol=0, atol=1e-14)


def test_initial_state_gradient_diagonal_closed_form():
    # Abar = diag(lam), C = I, D = 0: y_l = lam^(l+1) x0 + ..., so
    # d sum(dy * y) / dx0 = sum_{l < min(L, T)} lam^(l+1) dy_l
    lam = np.array([0.9, -0.5, 0.7])
    L, N = 9, 2  # T = 8 < L: the last row's free response is cut
    dy = np.random.default_rng(8).standard_normal((L, 3))
    u = np.zeros((L, 1))
    g = O.grads_truncated_bruteforce(np.diag(lam), np.zeros((3, 1)), np.eye(3), np.zeros((3, 1)), u, dy, N,
                                     x0=np.ones(3))
    l = np.arange(8)[:, None]
    want = np.sum(lam[None, :] ** (l + 1) * dy[:8], axis=0)
    np.testing.assert_allclose(g["x0"], want, rtol=1e-14, atol=1e-15)
