"""Plain, slow, obviously-correct FP64 reference for the fast cascade.

TEST INFRASTRUCTURE ONLY (see the package docstring): the HIP library never
calls into this file, and this file never imports the HIP library.

Everything here is numpy float64 on the CPU, one sequence at a time, written
for a reader holding the paper (Beylkin, arXiv 2411.17729) next to it:

* ``trapezoid``        -- the trapezoidal discretization of §1 (after eq. (1.2)).
* ``zoh``              -- the exponential discretization named in §5:
  Abar = exp(delta A) and the matching Bbar (reading below).
* ``recursion``        -- the discrete LTI recursion, eq. (1.2), from x_{-1} = 0 or a
  given initial state.
* ``powers``           -- Abar, Abar^2, Abar^4, ... by repeated squaring (end of §2).
* ``impulse_response`` / ``truncated_sum`` -- the convolution sum eq. (3.1)
  restricted to the lags that the degree-(2^{N+1}-1) polynomial H_N of
  eq. (2.2)/(2.3) keeps.
* ``cascade``          -- the stage-by-stage algorithm of §3, eqs. (3.2)-(3.4)
  and the general step, followed by the output y = C v + D u.
* ``transfer`` / ``transfer_truncated`` -- H(z) of eq. (1.3) and H_N(z) of
  eq. (2.2) evaluated at a point z of the unit circle.
* ``grads_*`` / ``trapezoid_adjoint`` / ``zoh_adjoint`` -- reverse-mode
  derivatives of the maps above (not in the paper; derived by the chain rule,
  pinned by finite differences in the tests).

Readings of points where the paper is loose (each also listed in the design
notes of the repository):

* Stage count. H_N has N+1 factors, so the cascade runs N+1 stages with shifts
  1, 2, ..., 2^N, and the output is taken after the last one (§2, eq. (2.2);
  §3 "N+1 matrix-vector multiplications"), even though the text of §3 writes
  the final output with V^(N).
* Output term. eq. (3.1) prints D u_k inside the sum; the output equation of
  eq. (1.2) and the final step of §3 both add D u_l once, which is used here.
* Boundary. Columns l < 2^n are copied unchanged at stage n (x_{-1} = 0,
  §3); a stage whose shift reaches past the sequence changes nothing.
* Exponential discretization. §5 prints Bbar = (delta A)^{-1} [exp(delta A) - I]
  delta A, which is m x m and cannot multiply u; the factor on the right is
  read as delta B, the zero-order hold: Bbar = int_0^delta exp(s A) ds B,
  which equals (delta A)^{-1} [exp(delta A) - I] delta B when A is invertible
  and stays defined when it is not.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "trapezoid",
    "trapezoid_adjoint",
    "zoh",
    "zoh_adjoint",
    "recursion",
    "powers",
    "impulse_response",
    "truncated_sum",
    "truncated_sum_fft",
    "cascade",
    "transfer",
    "transfer_truncated",
    "grads_recursion",
    "grads_truncated_bruteforce",
    "grads_full",
    "effective_stages",
]


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def _as_matrix_u(u):
    u = _f64(u)
    if u.ndim == 1:
        u = u[:, None]
    return u


# --------------------------------------------------------------------------
# Discretization (§1, the trapezoidal rule stated after eq. (1.2); also
# eq. (4.2) for the HiPPO example of §4)
# --------------------------------------------------------------------------
def trapezoid(A, B, delta):
    """Abar = (I - delta/2 A)^{-1} (I + delta/2 A),  Bbar = delta (I - delta/2 A)^{-1} B.

    Both are obtained from one linear solve with the matrix I - delta/2 A, as
    the formulas state (no explicit inverse).
    """
    A = _f64(A)
    B = _f64(B)
    if B.ndim == 1:
        B = B[:, None]
    m = A.shape[0]
    eye = np.eye(m)
    lhs = eye - 0.5 * delta * A
    rhs = np.concatenate([eye + 0.5 * delta * A, delta * B], axis=1)
    sol = np.linalg.solve(lhs, rhs)
    return sol[:, :m], sol[:, m:]


def trapezoid_adjoint(A, B, delta, gAbar, gBbar):
    """Gradients of a scalar loss w.r.t. A and B given its gradients w.r.t. Abar, Bbar.

    Derived by the chain rule from the two formulas of ``trapezoid``. With
    M = I - delta/2 A:
        dAbar = delta/2 M^{-1} dA (I + Abar)
        dBbar = delta/2 M^{-1} dA Bbar + delta M^{-1} dB
    hence
        gA = delta/2 M^{-T} gAbar (I + Abar)^T + delta/2 M^{-T} gBbar Bbar^T
        gB = delta M^{-T} gBbar.
    """
    A = _f64(A)
    B = _f64(B)
    if B.ndim == 1:
        B = B[:, None]
    m = A.shape[0]
    eye = np.eye(m)
    M = eye - 0.5 * delta * A
    Abar, Bbar = trapezoid(A, B, delta)
    # M^{-T} X is the solution of M^T Z = X.
    gA = 0.5 * delta * np.linalg.solve(M.T, gAbar @ (eye + Abar).T)
    gA += 0.5 * delta * np.linalg.solve(M.T, gBbar @ Bbar.T)
    gB = delta * np.linalg.solve(M.T, gBbar)
    return gA, gB


# --------------------------------------------------------------------------
# Exponential discretization (§5, the choice Abar = exp(delta A) discussed
# for structured representations of the HiPPO matrix)
# --------------------------------------------------------------------------
def _zoh_augmented(A, B, delta):
    A = _f64(A)
    B = _f64(B)
    if B.ndim == 1:
        B = B[:, None]
    m, p = A.shape[0], B.shape[1]
    E = np.zeros((m + p, m + p))
    E[:m, :m] = delta * A
    E[:m, m:] = delta * B
    return E, m


def zoh(A, B, delta):
    """Abar = exp(delta A),  Bbar = int_0^delta exp(s A) ds B.

    Both are blocks of one matrix exponential: for E = [[delta A, delta B],
    [0, 0]], exp(E) = [[exp(delta A), Bbar], [0, I]] (the series of exp(E)
    has upper-right block sum_k (delta A)^k delta B / (k+1)!, the series of
    the integral). The exponential is the library step (scipy.linalg.expm).
    """
    from scipy.linalg import expm

    E, m = _zoh_augmented(A, B, delta)
    F = expm(E)
    return F[:m, :m], F[:m, m:]


def zoh_adjoint(A, B, delta, gAbar, gBbar):
    """Gradients of a scalar loss w.r.t. A and B given its gradients w.r.t. Abar, Bbar.

    With F = exp(E) and E the augmented matrix of ``zoh``, dF = L(E, dE), the
    Frechet derivative of the exponential, L(E, X) = int_0^1 exp(sE) X
    exp((1-s)E) ds. Its adjoint under the trace inner product is L(E^T, .),
    so gE = L(E^T, G) with G = [[gAbar, gBbar], [0, 0]]; E holds delta A and
    delta B, hence gA = delta gE[:m, :m] and gB = delta gE[:m, m:]. L is the
    library step (scipy.linalg.expm_frechet).
    """
    from scipy.linalg import expm_frechet

    E, m = _zoh_augmented(A, B, delta)
    G = np.zeros_like(E)
    G[:m, :m] = _f64(gAbar)
    G[:m, m:] = _f64(gBbar).reshape(m, -1)
    _, gE = expm_frechet(E.T, G)
    return delta * gE[:m, :m], delta * gE[:m, m:]


# --------------------------------------------------------------------------
# The recursion, eq. (1.2)
# --------------------------------------------------------------------------
def recursion(Abar, Bbar, C, D, u, x0=None):
    """x_n = Abar x_{n-1} + Bbar u_n, y_n = C x_n + D u_n, eq. (1.2).

    The state before the first step is x_{-1} = x0 (zero when x0 is None), the
    initial condition that the problem statement of §1 sets to zero.
    Returns (y, x) with y of shape (L, q) and x of shape (L, m).
    """
    Abar, Bbar, C, D = _f64(Abar), _f64(Bbar), _f64(C), _f64(D)
    u = _as_matrix_u(u)
    L = u.shape[0]
    m = Abar.shape[0]
    x = np.zeros(m) if x0 is None else _f64(x0).reshape(m).copy()
    xs = np.empty((L, m))
    for n in range(L):
        x = Abar @ x + Bbar @ u[n]
        xs[n] = x
    y = xs @ C.T + u @ D.T
    return y, xs


# --------------------------------------------------------------------------
# Powers by repeated squaring (end of §2; §3 "compute the powers")
# --------------------------------------------------------------------------
def powers(Abar, N):
    """[Abar^(2^0), Abar^(2^1), ..., Abar^(2^N)], each the square of the previous."""
    P = [_f64(Abar).copy()]
    for _ in range(N):
        P.append(P[-1] @ P[-1])
    return P


def auto_stages(Abar, L, tol):
    """N chosen for a sequence of length L at tolerance tol: the smallest N
    whose first left-out power, Abar^(2^(N+1)) (the polynomial of eq. (2.2)
    keeps Abar^j for j < 2^(N+1)), has Frobenius norm at most tol, the way §4
    picks N from the size of that power; at most the smallest N whose window
    2^(N+1) covers L (there the cascade is the recursion itself).
    """
    cap = 0
    while (1 << (cap + 1)) < L:
        cap += 1
    P = powers(Abar, cap)
    for n in range(cap):
        if np.linalg.norm(P[n + 1], "fro") <= tol:
            return n
    return cap


def effective_stages(N, L):
    """Number of cascade stages that change anything for a length-L sequence.

    Stage n (shift 2^n) updates the columns 2^n <= l <= L-1 (§3); once
    2^n >= L it updates nothing, so at most floor(log2(L-1)) + 1 stages act.
    """
    if L <= 1:
        return 0
    act = 0
    while act <= N and (1 << act) <= L - 1:
        act += 1
    return act


# --------------------------------------------------------------------------
# The convolution sum, eq. (3.1), restricted to the lags of H_N (eq. (2.3))
# --------------------------------------------------------------------------
def impulse_response(Abar, Bbar, C, T):
    """h_j = C Abar^j Bbar for j = 0..T-1, via w_{j+1} = Abar w_j, w_0 = Bbar.

    Returns an array of shape (T, q, p).
    """
    Abar, Bbar, C = _f64(Abar), _f64(Bbar), _f64(C)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    h = np.empty((T, C.shape[0], Bbar.shape[1]))
    w = Bbar.copy()
    for j in range(T):
        h[j] = C @ w
        w = Abar @ w
    return h


def free_response(Abar, C, x0, L, N):
    """z_l = C Abar^(l+1) x0 for l < min(L, T), zero from T on, T = 2^(N+1).

    The part of the output that an initial state x_{-1} = x0 contributes. Unrolling
    eq. (1.2) gives x_l = Abar^(l+1) x_{-1} + sum_{j<=l} Abar^j Bbar u_{l-j}, i.e.
    x_{-1} acts as one more input Abar x_{-1} at l = 0, and the degree-(T-1)
    polynomial H_N of eq. (2.2) keeps its lags l < T. Computed by
    w_0 = Abar x0, w_{l+1} = Abar w_l.
    """
    Abar, C = _f64(Abar), _f64(C)
    m = Abar.shape[0]
    z = np.zeros((L, C.shape[0]))
    w = Abar @ _f64(x0).reshape(m)
    for l in range(min(L, 1 << (N + 1))):
        z[l] = C @ w
        w = Abar @ w
    return z


def truncated_sum(Abar, Bbar, C, D, u, N, x0=None):
    """y_l = sum_{j=0}^{min(l, T-1)} C Abar^j Bbar u_{l-j} + D u_l with T = 2^(N+1).

    This is eq. (3.1) with the lags cut where the polynomial H_N of
    eq. (2.2)/(2.3) stops (degree T-1). When T >= L nothing is cut and this
    equals ``recursion``. With an initial state x0, ``free_response`` is added
    (then with T >= L this equals ``recursion`` from x_{-1} = x0).
    """
    u = _as_matrix_u(u)
    L = u.shape[0]
    T = 1 << (N + 1)
    Tu = min(T, L)
    h = impulse_response(Abar, Bbar, C, Tu)
    y = u @ _f64(D).T
    for j in range(Tu):
        y[j:] += u[: L - j] @ h[j].T
    if x0 is not None:
        y += free_response(Abar, C, x0, L, N)
    return y


def truncated_sum_fft(Abar, Bbar, C, D, u, N):
    """The same sum as ``truncated_sum``, each (output, input) channel pair a
    causal convolution of u with the taps h_j = C Abar^j Bbar (j < T),
    evaluated with an FFT (scipy.signal.fftconvolve) for long sequences."""
    from scipy.signal import fftconvolve

    u = _as_matrix_u(u)
    L = u.shape[0]
    T = 1 << (N + 1)
    h = impulse_response(Abar, Bbar, C, min(T, L))
    y = u @ _f64(D).T
    for qi in range(h.shape[1]):
        for pi in range(h.shape[2]):
            y[:, qi] += fftconvolve(u[:, pi], h[:, qi, pi])[:L]
    return y


# --------------------------------------------------------------------------
# The cascade of §3, stage by stage
# --------------------------------------------------------------------------
def cascade(Abar, Bbar, C, D, u, N, return_stages=False):
    """Apply H_N of eq. (2.3) in the time domain by the cascade of §3.

    V^(0) has columns v_l = Bbar u_l (an m x L matrix). Stage n = 1..N+1 uses
    the power Abar^(2^(n-1)) and the shift 2^(n-1):
        v_l^(n) = Abar^(2^(n-1)) v_{l-2^(n-1)}^(n-1) + v_l^(n-1)   for 2^(n-1) <= l <= L-1,
        v_l^(n) = v_l^(n-1)                                         otherwise
    (eqs. (3.2)-(3.4) and the general step). Output y_l = C v_l^(N+1) + D u_l.

    Returns y of shape (L, q); with ``return_stages`` also the list
    [V^(0), ..., V^(N+1)], each of shape (m, L).
    """
    Abar, Bbar, C, D = _f64(Abar), _f64(Bbar), _f64(C), _f64(D)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    u = _as_matrix_u(u)
    L = u.shape[0]
    P = powers(Abar, N)
    V = Bbar @ u.T  # m x L, column l is v_l^(0)
    stages = [V.copy()]
    for n in range(1, N + 2):
        shift = 1 << (n - 1)
        Vn = V.copy()
        if shift <= L - 1:
            Vn[:, shift:] = P[n - 1] @ V[:, : L - shift] + V[:, shift:]
        V = Vn
        stages.append(V.copy())
    y = (C @ V).T + u @ D.T
    if return_stages:
        return y, stages
    return y


# --------------------------------------------------------------------------
# Transfer functions, eq. (1.3) and eq. (2.2)
# --------------------------------------------------------------------------
def transfer(Abar, Bbar, C, D, z):
    """H(z) = C (I - z^{-1} Abar)^{-1} Bbar + D (eq. (1.3))."""
    Abar = _f64(Abar)
    m = Abar.shape[0]
    Bbar = _f64(Bbar)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    X = np.linalg.solve(np.eye(m) - Abar / z, Bbar.astype(complex))
    return _f64(C) @ X + _f64(D)


def transfer_truncated(Abar, Bbar, C, D, z, N):
    """H_N(z) = C prod_{n=0}^{N} [I + (z^{-1} Abar)^(2^n)] Bbar + D (eq. (2.2)).

    The factors commute, so the order of the product is immaterial; they are
    multiplied in increasing n.
    """
    Abar = _f64(Abar)
    m = Abar.shape[0]
    Bbar = _f64(Bbar)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    Z = Abar.astype(complex) / z
    prod = np.eye(m, dtype=complex)
    Zp = Z.copy()
    for _ in range(N + 1):
        prod = prod @ (np.eye(m) + Zp)
        Zp = Zp @ Zp
    return _f64(C) @ prod @ Bbar + _f64(D)


# --------------------------------------------------------------------------
# Reverse-mode derivatives (not in the paper)
# --------------------------------------------------------------------------
def grads_recursion(Abar, Bbar, C, D, u, dy, x0=None):
    """Gradients of sum(dy * y) for y = recursion(..., x0), by backpropagation in time.

    lambda_l = C^T dy_l + Abar^T lambda_{l+1}  (lambda_L = 0),
    gAbar = sum_{l>=0} lambda_l x_{l-1}^T (x_{-1} = x0),  gBbar = sum_l lambda_l u_l^T,
    gC = sum_l dy_l x_l^T,  gD = sum_l dy_l u_l^T,  gu_l = Bbar^T lambda_l + D^T dy_l,
    gx0 = Abar^T lambda_0 (the initial state enters only through x_0 = Abar x0 + ...).

    When 2^(N+1) >= L the cascade output equals the recursion output, so these
    are also the cascade's gradients.
    Returns dict(u, Abar, Bbar, C, D, x0); x0 is None when x0 is None.
    """
    Abar, Bbar, C, D = _f64(Abar), _f64(Bbar), _f64(C), _f64(D)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    u = _as_matrix_u(u)
    dy = _as_matrix_u(dy)
    L = u.shape[0]
    m = Abar.shape[0]
    _, xs = recursion(Abar, Bbar, C, D, u, x0)
    lam = np.zeros(m)
    gA = np.zeros((m, m))
    gB = np.zeros_like(Bbar)
    gu = np.empty_like(u)
    for n in range(L - 1, -1, -1):
        lam = C.T @ dy[n] + Abar.T @ lam
        if n >= 1:
            gA += np.outer(lam, xs[n - 1])
        elif x0 is not None:
            gA += np.outer(lam, _f64(x0).reshape(m))
        gB += np.outer(lam, u[n])
        gu[n] = Bbar.T @ lam + D.T @ dy[n]
    gC = dy.T @ xs
    gD = dy.T @ u
    gx0 = Abar.T @ lam if x0 is not None else None
    return {"u": gu, "Abar": gA, "Bbar": gB, "C": gC, "D": gD, "x0": gx0}


def grads_truncated_bruteforce(Abar, Bbar, C, D, u, dy, N, x0=None):
    """Gradients of sum(dy * y) for y = truncated_sum(..., N, x0), by brute force.

    With T = 2^(N+1) and x_l = sum_{j<=min(l,T-1)} Abar^j Bbar u_{l-j}:
    d(Abar^j) = sum_{a+b=j-1} Abar^a dAbar Abar^b, so
        gAbar = sum_l sum_{1<=j<=min(l,T-1)} sum_{a+b=j-1} (Abar^T)^a g_l (Abar^b Bbar u_{l-j})^T
    with g_l = C^T dy_l. An initial state adds Abar^(l+1) x0 to x_l for l < T
    (``free_response``): gx0 = sum_{l<T} (Abar^(l+1))^T g_l and
    gAbar += sum_{l<T} sum_{a+b=l} (Abar^T)^a g_l (Abar^b x0)^T.
    Cost O(L T^2 m^3): tiny inputs only.
    """
    Abar, Bbar, C, D = _f64(Abar), _f64(Bbar), _f64(C), _f64(D)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    u = _as_matrix_u(u)
    dy = _as_matrix_u(dy)
    L = u.shape[0]
    m = Abar.shape[0]
    T = 1 << (N + 1)
    pw = [np.eye(m)]
    for _ in range(max(T, 2)):
        pw.append(pw[-1] @ Abar)
    g = dy @ C  # row l is (C^T dy_l)^T
    gA = np.zeros((m, m))
    gB = np.zeros_like(Bbar)
    gu = np.zeros_like(u)
    xs = np.zeros((L, m))
    for l in range(L):
        for j in range(min(l, T - 1) + 1):
            xs[l] += pw[j] @ Bbar @ u[l - j]
            # gradient w.r.t. u_{l-j} and Bbar through the term Abar^j Bbar u_{l-j}
            lamj = pw[j].T @ g[l]
            gu[l - j] += Bbar.T @ lamj
            gB += np.outer(lamj, u[l - j])
            for a in range(j):
                b = j - 1 - a
                gA += np.outer(pw[a].T @ g[l], pw[b] @ Bbar @ u[l - j])
    gx0 = None
    if x0 is not None:
        x0 = _f64(x0).reshape(m)
        gx0 = np.zeros(m)
        for l in range(min(L, T)):
            xs[l] += pw[l + 1] @ x0
            gx0 += pw[l + 1].T @ g[l]
            for a in range(l + 1):
                gA += np.outer(pw[a].T @ g[l], pw[l - a] @ x0)
    gu += dy @ D
    gC = dy.T @ xs
    gD = dy.T @ u
    return {"u": gu, "Abar": gA, "Bbar": gB, "C": gC, "D": gD, "x0": gx0}


def grads_full(A, B, C, D, delta, u, dy, N=None, disc="trapezoid", x0=None):
    """Gradients of sum(dy * y) w.r.t. (u, A, B, C, D, and x0 when given)
    through the trapezoidal (disc = "trapezoid") or exponential ("zoh")
    discretization. Uses BPTT when N is None or 2^(N+1) >= L, else brute force.
    """
    Abar, Bbar = (trapezoid if disc == "trapezoid" else zoh)(A, B, delta)
    u = _as_matrix_u(u)
    L = u.shape[0]
    if N is None or (1 << (N + 1)) >= L:
        g = grads_recursion(Abar, Bbar, C, D, u, dy, x0)
    else:
        g = grads_truncated_bruteforce(Abar, Bbar, C, D, u, dy, N, x0)
    gA, gB = (trapezoid_adjoint if disc == "trapezoid" else zoh_adjoint)(A, B, delta, g["Abar"], g["Bbar"])
    return {"u": g["u"], "A": gA, "B": gB, "C": g["C"], "D": g["D"],
            "Abar": g["Abar"], "Bbar": g["Bbar"], "x0": g["x0"]}
