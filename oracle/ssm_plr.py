"""Partitioned low-rank (PLR) powers for the cascade: plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring): the HIP library never
calls into this file, and this file never imports the HIP library.

§5 of the paper observes that the trapezoidal HiPPO matrix, eq. (4.2), has a
partitioned low-rank representation whose off-diagonal blocks have rank 1, so
that it and its powers can be applied in O(m log m) instead of O(m^2). The
paper gives no ranks, tolerances or construction for the powers; the readings
taken here (also listed in the design notes of the repository):

* Partition. The dyadic one: the matrix (zero-padded to n = leaf 2^D) is split
  into 2 x 2 blocks, the two off-diagonal blocks are stored in low-rank form
  and the two diagonal blocks are split again, down to dense diagonal leaves of
  size ``leaf``. Level d = 1..D holds 2^(d-1) nodes of block size s = n / 2^d;
  node g covers rows and columns [2 g s, 2 g s + 2 s), its lower block is rows
  [2 g s + s, 2 g s + 2 s) x columns [2 g s, 2 g s + s) and its upper block is
  the transposed position.
* Rank. An off-diagonal block B is kept as U V^T with the smallest r whose
  truncated SVD leaves a Frobenius error ||B - U V^T||_F <= tol (Eckart-Young:
  sqrt(sum of the squared discarded singular values)); U = U_r diag(sigma_r),
  V = V_r. ``tol`` is absolute.
* Error. The lower blocks of one level occupy disjoint rows and disjoint
  columns, so together their errors have spectral norm <= tol; the same holds
  for the upper blocks, hence ||M - PLR(M)||_2 <= 2 D tol.

Functions:

* ``plr_compress`` -- the PLR form of a square matrix at a tolerance.
* ``plr_dense``    -- the matrix that a PLR form represents.
* ``plr_apply``    -- the PLR form applied to columns, block by block (leaf
  products, then V^T x and U (V^T x) for every off-diagonal block).
* ``plr_ranks`` / ``plr_flops`` -- ranks per level, node and side; flops per
  applied column.
* ``cascade_plr``  -- the cascade of §3 with each P_k = Abar^(2^k) replaced by
  its PLR form (on every stage, or on the stages named).
"""

from __future__ import annotations

import numpy as np

from .ssm_oracle import powers

__all__ = [
    "plr_compress",
    "plr_dense",
    "plr_apply",
    "plr_ranks",
    "plr_flops",
    "plr_error_bound",
    "cascade_plr",
]


def _levels(n, leaf):
    """Padded size leaf 2^D >= n and the level count D."""
    D = 0
    while (leaf << D) < n:
        D += 1
    return leaf << D, D


def _truncate(B, tol):
    """Smallest-rank factors U V^T of B with ||B - U V^T||_F <= tol (truncated SVD)."""
    U, sv, Vt = np.linalg.svd(B)
    # tail[r] = Frobenius error when the first r singular values are kept
    tail = np.sqrt(np.concatenate([np.cumsum((sv * sv)[::-1])[::-1], [0.0]]))
    r = int(np.argmax(tail <= tol))
    return U[:, :r] * sv[:r], Vt[:r].T.copy()


def plr_compress(M, tol, leaf=16):
    """PLR form of the square matrix M at absolute tolerance ``tol`` (§5).

    Returns a dict with ``n`` (size of M), ``npad``, ``leaf``, ``D``, ``leaves``
    (the npad / leaf dense diagonal blocks) and ``levels``: levels[d - 1][g] =
    ((U_low, V_low), (U_up, V_up)) for node g of level d.
    """
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    if M.shape != (n, n):
        raise ValueError("square matrix expected")
    npad, D = _levels(n, leaf)
    Mp = np.zeros((npad, npad))
    Mp[:n, :n] = M
    leaves = [Mp[f * leaf:(f + 1) * leaf, f * leaf:(f + 1) * leaf].copy() for f in range(npad // leaf)]
    levels = []
    for d in range(1, D + 1):
        s = npad >> d
        nodes = []
        for g in range(1 << (d - 1)):
            a = 2 * g * s
            low = _truncate(Mp[a + s:a + 2 * s, a:a + s], tol)
            up = _truncate(Mp[a:a + s, a + s:a + 2 * s], tol)
            nodes.append((low, up))
        levels.append(nodes)
    return {"n": n, "npad": npad, "leaf": leaf, "D": D, "leaves": leaves, "levels": levels}


def plr_dense(T):
    """The n x n matrix that the PLR form T represents."""
    npad, leaf = T["npad"], T["leaf"]
    M = np.zeros((npad, npad))
    for f, Lf in enumerate(T["leaves"]):
        M[f * leaf:(f + 1) * leaf, f * leaf:(f + 1) * leaf] = Lf
    for d, nodes in enumerate(T["levels"], start=1):
        s = npad >> d
        for g, ((Ul, Vl), (Uu, Vu)) in enumerate(nodes):
            a = 2 * g * s
            M[a + s:a + 2 * s, a:a + s] = Ul @ Vl.T
            M[a:a + s, a + s:a + 2 * s] = Uu @ Vu.T
    n = T["n"]
    return M[:n, :n]


def plr_apply(T, X):
    """PLR(M) X for X of shape (n, c): leaf blocks dense, every off-diagonal
    block as U (V^T x) -- the O(m log m)-per-column application of §5."""
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    if vec:
        X = X[:, None]
    n, npad, leaf = T["n"], T["npad"], T["leaf"]
    Xp = np.zeros((npad, X.shape[1]))
    Xp[:n] = X
    Y = np.zeros_like(Xp)
    for f, Lf in enumerate(T["leaves"]):
        Y[f * leaf:(f + 1) * leaf] += Lf @ Xp[f * leaf:(f + 1) * leaf]
    for d, nodes in enumerate(T["levels"], start=1):
        s = npad >> d
        for g, ((Ul, Vl), (Uu, Vu)) in enumerate(nodes):
            a = 2 * g * s
            Y[a + s:a + 2 * s] += Ul @ (Vl.T @ Xp[a:a + s])
            Y[a:a + s] += Uu @ (Vu.T @ Xp[a + s:a + 2 * s])
    Y = Y[:n]
    return Y[:, 0] if vec else Y


def plr_ranks(T):
    """ranks[d - 1][g] = (rank of the lower block, rank of the upper block)."""
    return [[(Ul.shape[1], Uu.shape[1]) for (Ul, _), (Uu, _) in nodes] for nodes in T["levels"]]


def plr_flops(T):
    """Multiply-adds times two per applied column: leaves plus 2 r s per block."""
    leaf = T["leaf"]
    f = len(T["leaves"]) * leaf * leaf
    for d, nodes in enumerate(T["levels"], start=1):
        s = T["npad"] >> d
        for (Ul, _), (Uu, _) in nodes:
            f += 2 * s * (Ul.shape[1] + Uu.shape[1])
    return 2 * f


def plr_error_bound(T, tol):
    """A priori bound 2 D tol on ||M - PLR(M)||_2 (see the module notes)."""
    return 2.0 * T["D"] * tol


def cascade_plr(Abar, Bbar, C, D, u, N, tol, leaf=16, stages=None, return_stages=False):
    """The cascade of §3 (eqs. (3.2)-(3.4), output y = C v + D u) with the
    stage-k power P_k = Abar^(2^k) applied in PLR form at tolerance ``tol``.

    ``stages``: the stage indices k that use the PLR form (default: all of
    0..N); the others apply P_k densely. Returns y (L x q), and with
    ``return_stages`` also the PLR forms used (None for dense stages).
    """
    Abar = np.asarray(Abar, dtype=np.float64)
    Bbar = np.asarray(Bbar, dtype=np.float64)
    if Bbar.ndim == 1:
        Bbar = Bbar[:, None]
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u[:, None]
    L = u.shape[0]
    P = powers(Abar, N)
    use = set(range(N + 1)) if stages is None else set(stages)
    forms = [plr_compress(P[k], tol, leaf) if k in use else None for k in range(N + 1)]
    V = Bbar @ u.T
    for k in range(N + 1):
        s = 1 << k
        if s > L - 1:
            continue
        prev = V[:, : L - s]
        upd = plr_apply(forms[k], prev) if forms[k] is not None else P[k] @ prev
        Vn = V.copy()
        Vn[:, s:] = V[:, s:] + upd
        V = Vn
    y = (np.asarray(C, dtype=np.float64) @ V).T + u @ np.asarray(D, dtype=np.float64).T
    if return_stages:
        return y, forms
    return y
