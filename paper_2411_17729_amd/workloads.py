"""Seeded synthetic workloads (inputs only).

This module builds the inputs that both the HIP library and the CPU checker
consume: state-space parameters (A, B, C, D), step sizes, sequence lengths,
stage counts and input sequences u. It contains none of the method's
arithmetic (no discretization, no powers, no cascade), only draws from
numpy's ``default_rng`` and the HiPPO matrix of §4, eq. (4.1).

Draw order for every workload: parameter sets (A, B, C, D) first, then the
per-sequence step sizes, lengths and state sizes, then u (and dy where a
workload has a cotangent).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def hippo_legs(m: int, one_based: bool = True):
    """HiPPO matrix of §4, eq. (4.1), and the input vector b_n = sqrt(2n+1).

    A[n,k] = -sqrt(2n+1) sqrt(2k+1) for n > k, -(n+1) for n == k, 0 for n < k,
    with 1 <= n, k <= m as the paper states (``one_based=True``); the 0-based
    variant is the common LegS convention and is kept for comparison only.
    Returns (A of shape (m, m), b of shape (m,)).
    """
    off = 1 if one_based else 0
    n = np.arange(m, dtype=np.float64) + off
    r = np.sqrt(2.0 * n + 1.0)
    A = -np.tril(np.outer(r, r), k=-1)
    A[np.diag_indices(m)] = -(n + 1.0)
    return A, r.copy()


@dataclass
class ParamSet:
    """Continuous-time (or already discrete, when ``given``) parameters, FP64."""
    A: np.ndarray  # (m, m)
    B: np.ndarray  # (m, p)
    C: np.ndarray  # (q, m)
    D: np.ndarray  # (q, p)

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def p(self):
        return self.B.shape[1]

    @property
    def q(self):
        return self.C.shape[0]


@dataclass
class Sequence:
    param_set: int
    delta: float
    L: int
    N: int
    u: np.ndarray  # (L, p) float64


@dataclass
class Workload:
    name: str
    sets: List[ParamSet]
    seqs: List[Sequence]
    given: bool = False  # True: (A, B) are already (Abar, Bbar)
    dy: Optional[List[np.ndarray]] = None
    meta: dict = field(default_factory=dict)

    @property
    def total_steps(self):
        return int(sum(s.L for s in self.seqs))


def _normal(rng, shape, var):
    return rng.standard_normal(shape) * math.sqrt(var)


def plain_fp64(seed=0, m=64, L=4096, N=11, delta=1e-2):
    """One HiPPO-LegS sequence: m=64, B_n = sqrt(2n+1), p=q=1, C ~ N(0,1/m),
    D ~ N(0,1), delta = 1e-2, u ~ N(0,1), L=4096, N=11 (degree 4095)."""
    rng = np.random.default_rng(seed)
    A, b = hippo_legs(m)
    C = _normal(rng, (1, m), 1.0 / m)
    D = _normal(rng, (1, 1), 1.0)
    ps = ParamSet(A, b[:, None].copy(), C, D)
    u = rng.standard_normal((L, 1))
    return Workload("hippo_m64_L4096_fp64", [ps], [Sequence(0, delta, L, N, u)],
                    meta={"seed": seed})


def batched(seed=0, batch=16, m=256, L=16384, N=13, p=8, q=8,
            log10_delta=(-3.0, -1.0)):
    """Shared HiPPO-LegS parameters, one step size per sequence:
    m=256, p=q=8, B, C, D ~ N(0,1/m); delta log-uniform in [1e-3, 1e-1];
    16 sequences of L=16384, N=13; u ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    A, _ = hippo_legs(m)
    B = _normal(rng, (m, p), 1.0 / m)
    C = _normal(rng, (q, m), 1.0 / m)
    D = _normal(rng, (q, p), 1.0 / m)
    ps = ParamSet(A, B, C, D)
    deltas = 10.0 ** rng.uniform(log10_delta[0], log10_delta[1], size=batch)
    seqs = [Sequence(0, float(d), L, N, None) for d in deltas]
    for s in seqs:
        s.u = rng.standard_normal((L, p))
    return Workload(f"hippo_m{m}_p{p}_B{batch}_L{L}", [ps], seqs, meta={"seed": seed})


def stability(seed=0, batch=4, m=128, L=65536, N=15, lam_lo=0.99, lam_hi=0.99999,
              lam_top=1.0 + 1e-5):
    """Structured diagonal-plus-rank-2 Abar with one eigenvalue past 1.

    Abar = diag(lambda) + U V^T, U (m x 2) nonzero on the first m/2 rows, V
    (m x 2) nonzero on the last m/2 rows, entries N(0, 1/m): the rank-2 part
    lives in the upper-right block, so Abar is block upper triangular and its
    eigenvalues are exactly lambda. lambda_i ~ U[lam_lo, lam_hi] for i < m-1
    and lambda_{m-1} = lam_top. Bbar, C ~ N(0, 1/m), D ~ N(0, 1); p = q = 1.
    The parameters are the discrete ones (``given``).
    """
    rng = np.random.default_rng(seed)
    h = m // 2
    lam = rng.uniform(lam_lo, lam_hi, size=m)
    lam[m - 1] = lam_top
    U = np.zeros((m, 2))
    V = np.zeros((m, 2))
    U[:h] = _normal(rng, (h, 2), 1.0 / m)
    V[h:] = _normal(rng, (m - h, 2), 1.0 / m)
    Abar = np.diag(lam) + U @ V.T
    Bbar = _normal(rng, (m, 1), 1.0 / m)
    C = _normal(rng, (1, m), 1.0 / m)
    D = _normal(rng, (1, 1), 1.0)
    ps = ParamSet(Abar, Bbar, C, D)
    seqs = [Sequence(0, 0.0, L, N, None) for _ in range(batch)]
    for s in seqs:
        s.u = rng.standard_normal((L, 1))
    return Workload(f"diag_rank2_m{m}_B{batch}_L{L}", [ps], seqs, given=True,
                    meta={"seed": seed, "eigenvalues": lam})


def backward(seed=0, batch=8, m=128, L=8192, N=12, p=4, q=4, delta=5e-3):
    """Shared HiPPO-LegS parameters for the gradient check: m=128, p=q=4,
    B, C, D ~ N(0,1/m), delta=5e-3, N=12, 8 sequences of L=8192, u and the
    output cotangent dy ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    A, _ = hippo_legs(m)
    B = _normal(rng, (m, p), 1.0 / m)
    C = _normal(rng, (q, m), 1.0 / m)
    D = _normal(rng, (q, p), 1.0 / m)
    ps = ParamSet(A, B, C, D)
    seqs = [Sequence(0, delta, L, N, None) for _ in range(batch)]
    for s in seqs:
        s.u = rng.standard_normal((L, p))
    dy = [rng.standard_normal((L, q)) for _ in range(batch)]
    return Workload(f"hippo_m{m}_p{p}_B{batch}_L{L}_bwd", [ps], seqs, dy=dy,
                    meta={"seed": seed})


def ragged(seed=0, n_seq=256, L_range=(512, 65536), m_choices=(64, 128, 256),
           p=4, q=4, log10_delta=(-3.0, -1.0), with_dy=True):
    """Ragged batch: per sequence its own HiPPO-LegS parameter set of size m_s
    drawn from ``m_choices``, B, C, D ~ N(0,1/m_s), L_s log-uniform in
    ``L_range``, delta_s log-uniform in [1e-3, 1e-1], N_s = ceil(log2 L_s) - 1."""
    rng = np.random.default_rng(seed)
    ms = rng.choice(np.asarray(m_choices), size=n_seq)
    sets = []
    for m in ms:
        A, _ = hippo_legs(int(m))
        B = _normal(rng, (m, p), 1.0 / m)
        C = _normal(rng, (q, m), 1.0 / m)
        D = _normal(rng, (q, p), 1.0 / m)
        sets.append(ParamSet(A, B, C, D))
    deltas = 10.0 ** rng.uniform(log10_delta[0], log10_delta[1], size=n_seq)
    Ls = np.rint(np.exp(rng.uniform(math.log(L_range[0]), math.log(L_range[1]),
                                    size=n_seq))).astype(np.int64)
    seqs = []
    for i in range(n_seq):
        L = int(Ls[i])
        N = max(0, int(math.ceil(math.log2(L))) - 1)
        seqs.append(Sequence(i, float(deltas[i]), L, N, None))
    for s in seqs:
        s.u = rng.standard_normal((s.L, p))
    dy = [rng.standard_normal((s.L, q)) for s in seqs] if with_dy else None
    return Workload(f"ragged_{n_seq}", sets, seqs, dy=dy, meta={"seed": seed})


def random_small(seed=0, m=6, p=2, q=3, L=40, N=3, n_seq=1, delta=0.1,
                 contraction=0.9, given=True):
    """Small dense random systems for exhaustive checks. With ``given`` the
    parameters are discrete (Abar scaled to spectral norm ``contraction``);
    otherwise A is a random stable continuous matrix."""
    rng = np.random.default_rng(seed)
    if given:
        A = rng.standard_normal((m, m))
        A *= contraction / np.linalg.norm(A, 2)
    else:
        A = rng.standard_normal((m, m)) / math.sqrt(m) - 1.5 * np.eye(m)
    B = rng.standard_normal((m, p))
    C = rng.standard_normal((q, m))
    D = rng.standard_normal((q, p))
    ps = ParamSet(A, B, C, D)
    seqs = [Sequence(0, delta, L, N, None) for _ in range(n_seq)]
    for s in seqs:
        s.u = rng.standard_normal((L, p))
    dy = [rng.standard_normal((L, q)) for _ in range(n_seq)]
    return Workload(f"random_m{m}", [ps], seqs, given=given, dy=dy, meta={"seed": seed})
