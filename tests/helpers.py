"""Shared test helpers: oracle evaluation of a workload and error metrics."""

import numpy as np

import oracle as O


def rel_err(a, b):
    """||a - b||_F / ||b||_F (b is the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def discretized(wl, seq, disc=None):
    ps = wl.sets[seq.param_set]
    if disc is None:
        disc = "given" if wl.given else "trapezoid"
    if disc == "given":
        return ps.A, ps.B
    return (O.zoh if disc == "zoh" else O.trapezoid)(ps.A, ps.B, seq.delta)


def oracle_outputs(wl, u_override=None, method="auto", disc=None):
    """Per-sequence FP64 outputs (L, q). ``method``: 'truncated', 'recursion'
    or 'auto' (recursion when the window covers the sequence, else the
    truncated sum)."""
    out = []
    cache = {}
    for i, s in enumerate(wl.seqs):
        key = (s.param_set, s.delta)
        if key not in cache:
            cache[key] = discretized(wl, s, disc)
        Abar, Bbar = cache[key]
        ps = wl.sets[s.param_set]
        u = s.u if u_override is None else u_override[i]
        T = 1 << (s.N + 1)
        use_rec = method == "recursion" or (method == "auto" and T >= s.L)
        if use_rec:
            y, _ = O.recursion(Abar, Bbar, ps.C, ps.D, u)
        else:
            y = O.truncated_sum(Abar, Bbar, ps.C, ps.D, u, s.N)
        out.append(y)
    return out


def state_part(wl, ys, u_override=None):
    """y - D u per sequence, the part of the output that goes through the state."""
    res = []
    for i, (s, y) in enumerate(zip(wl.seqs, ys)):
        u = s.u if u_override is None else u_override[i]
        res.append(y - u @ wl.sets[s.param_set].D.T)
    return res


def max_rel(got, ref):
    return max(rel_err(g, r) for g, r in zip(got, ref))
