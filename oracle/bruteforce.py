"""Exact density of states of tiny Potts lattices by complete enumeration.

Test infrastructure (see oracle/__init__.py).  Eq. (2) of the paper,
H = -sum over nearest-neighbour pairs delta(s_i, s_j), on an L x L periodic
lattice with each bond counted once.  All q^N configurations are listed as
base-q digit strings and their energies histogrammed; g(E) is returned as
exact integer counts over E = -2N .. 0.  Feasible for q^N up to a few 10^6.
"""
import numpy as np


def potts_energies(L, q, chunk=1 << 20):
    """Energies of all q^(L*L) configurations, in enumeration order."""
    N = L * L
    total = q ** N
    if total > 50_000_000:
        raise ValueError("too many configurations to enumerate")
    out = np.empty(total, dtype=np.int32)
    for first in range(0, total, chunk):
        idx = np.arange(first, min(first + chunk, total), dtype=np.int64)
        digits = np.empty((idx.size, N), dtype=np.int8)
        rest = idx.copy()
        for i in range(N):
            digits[:, i] = rest % q
            rest //= q
        s = digits.reshape(-1, L, L)
        e = -(s == np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s == np.roll(s, -1, axis=1)).sum(axis=(1, 2))
        out[first:first + idx.size] = e
    return out


def potts_dos(L, q):
    """Exact g(E) for E = -2N..0 as int64 counts (index b <-> E = -2N + b)."""
    N = L * L
    e = potts_energies(L, q)
    return np.bincount(e + 2 * N, minlength=2 * N + 1).astype(np.int64)


def potts_partition(L, q, T):
    """Brute-force ln Z, U and C_v at temperatures T, summed over configurations
    directly (not through g(E)), for pinning the thermodynamics routine."""
    e = potts_energies(L, q).astype(np.float64)
    out = []
    for t in np.atleast_1d(T):
        x = -e / t
        mx = x.max()
        w = np.exp(x - mx)
        Z = w.sum()
        U = (w * e).sum() / Z
        var = (w * (e - U) ** 2).sum() / Z
        out.append((mx + np.log(Z), U, var / (t * t)))
    return np.array(out)
