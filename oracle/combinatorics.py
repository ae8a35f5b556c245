"""Pure-Python hashing of bosonic configurations (test infrastructure only).

Follows Sec. III of arXiv:2005.13679:
  * Eq. (nc):  N_c(N, M) = (N + M - 1)! / (N! (M - 1)!),  N_c(n, 0) = 0;
  * Eq. (TotalCost): occupation vector -> index (sum of particle costs),
    the map of Algorithm 1;
  * its inverse (the map of Algorithm 2) by bisection on that index.
Indices and orbitals are 0-based as in the algorithms.
"""

from __future__ import annotations

from math import factorial


def nc(n: int, m: int) -> int:
    """Eq. (nc) written with factorials; N_c(n, 0) = 0 (Eq. TotalCost)."""
    if m <= 0 or n < 0:
        return 0
    return factorial(n + m - 1) // (factorial(n) * factorial(m - 1))


def dim(N: int, M: int) -> int:
    """Size of the multiconfigurational space of N bosons in M orbitals."""
    return nc(N, M)


def index_of(occ) -> int:
    """Configuration -> index from Eq. (TotalCost): the particles, listed by
    nondecreasing orbital, cost N_c(i, p_i) each (i = 1..N); the index is the
    total.  (The map of Algorithm 1, evaluated from the lowest orbital up.)"""
    positions = [m for m in range(len(occ)) for _ in range(occ[m])]
    return total_cost(positions, len(occ))


def config_of(beta: int, N: int, M: int) -> list[int]:
    """Index -> configuration by bisection on ``index_of``.  Orbital M-1 is
    the most significant; with the orbitals above m fixed, the first
    configuration with n_m = t keeps the rest in orbital 0 and its index
    grows with t, so n_m is the largest t whose first configuration does not
    exceed beta.  The remainder goes to orbital 0."""
    if not (0 <= beta < nc(N, M)):
        raise ValueError("index out of range")
    n = [0] * M
    left = N
    for m in range(M - 1, 0, -1):
        lo, hi = 0, left
        while lo < hi:
            mid = (lo + hi + 1) // 2
            n[m], n[0] = mid, left - mid
            if index_of(n) <= beta:
                lo = mid
            else:
                hi = mid - 1
        n[m], n[0] = lo, 0
        left -= lo
    n[0] = left
    return n


def compositions(N: int, M: int):
    """All occupation vectors with sum N over M orbitals, generated
    recursively (orbital 0 outermost).  Independent of the hash order."""
    if M == 1:
        yield [N]
        return
    for first in range(N + 1):
        for rest in compositions(N - first, M - 1):
            yield [first] + rest


def total_cost(positions, M: int) -> int:
    """Eq. (TotalCost): I(p) = sum_n N_c(n, p_n) for the sorted particle
    positions 0 <= p_1 <= ... <= p_N < M."""
    return sum(nc(i + 1, p) for i, p in enumerate(sorted(positions)))
