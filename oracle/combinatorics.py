"""Pure-Python hashing of bosonic configurations (test infrastructure only).

Follows Sec. III of arXiv:2005.13679:
  * Eq. (nc):  N_c(N, M) = (N + M - 1)! / (N! (M - 1)!),  N_c(n, 0) = 0;
  * Algorithm 1: occupation vector -> index (sum of particle costs);
  * Algorithm 2: index -> occupation vector (greedy descent).
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


def hash_alg1(occ, N: int | None = None) -> int:
    """Algorithm 1.  Scan orbitals m = M-1 .. 1; for each particle found in
    orbital m add the cost N_c(s, m), s being the particles still in the
    basket, then remove the particle from the basket."""
    M = len(occ)
    if N is None:
        N = sum(occ)
    k = 0
    s = N
    for m in range(M - 1, 0, -1):
        j = occ[m]
        while j > 0:
            k += nc(s, m)
            s -= 1
            j -= 1
    return k


def unhash_alg2(beta: int, N: int, M: int) -> list[int]:
    """Algorithm 2.  Starting from orbital M-1, move a particle from the
    basket into orbital m while the remaining index covers its cost N_c(s, m);
    otherwise go down one orbital.  Leftover particles go to orbital 0."""
    if not (0 <= beta < nc(N, M)):
        raise ValueError("index out of range")
    n = [0] * M
    k = beta
    m = M - 1
    s = N
    while k > 0:
        while k - nc(s, m) < 0:
            m -= 1
        k -= nc(s, m)
        n[m] += 1
        s -= 1
    if s > 0:
        n[0] += s
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
