"""The closed forms behind the table-free apply (mc_apply_H_direct), checked
on the CPU against the oracle's Algorithms 1 and 2 and its single-jump map:

  index  g = D - 1 - sum_{m=0}^{M-2} C(S_m + m, m + 1),  S_m = n_0 + ... + n_m
  inverse  S_m greedily from J = D - 1 - g, m = M-2 .. 1, then S_0 = rest
  target of a jump  g + sum_m [G_m(S_m) - G_m(S_m + Delta_m)]

and the bound that keeps the kernel's double-precision products exact.  The
kernel's own arithmetic is checked on the GPU (test_gpu_direct.py)."""

import math

import numpy as np
import pytest

from oracle import native


def G(m, x):
    return math.comb(x + m, m + 1)


def closed_index(n, N):
    M = len(n)
    D = math.comb(N + M - 1, M - 1)
    S = np.cumsum(n)
    return D - 1 - sum(G(m, int(S[m])) for m in range(M - 1))


def greedy_prefix(g, N, M):
    """The kernel's inverse: bitwise search for the largest S_m with
    P_m(S_m) <= J (m+1)!, S_m <= S_{m+1}."""
    D = math.comb(N + M - 1, M - 1)
    J = D - 1 - g
    S = [0] * M
    S[M - 1] = N
    nbits = N.bit_length()
    for m in range(M - 2, 0, -1):
        lim = J * math.factorial(m + 1)
        s = 0
        for b in range(nbits - 1, -1, -1):
            c = s | (1 << b)
            if c <= S[m + 1] and math.prod(c + i for i in range(m + 1)) <= lim:
                s = c
        S[m] = s
        J -= G(m, s)
    if M >= 2:
        S[0] = J
    return np.diff([0] + S)


SPACES = [(1, 1), (3, 1), (1, 4), (4, 3), (6, 4), (5, 5), (3, 7), (4, 8), (12, 2), (9, 3)]


@pytest.mark.parametrize("N,M", SPACES)
def test_closed_form_index_is_alg1(N, M):
    occ = native.occ_rows(N, M)               # Alg. 2 for every index
    for g, n in enumerate(occ):
        assert closed_index(n, N) == g


@pytest.mark.parametrize("N,M", SPACES)
def test_greedy_inverse_is_alg2(N, M):
    occ = native.occ_rows(N, M)
    for g, n in enumerate(occ):
        assert np.array_equal(greedy_prefix(g, N, M), n)


def prefix_delta(m, removed, added):
    return sum(a <= m for a in added) - sum(r <= m for r in removed)


def target(n, N, removed, added):
    M = len(n)
    S = np.cumsum(n)
    t = closed_index(n, N)
    for m in range(M - 1):
        d = prefix_delta(m, removed, added)
        if d:
            t += G(m, int(S[m])) - G(m, int(S[m]) + d)
    return t


@pytest.mark.parametrize("N,M", [(4, 3), (6, 4), (5, 5), (3, 7), (2, 8)])
def test_index_delta_gives_single_jump_map(N, M):
    occ = native.occ_rows(N, M)
    t1 = native.t1_rows(N, M)
    for g, n in enumerate(occ):
        for a in range(M):
            for b in range(M):
                if n[a] >= 1:
                    assert target(n, N, [a], [b]) == t1[g, a, b]


@pytest.mark.parametrize("N,M", [(4, 4), (5, 5), (3, 6), (4, 8)])
def test_index_delta_gives_double_jumps(N, M):
    """Every true double jump {k,s} -> {q,l} against Alg. 1 on the moved vector."""
    occ = native.occ_rows(N, M)
    for g, n in enumerate(occ):
        for k in range(M):
            for s in range(k, M):
                if (n[k] < 2) if k == s else (n[k] < 1 or n[s] < 1):
                    continue
                for q in range(M):
                    for l in range(q, M):
                        if {q, l} & {k, s}:
                            continue
                        m = n.copy()
                        m[k] -= 1
                        m[s] -= 1
                        m[q] += 1
                        m[l] += 1
                        assert target(n, N, [k, s], [q, l]) == native.hash_occ(m, N)


@pytest.mark.parametrize("M", range(2, 9))
def test_products_exact_in_double(M):
    """Largest N with D < 2^31: every P_m(x) = x..(x+m) (x <= N, m <= M-2) and
    J (m+1)! stay below 2^53, so the kernel's double arithmetic is exact."""
    lo, hi = 1, 2 ** 31                      # largest N with C(N+M-1, M-1) < 2^31
    while lo < hi:
        mid = (lo + hi + 1) // 2
        lo, hi = (mid, hi) if math.comb(mid + M - 1, M - 1) < 2 ** 31 else (lo, mid - 1)
    N = lo
    D = math.comb(N + M - 1, M - 1)
    assert D < 2 ** 31
    for m in range(M - 1):
        assert math.prod(N + i for i in range(m + 1)) < 2 ** 53
        assert (D - 1) * math.factorial(m + 1) < 2 ** 53
