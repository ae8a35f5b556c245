"""Pins for the oracle's one- and two-body density matrices (CPU only)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import combinatorics as cb
from oracle import dense


def closed_form_index(occ):
    S = np.cumsum(occ)
    return sum(math.comb(int(S[m]) + m, m) - math.comb(int(S[m - 1]) + m, m)
               for m in range(1, len(occ)))


def appendix_b(N, M, C):
    """The element rules of App. B (reduced density matrices), written out
    case by case with the jump notation beta_a^b / beta_ab^cd, using an
    enumeration and index formula independent of the oracle.  Returns the
    dictionary of rho1 / rho2 elements the appendix covers."""
    configs = list(cb.compositions(N, M))
    idx = {tuple(c): closed_form_index(c) for c in configs}

    def jump(c, rem, add):
        m = list(c)
        for a in rem:
            m[a] -= 1
        for a in add:
            m[a] += 1
        return idx[tuple(m)]

    out = {}
    for k in range(M):
        out[("kk", k)] = sum(abs(C[idx[tuple(c)]]) ** 2 * c[k] for c in configs)
        out[("kkkk", k)] = sum(abs(C[idx[tuple(c)]]) ** 2 * (c[k] ** 2 - c[k]) for c in configs)
        for s in range(M):
            if s == k:
                continue
            out[("ksks", k, s)] = sum(abs(C[idx[tuple(c)]]) ** 2 * c[k] * c[s] for c in configs)
    for k in range(M):
        for l in range(M):
            if k == l:
                continue
            v = 0
            w = 0
            for c in configs:
                if c[k] >= 1:
                    b = idx[tuple(c)]
                    v += np.conj(C[b]) * C[jump(c, [k], [l])] * math.sqrt((c[l] + 1) * c[k])
                    # rho_kkkl = sum C*_b C_{b_k^l} (n_k - 1) sqrt(n_k (n_l + 1))
                    w += np.conj(C[b]) * C[jump(c, [k], [l])] * (c[k] - 1) * math.sqrt(c[k] * (c[l] + 1))
            out[("kl", k, l)] = v
            out[("kkkl", k, l)] = w
    # rho_kkqq, k != q: here with the factor sqrt(n_k(n_k-1)(n_q+1)(n_q+2)) that the
    # operator algebra gives (the appendix prints the sum without it)
    for k in range(M):
        for q in range(M):
            if k == q:
                continue
            v = 0
            for c in configs:
                if c[k] >= 2:
                    b = idx[tuple(c)]
                    v += np.conj(C[b]) * C[jump(c, [k, k], [q, q])] * math.sqrt(
                        c[k] * (c[k] - 1) * (c[q] + 1) * (c[q] + 2))
            out[("kkqq", k, q)] = v
    # rho_kkql, q != l, k not in {q, l}
    for k in range(M):
        for q in range(M):
            for l in range(M):
                if len({k, q, l}) < 3:
                    continue
                v = 0
                for c in configs:
                    if c[k] >= 2:
                        b = idx[tuple(c)]
                        v += np.conj(C[b]) * C[jump(c, [k, k], [q, l])] * math.sqrt(
                            (c[k] - 1) * c[k] * (c[q] + 1) * (c[l] + 1))
                out[("kkql", k, q, l)] = v
    # rho_ksqq, k != s, q not in {k, s}
    for k in range(M):
        for s in range(M):
            for q in range(M):
                if len({k, s, q}) < 3:
                    continue
                v = 0
                for c in configs:
                    if c[k] >= 1 and c[s] >= 1:
                        b = idx[tuple(c)]
                        v += np.conj(C[b]) * C[jump(c, [k, s], [q, q])] * math.sqrt(
                            c[k] * c[s] * (c[q] + 1) * (c[q] + 2))
                out[("ksqq", k, s, q)] = v
    # rho_ksss (k != s) and rho_kssl (k, s, l distinct)
    for k in range(M):
        for s in range(M):
            if k == s:
                continue
            v = 0
            for c in configs:
                if c[k] >= 1:
                    b = idx[tuple(c)]
                    v += np.conj(C[b]) * C[jump(c, [k], [s])] * c[s] * math.sqrt(c[k] * (c[s] + 1))
            out[("ksss", k, s)] = v
            for l in range(M):
                if l in (k, s):
                    continue
                v = 0
                for c in configs:
                    if c[k] >= 1:
                        b = idx[tuple(c)]
                        v += np.conj(C[b]) * C[jump(c, [k], [l])] * c[s] * math.sqrt(c[k] * (c[l] + 1))
                out[("kssl", k, s, l)] = v
    # rho_ksql, all four distinct
    for k in range(M):
        for s in range(M):
            for q in range(M):
                for l in range(M):
                    if len({k, s, q, l}) < 4:
                        continue
                    v = 0
                    for c in configs:
                        if c[k] >= 1 and c[s] >= 1:
                            b = idx[tuple(c)]
                            v += np.conj(C[b]) * C[jump(c, [k, s], [q, l])] * math.sqrt(
                                c[k] * c[s] * (c[q] + 1) * (c[l] + 1))
                    out[("ksql", k, s, q, l)] = v
    return out


def test_appendix_b_element_rules(oracle_native):
    """rho1/rho2 follow the per-case rules of App. B.  Index conventions:
    the appendix writes rho_{ksql} for <a+_k a+_s a_q a_l> where the
    destroyed particles leave k, s and reappear in q, l when read as the jump
    beta_{ks}^{ql} from the bra's configuration; for bosons the pairs are
    symmetric so this matches the operator definition up to k<->s, q<->l."""
    N, M = 5, 4
    C, _, _ = W.random_instance(N, M, 21)
    r1 = oracle_native.rho1(N, M, C)
    r2 = oracle_native.rho2(N, M, C)
    ab = appendix_b(N, M, C)
    tol = 1e-13
    for key, v in ab.items():
        kind = key[0]
        if kind == "kk":
            k = key[1]
            got = r1[k, k]
        elif kind == "kl":
            _, k, l = key
            got = r1[k, l]
        elif kind == "kkkk":
            k = key[1]
            got = r2[k, k, k, k]
        elif kind == "ksks":
            _, k, s = key
            got = r2[k, s, k, s]
        elif kind == "kkqq":
            _, k, q = key
            got = r2[k, k, q, q]
        elif kind == "kkql":
            _, k, q, l = key
            got = r2[k, k, q, l]
        elif kind == "kkkl":
            _, k, l = key
            got = r2[k, k, k, l]
        elif kind == "ksqq":
            _, k, s, q = key
            got = r2[k, s, q, q]
        elif kind == "ksss":
            _, k, s = key
            got = r2[k, s, s, s]
        elif kind == "kssl":
            _, k, s, l = key
            got = r2[k, s, s, l]
        elif kind == "ksql":
            _, k, s, q, l = key
            got = r2[k, s, q, l]
        assert abs(got - v) < tol, (key, got, v)


def test_rho_from_dense_ladder_operators(oracle_native):
    N, M = 4, 3
    C, _, _ = W.random_instance(N, M, 5)
    r1 = oracle_native.rho1(N, M, C)
    r2 = oracle_native.rho2(N, M, C)
    for k in range(M):
        for l in range(M):
            h = np.zeros((M, M), complex)
            h[k, l] = 1
            Hk = dense.hamiltonian(N, M, h, np.zeros((M,) * 4))
            assert abs(np.vdot(C, Hk @ C) - r1[k, l]) < 1e-13
    for (k, s, q, l) in [(0, 1, 2, 0), (1, 1, 0, 2), (2, 0, 0, 2), (0, 0, 0, 0), (2, 1, 1, 1)]:
        g = np.zeros((M,) * 4, complex)
        g[k, s, q, l] = 2.0       # the Hamiltonian carries 1/2
        Hk = dense.hamiltonian(N, M, np.zeros((M, M)), g)
        assert abs(np.vdot(C, Hk @ C) - r2[k, s, q, l]) < 1e-13


@pytest.mark.parametrize("N,M,seed", [(10, 5, 0), (6, 4, 3), (3, 6, 9)])
def test_density_matrix_invariants(oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    r1 = oracle_native.rho1(N, M, C)
    r2 = oracle_native.rho2(N, M, C)
    assert abs(np.trace(r1) - N) < 1e-12
    assert np.allclose(r1, r1.conj().T, atol=1e-13)
    assert np.allclose(np.einsum("kssl->kl", r2), (N - 1) * r1, atol=1e-12)
    assert abs(np.einsum("kssk->", r2) - N * (N - 1)) < 1e-11
    assert np.allclose(r2, r2.transpose(1, 0, 2, 3), atol=1e-13)
    assert np.allclose(r2, r2.transpose(0, 1, 3, 2), atol=1e-13)
    assert np.allclose(r2, r2.transpose(2, 3, 0, 1).conj(), atol=1e-13)
    # the energy from the density matrices equals <C|H C>
    HC = oracle_native.apply_h(N, M, h, g, C)
    E1 = np.vdot(C, HC)
    E2 = np.sum(h * r1) + 0.5 * np.sum(g * r2)
    assert abs(E1 - E2) < 1e-12 * max(1.0, abs(E1))


def test_rho2_selected_elements(oracle_native):
    N, M = 10, 5
    C, _, _ = W.random_instance(N, M, 0)
    full = oracle_native.rho2(N, M, C).reshape(-1)
    idx = np.array([0, 7, 311, 624, 100], dtype=np.int64)
    assert np.array_equal(oracle_native.rho2_elements(N, M, C, idx), full[idx])
