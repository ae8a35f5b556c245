"""Dense brute-force Hamiltonian (test infrastructure only).

Textbook construction, independent of the jump maps and of the operator
algebra in ``mc_oracle.c``: each mode k gets the ladder matrix
a = superdiag(sqrt(1), ..., sqrt(N)) on its (N+1)-dimensional occupation
space, a_k = I x ... x a x ... x I (Kronecker products), and

    H = sum_kl h_kl a+_k a_l + 1/2 sum_ksql g_ksql a+_k a+_s a_q a_l

is assembled as a sparse matrix over all (N+1)^M product states, then
restricted to the states with exactly N particles, ordered by their index.
Only for tiny spaces ((N+1)^M up to a few 10^5).
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from .combinatorics import index_of, nc


def _ladder_ops(N: int, M: int):
    d = N + 1
    a1 = sp.diags(np.sqrt(np.arange(1, d, dtype=np.float64)), 1, shape=(d, d), format="csr")
    eye = sp.identity(d, format="csr")
    ops = []
    for k in range(M):
        mats = [eye] * M
        mats[k] = a1
        A = mats[0]
        for m in mats[1:]:
            A = sp.kron(A, m, format="csr")
        ops.append(A)
    return ops


def _restriction(N: int, M: int):
    """Selection matrix P (D x (N+1)^M): row beta picks the product state
    |n_0 ... n_{M-1}> (mode 0 most significant in the Kronecker order) whose
    occupation vector has index beta."""
    d = N + 1
    D = nc(N, M)
    rows, cols = [], []
    for occ in itertools.product(range(d), repeat=M):
        if sum(occ) != N:
            continue
        flat = 0
        for o in occ:
            flat = flat * d + o
        rows.append(index_of(list(occ)))
        cols.append(flat)
    P = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(D, d ** M))
    return P


def hamiltonian(N: int, M: int, h, g) -> np.ndarray:
    """Dense D x D matrix <gamma|H|beta>."""
    h = np.asarray(h, dtype=np.complex128).reshape(M, M)
    g = np.asarray(g, dtype=np.complex128).reshape(M, M, M, M)
    a = _ladder_ops(N, M)
    ad = [x.T.tocsr() for x in a]          # real matrices: adjoint = transpose
    P = _restriction(N, M)
    # apply everything to the restricted states only: X = op @ P^T
    PT = P.T.tocsr().astype(np.complex128)
    H = sp.csr_matrix((P.shape[0], P.shape[0]), dtype=np.complex128)
    for k in range(M):
        for l in range(M):
            if h[k, l] != 0:
                H = H + h[k, l] * (P @ (ad[k] @ (a[l] @ PT)))
    al_cache = {}
    for q in range(M):
        for l in range(M):
            al_cache[(q, l)] = a[q] @ (a[l] @ PT)
    for k in range(M):
        for s in range(M):
            left = P @ (ad[k] @ ad[s])
            for q in range(M):
                for l in range(M):
                    c = g[k, s, q, l]
                    if c != 0:
                        H = H + (0.5 * c) * (left @ al_cache[(q, l)])
    return H.toarray()


def number_operator_check(N: int, M: int) -> np.ndarray:
    """sum_k a+_k a_k restricted to N particles (should be N * identity)."""
    a = _ladder_ops(N, M)
    P = _restriction(N, M)
    PT = P.T.tocsr()
    Nop = sum(P @ (a[k].T @ (a[k] @ PT)) for k in range(M))
    return Nop.toarray()
