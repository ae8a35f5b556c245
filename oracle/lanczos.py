"""Lanczos ground state with full reorthogonalisation (test infrastructure only).

Sec. VI of arXiv:2005.13679: the ground state of the Lieb-Liniger gas is found
by Lanczos tridiagonalisation with complete reorthogonalisation, the
tridiagonal matrix being diagonalised by a dense eigensolver (here
``scipy.linalg.eigh_tridiagonal`` in place of LAPACK).

The paper caps the iteration count at dim/8; we stop earlier once the lowest
Ritz value is converged (relative change < ``tol`` and residual
beta_j * |s_j| < ``res_tol``), with ``max_iter`` as a hard cap.
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos_ground(apply_h, v0: np.ndarray, max_iter: int = 300,
                   tol: float = 1e-12, res_tol: float = 1e-9):
    """Lowest eigenvalue of the Hermitian operator ``apply_h``.

    Returns (E0, alphas, betas, iterations).
    """
    D = v0.size
    cap = max(2, min(max_iter, D))
    V = np.zeros((cap, D), dtype=np.complex128)
    v = v0.astype(np.complex128) / np.linalg.norm(v0)
    V[0] = v
    alphas, betas = [], []
    prev = None
    e0 = None
    for j in range(cap):
        w = apply_h(V[j])
        a = np.vdot(V[j], w).real
        alphas.append(a)
        # full reorthogonalisation (two passes of classical Gram-Schmidt)
        for _ in range(2):
            w = w - V[: j + 1].T @ (V[: j + 1].conj() @ w)
        b = np.linalg.norm(w)
        evals, evecs = eigh_tridiagonal(np.array(alphas), np.array(betas)) if j > 0 else \
            (np.array([a]), np.ones((1, 1)))
        e0 = evals[0]
        resid = b * abs(evecs[-1, 0])
        if prev is not None and abs(e0 - prev) <= tol * max(1.0, abs(e0)) and resid < res_tol:
            return e0, np.array(alphas), np.array(betas), j + 1
        prev = e0
        if b < 1e-14 or j + 1 == cap:
            break
        betas.append(b)
        V[j + 1] = w / b
    return e0, np.array(alphas), np.array(betas), len(alphas)


def lanczos_recurrence(apply_h, v0: np.ndarray, steps: int):
    """Plain three-term recurrence without reorthogonalisation.

    Returns (alphas, betas) of ``steps`` iterations: alpha_j = <v_j|H v_j>,
    w = H v_j - alpha_j v_j - beta_{j-1} v_{j-1}, beta_j = |w|."""
    v = v0.astype(np.complex128) / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    b_prev = 0.0
    alphas, betas = [], []
    for _ in range(steps):
        w = apply_h(v)
        a = np.vdot(v, w).real
        w = w - a * v - b_prev * v_prev
        b = np.linalg.norm(w)
        alphas.append(a)
        betas.append(b)
        v_prev, v, b_prev = v, w / b, b
    return np.array(alphas), np.array(betas)
