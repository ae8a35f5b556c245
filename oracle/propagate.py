"""Time steps C(t + dt) = exp(-i H dt) C(t) (test infrastructure only).

Sec. II of arXiv:2005.13679 names the Short Iterative Lanczos (SIL)
integrator as the time-dependent use of repeated H.C.  Two references:

- ``expm_step``: the definition, exp(-i H dt) C with the dense H of
  ``oracle.dense`` and scipy's matrix exponential (tiny spaces only);
- ``sil_step``: Park and Light's SIL step written out: Lanczos with full
  reorthogonalisation from C/|C|, the k x k tridiagonal T, y = exp(-i T dt)
  e_0 (scipy's expm on the small dense T), C(t + dt) = |C| V y, and the
  a-posteriori error estimate |C| beta_k |y_{k-1}|.  ``apply_h`` is any H.C
  (the oracle's operator algebra in the tests).
"""

from __future__ import annotations

import numpy as np
from scipy.linalg import expm


def expm_step(H: np.ndarray, C: np.ndarray, dt: float) -> np.ndarray:
    return expm(-1j * dt * H) @ C


def sil_step(apply_h, C: np.ndarray, dt: float, k: int, tol: float | None = None):
    """Returns (C(t+dt), krylov_dim, error_estimate).  Exactly k vectors
    unless the Krylov space is exhausted, or (tol given) the estimate drops
    below tol first."""
    D = C.size
    norm_c = np.linalg.norm(C)
    if norm_c == 0.0:
        return C.copy(), 0, 0.0
    k = max(1, min(k, D))
    V = np.zeros((k + 1, D), dtype=np.complex128)
    V[0] = C / norm_c
    alphas, betas = [], []
    y, err, m = None, np.inf, 0
    for j in range(k):
        w = apply_h(V[j])
        alphas.append(np.vdot(V[j], w).real)
        for _ in range(2):
            w = w - V[: j + 1].T @ (V[: j + 1].conj() @ w)
        b = np.linalg.norm(w)
        m = j + 1
        T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
        y = expm(-1j * dt * T)[:, 0]
        err = norm_c * b * abs(y[-1])
        if b < 1e-14 * max(1.0, abs(alphas[-1])):
            err = 0.0
            break
        if tol is not None and err < tol:
            break
        betas.append(b)
        V[j + 1] = w / b
    return norm_c * (V[:m].T @ y), m, err
