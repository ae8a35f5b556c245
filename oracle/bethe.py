"""Bethe-ansatz ground-state energy of the Lieb-Liniger gas (test infrastructure only).

Eqs. (LLsystem) and (LLE0) of arXiv:2005.13679 with hbar = m = 1:

    k_j = (2 pi / L) I_j - (2 / L) sum_i arctan((k_j - k_i) / c),
    I_j = j - (N + 1)/2,  j = 1..N,
    E_0 = (1/2) sum_j k_j^2,

c being the contact strength of  c * sum_{i<j} delta(x_i - x_j).  Solved by
damped Newton iteration with the analytic Jacobian, starting from the hard-core
(Tonks-Girardeau) momenta scaled by c / (c + 2N/L).
"""

from __future__ import annotations

import math

import numpy as np


def quantum_numbers(N: int) -> np.ndarray:
    return np.arange(1, N + 1) - (N + 1) / 2.0


def residual(k: np.ndarray, c: float, L: float) -> np.ndarray:
    I = quantum_numbers(k.size)
    d = (k[:, None] - k[None, :]) / c
    return k - (2.0 * math.pi / L) * I + (2.0 / L) * np.arctan(d).sum(axis=1)


def jacobian(k: np.ndarray, c: float, L: float) -> np.ndarray:
    d = (k[:, None] - k[None, :]) / c
    w = (2.0 / L) * (1.0 / c) / (1.0 + d * d)
    np.fill_diagonal(w, 0.0)
    J = -w
    J[np.diag_indices_from(J)] = 1.0 + w.sum(axis=1)
    return J


def solve_rapidities(N: int, c: float, L: float = 1.0, tol: float = 1e-14,
                     max_iter: int = 200) -> np.ndarray:
    if c <= 0:
        raise ValueError("repulsive coupling c > 0 required")
    I = quantum_numbers(N)
    k = (2.0 * math.pi / L) * I * (c / (c + 2.0 * N / L))
    for _ in range(max_iter):
        F = residual(k, c, L)
        if np.max(np.abs(F)) < tol * max(1.0, np.max(np.abs(k))):
            return k
        step = np.linalg.solve(jacobian(k, c, L), F)
        t = 1.0
        f0 = np.linalg.norm(F)
        while t > 1e-6:
            kn = k - t * step
            if np.linalg.norm(residual(kn, c, L)) < f0:
                break
            t *= 0.5
        k = kn
    F = residual(k, c, L)
    if np.max(np.abs(F)) > 1e-9 * max(1.0, np.max(np.abs(k))):
        raise RuntimeError("Bethe equations did not converge")
    return k


def ground_energy(N: int, c: float, L: float = 1.0) -> float:
    k = solve_rapidities(N, c, L)
    return 0.5 * float(np.sum(k * k))


def tonks_girardeau_energy(N: int, L: float = 1.0) -> float:
    """c -> infinity limit: k_j = 2 pi I_j / L, E = pi^2 N (N^2 - 1) / (6 L^2)."""
    return math.pi ** 2 * N * (N * N - 1) / (6.0 * L * L)


def two_body_energy_bisection(c: float, L: float = 1.0) -> float:
    """N = 2 by bisection: k_2 = -k_1 = k solves
    k = pi/L - (2/L) arctan(2k/c), k in (0, pi/L)."""
    f = lambda k: k - math.pi / L + (2.0 / L) * math.atan(2.0 * k / c)
    lo, hi = 0.0, math.pi / L
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    k = 0.5 * (lo + hi)
    return k * k
