"""Seeded synthetic inputs for the bosonic Hamiltonian apply.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws and arranges random numbers (and builds the Lieb-Liniger coupling
tensors from their definition); it performs none of the method's arithmetic:
no hashing, no jump tables, no operator application.

Conventions (row-major, complex128):
  h[k, l]        one-body matrix elements  <phi_k|T|phi_l>
  g[k, s, q, l]  two-body matrix elements  <phi_k, phi_s|V|phi_q, phi_l>
  C[gamma]       Fock-basis coefficients, gamma in [0, dim)

Draw order for a seed is fixed: C first, then h, then g, all from one
``numpy.random.default_rng(seed)`` stream.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "fock_dim",
    "random_coefficients",
    "random_hermitian_h",
    "random_symmetric_g",
    "random_instance",
    "lieb_liniger_h",
    "lieb_liniger_g",
    "lieb_liniger_momenta",
    "batch_draws",
    "CONFIGS",
]


def fock_dim(N: int, M: int) -> int:
    """Number of ways to put N identical bosons in M orbitals, C(N+M-1, N).

    Used only to size the coefficient vector; it is the closed form of the
    paper's Eq. (nc), computed with Python's exact integer binomial.
    """
    if M <= 0 or N < 0:
        return 0
    return math.comb(N + M - 1, N)


def random_coefficients(rng: np.random.Generator, dim: int) -> np.ndarray:
    """Complex-normal coefficients (Re, Im iid N(0, 1/2)), normalised to 1.

    The paper draws a random coefficient vector and normalises it before
    timing the operators (Sec. III, density-matrix timings).
    """
    re = rng.standard_normal(dim)
    im = rng.standard_normal(dim)
    c = np.empty(dim, dtype=np.complex128)
    c.real = re
    c.imag = im
    c *= math.sqrt(0.5)
    c /= np.linalg.norm(c)
    return c


def random_hermitian_h(rng: np.random.Generator, M: int) -> np.ndarray:
    """h = (A + A^H)/2 with Re A, Im A iid N(0, 1)."""
    a = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    return np.ascontiguousarray((a + a.conj().T) / 2.0)


def random_symmetric_g(rng: np.random.Generator, M: int) -> np.ndarray:
    """Random two-body tensor with the symmetries of a physical interaction.

    A complex Gaussian tensor G is averaged over the order-8 group generated
    by  k<->s,  q<->l  and  (k,s,q,l) -> conj(q,l,k,s), so that
    g_ksql = g_skql = g_kslq = conj(g_qlks); with these the Hamiltonian is
    Hermitian.  The average is taken one generator at a time (three
    two-term means), so every symmetry holds bit for bit: a two-term sum is
    the same in either order, a four- or eight-term sum in another order
    need not be.
    """
    G = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    S = (G + G.transpose(1, 0, 2, 3)) / 2.0
    S = (S + S.transpose(0, 1, 3, 2)) / 2.0
    g = (S + S.transpose(2, 3, 0, 1).conj()) / 2.0
    return np.ascontiguousarray(g)


def random_instance(N: int, M: int, seed: int):
    """(C, h, g) drawn from one seeded stream in the fixed order C, h, g."""
    rng = np.random.default_rng(seed)
    C = random_coefficients(rng, fock_dim(N, M))
    h = random_hermitian_h(rng, M)
    g = random_symmetric_g(rng, M)
    return C, h, g


def lieb_liniger_momenta(M: int, L: float = 1.0) -> np.ndarray:
    """Plane-wave momenta 2*pi*n/L, n = -(M-1)/2 .. (M-1)/2 (M odd)."""
    if M % 2 != 1:
        raise ValueError("plane-wave window needs an odd number of orbitals")
    n = np.arange(M) - (M - 1) // 2
    return 2.0 * math.pi * n / L


def lieb_liniger_h(M: int, L: float = 1.0) -> np.ndarray:
    """Kinetic energy of plane waves, hbar = m = 1: h_kk = p_k^2 / 2."""
    p = lieb_liniger_momenta(M, L)
    return np.ascontiguousarray(np.diag(0.5 * p * p).astype(np.complex128))


def lieb_liniger_g(M: int, c: float, L: float = 1.0) -> np.ndarray:
    """Contact interaction c*delta(x - y) between plane waves on a ring.

    <phi_k phi_s| c delta |phi_q phi_l> = (c/L) * [n_k + n_s == n_q + n_l],
    i.e. momentum conservation (Sec. VI, plane-wave orbitals).
    """
    n = np.arange(M) - (M - 1) // 2
    tot_in = n[:, None] + n[None, :]
    mask = tot_in[:, :, None, None] == tot_in[None, None, :, :]
    return np.ascontiguousarray(np.where(mask, c / L, 0.0).astype(np.complex128))


def batch_draws(count: int, seed: int, n_range=(8, 40), m_range=(3, 8)):
    """(N, M) pairs for the batched workload: N ~ U{8..40}, M ~ U{3..8}."""
    rng = np.random.default_rng(seed)
    Ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    Ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(Ns, Ms)]


# Workloads named by what they are.  "small" is sized for exhaustive checks,
# "large" is the throughput workload.
CONFIGS = {
    "small_random": dict(N=10, M=5, seed=0),
    "lieb_liniger": dict(N=20, M=7, L=1.0, gammas=(0.1, 1.0, 10.0)),
    "large_random": dict(N=200, M=5, seed=2),
    "autograd": dict(N=50, M=6, seed=3),
    "batched": dict(count=64, seed=4, steps=50),
}
