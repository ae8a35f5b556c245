"""Pins for the oracle's time steps (CPU only).

The SIL step is checked against the matrix exponential it approximates and
against properties exp(-i H dt) has for Hermitian H: unitarity, energy
conservation (exact for the Krylov projection: <C'|H|C'> = y^H T y = alpha_0),
eigenvector phases, reversibility, and the single-particle case exp(-i h dt).
"""

import numpy as np
import pytest
from scipy.linalg import expm

import workloads as W
from oracle import dense
from oracle import propagate as pr


def apply_of(native, N, M, h, g):
    return lambda v: native.apply_h(N, M, h, g, v)


@pytest.mark.parametrize("N,M,seed", [(3, 3, 0), (2, 4, 1), (4, 2, 2), (1, 5, 3)])
def test_full_krylov_equals_expm(oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    H = dense.hamiltonian(N, M, h, g)
    for dt in (0.01, 0.3, 2.0):
        got, m, err = pr.sil_step(apply_of(oracle_native, N, M, h, g), C, dt, k=C.size)
        assert np.max(np.abs(got - pr.expm_step(H, C, dt))) <= 1e-12 * max(1.0, abs(dt) * np.linalg.norm(H, 2))


def test_single_particle_is_exp_of_h(oracle_native):
    # one boson: H = h on the M orbitals (no dense builder involved)
    M = 6
    _, h, g = W.random_instance(1, M, 4)
    C = W.random_coefficients(np.random.default_rng(5), M)
    got, _, _ = pr.sil_step(apply_of(oracle_native, 1, M, h, g), C, 0.7, k=M)
    assert np.allclose(got, expm(-0.7j * h) @ C, atol=1e-13)


@pytest.mark.parametrize("k", [4, 8, 12])
def test_unitary_and_energy_conserving(oracle_native, k):
    N, M = 6, 4
    C, h, g = W.random_instance(N, M, 6)
    ap = apply_of(oracle_native, N, M, h, g)
    got, m, err = pr.sil_step(ap, C, 0.05, k=k)
    assert m == k
    assert abs(np.linalg.norm(got) - np.linalg.norm(C)) <= 1e-13
    e0 = np.vdot(C, ap(C)).real
    e1 = np.vdot(got, ap(got)).real
    assert abs(e1 - e0) <= 1e-12 * max(1.0, abs(e0))


def test_eigenvector_gets_its_phase(oracle_native):
    N, M = 4, 3
    _, h, g = W.random_instance(N, M, 7)
    H = dense.hamiltonian(N, M, h, g)
    E, U = np.linalg.eigh(H)
    C = U[:, 1].astype(np.complex128)
    got, m, err = pr.sil_step(apply_of(oracle_native, N, M, h, g), C, 0.9, k=5)
    assert m == 1 and err == 0.0      # the Krylov space of an eigenvector is one-dimensional
    assert np.allclose(got, np.exp(-0.9j * E[1]) * C, atol=1e-12)


def test_error_estimate_tracks_the_true_error(oracle_native):
    N, M = 5, 4
    C, h, g = W.random_instance(N, M, 8)
    H = dense.hamiltonian(N, M, h, g)
    exact = pr.expm_step(H, C, 0.02)     # |H| dt ~ 0.7
    prev = np.inf
    for k in (3, 5, 7, 9, 11):
        got, m, est = pr.sil_step(apply_of(oracle_native, N, M, h, g), C, 0.02, k=k)
        actual = np.linalg.norm(got - exact)
        assert actual <= 10.0 * est + 1e-14
        assert actual <= prev            # more Krylov vectors, smaller error
        prev = actual
    assert prev < 1e-9


def test_step_reverses(oracle_native):
    N, M = 5, 3
    C, h, g = W.random_instance(N, M, 9)
    ap = apply_of(oracle_native, N, M, h, g)
    fwd, _, e1 = pr.sil_step(ap, C, 0.05, k=10)
    back, _, e2 = pr.sil_step(ap, fwd, -0.05, k=10)
    assert np.linalg.norm(back - C) <= 10 * (e1 + e2) + 1e-13


def test_tolerance_stops_early(oracle_native):
    N, M = 8, 4
    C, h, g = W.random_instance(N, M, 10)
    got, m, est = pr.sil_step(apply_of(oracle_native, N, M, h, g), C, 1e-3, k=40, tol=1e-12)
    assert m < 40 and est < 1e-12
