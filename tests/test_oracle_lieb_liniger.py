"""Pins for the Bethe-ansatz solver and the oracle Lanczos (CPU only)."""

import math

import numpy as np
import pytest

import workloads as W
from oracle import bethe, dense
from oracle import combinatorics as cb
from oracle.lanczos import lanczos_ground, lanczos_recurrence


def test_tonks_girardeau_limit():
    for N in (2, 5, 20):
        assert abs(bethe.ground_energy(N, 1e9) / bethe.tonks_girardeau_energy(N) - 1) < 1e-6
    assert abs(bethe.tonks_girardeau_energy(20) - 13126.57) < 0.01


def test_weak_coupling_first_order():
    # E = c N (N-1) / (2L) + O(c^2)
    for N in (2, 5, 20):
        c = 1e-6
        assert abs(bethe.ground_energy(N, c) / (c * N * (N - 1) / 2) - 1) < 1e-3


def test_two_bosons_bisection():
    for c in (0.1, 1.0, 7.0, 100.0):
        assert abs(bethe.ground_energy(2, c) - bethe.two_body_energy_bisection(c)) < 1e-11


def test_energy_bounds_and_monotone():
    N = 5
    Es = [bethe.ground_energy(N, c) for c in (0.5, 2, 8, 32, 128)]
    assert all(a < b for a, b in zip(Es, Es[1:]))
    for c, E in zip((0.5, 2, 8, 32, 128), Es):
        assert 0 < E <= min(c * N * (N - 1) / 2, bethe.tonks_girardeau_energy(N)) + 1e-12


def test_lanczos_matches_dense_eigensolver(oracle_native):
    N, M = 4, 4
    _, h, g = W.random_instance(N, M, 8)
    H = dense.hamiltonian(N, M, h, g)
    v0 = W.random_coefficients(np.random.default_rng(1), H.shape[0])
    e0, *_ = lanczos_ground(lambda v: H @ v, v0, max_iter=H.shape[0])
    assert abs(e0 - np.linalg.eigvalsh(H)[0]) < 1e-10
    e0o, *_ = lanczos_ground(lambda v: oracle_native.apply_h(N, M, h, g, v), v0, max_iter=H.shape[0])
    assert abs(e0o - np.linalg.eigvalsh(H)[0]) < 1e-10


def test_recurrence_coefficients_dense(oracle_native):
    N, M = 5, 3
    _, h, g = W.random_instance(N, M, 9)
    H = dense.hamiltonian(N, M, h, g)
    v0 = W.random_coefficients(np.random.default_rng(2), H.shape[0])
    a1, b1 = lanczos_recurrence(lambda v: H @ v, v0, 8)
    a2, b2 = lanczos_recurrence(lambda v: oracle_native.apply_h(N, M, h, g, v), v0, 8)
    assert np.allclose(a1, a2, atol=1e-11) and np.allclose(b1, b2, atol=1e-11)


def test_lieb_liniger_single_orbital_is_mean_field(oracle_native):
    # one plane wave (k = 0): E = c N (N-1) / (2L), the first-order Bethe result
    N, c = 20, 3.0
    h = W.lieb_liniger_h(1)
    g = W.lieb_liniger_g(1, c)
    hc = oracle_native.apply_h(N, 1, h, g, np.array([1.0 + 0j]))
    assert abs(hc[0] - c * N * (N - 1) / 2) < 1e-10


@pytest.mark.slow
def test_lieb_liniger_converges_from_above(oracle_native):
    """Sec. VI: plane-wave truncations approach the Bethe-ansatz energy from
    above as the number of orbitals grows (N = 5 as in Fig. LiebComparison)."""
    N, L = 5, 1.0
    for c in (1.0, 10.0):
        E_ba = bethe.ground_energy(N, c, L)
        prev = math.inf
        for M in (3, 5, 7, 9):
            h = W.lieb_liniger_h(M, L)
            g = W.lieb_liniger_g(M, c, L)
            D = cb.dim(N, M)
            v0 = W.random_coefficients(np.random.default_rng(M), D)
            e0, *_ = lanczos_ground(lambda v: oracle_native.apply_h(N, M, h, g, v), v0,
                                    max_iter=min(D, 200))
            assert e0 >= E_ba - 1e-9
            assert e0 <= prev + 1e-9
            prev = e0
        # with 9 plane waves the weak-coupling case is already close
        if c == 1.0:
            assert prev - E_ba < 0.02 * E_ba


def test_workload_symmetries():
    for M in (2, 3, 5):
        _, h, g = W.random_instance(4, M, M)
        assert np.allclose(h, h.conj().T)
        assert np.allclose(g, g.transpose(1, 0, 2, 3))
        assert np.allclose(g, g.transpose(0, 1, 3, 2))
        assert np.allclose(g, g.transpose(2, 3, 0, 1).conj())
    C, _, _ = W.random_instance(10, 5, 0)
    assert abs(np.linalg.norm(C) - 1) < 1e-14
    C2, _, _ = W.random_instance(10, 5, 0)
    assert np.array_equal(C, C2)
    g = W.lieb_liniger_g(7, 20.0)
    assert np.count_nonzero(g) == 231
