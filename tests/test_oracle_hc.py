"""Pins for the oracle's H.C (CPU only): brute force, Hermiticity, closed forms."""

import numpy as np
import pytest

import workloads as W
from oracle import combinatorics as cb
from oracle import dense


@pytest.mark.parametrize("N,M,seed", [(1, 4, 1), (2, 3, 2), (3, 3, 3), (4, 2, 4), (5, 3, 5), (3, 5, 6), (10, 5, 0)])
def test_matches_dense_brute_force(oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    H = dense.hamiltonian(N, M, h, g)
    assert np.allclose(H, H.conj().T, atol=1e-12)
    hc = oracle_native.apply_h(N, M, h, g, C)
    ref = H @ C
    assert np.max(np.abs(hc - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_dense_brute_force_general_nonhermitian(oracle_native):
    # arbitrary complex h, g (no symmetry) still agree: the oracle must not
    # rely on any symmetry of the inputs
    N, M = 3, 3
    rng = np.random.default_rng(11)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    C = rng.standard_normal(cb.dim(N, M)) + 1j * rng.standard_normal(cb.dim(N, M))
    H = dense.hamiltonian(N, M, h, g)
    assert np.allclose(oracle_native.apply_h(N, M, h, g, C), H @ C, rtol=0, atol=1e-12)


def test_number_operator_restriction():
    assert np.allclose(dense.number_operator_check(4, 3), 4 * np.eye(cb.dim(4, 3)))


@pytest.mark.parametrize("N,M", [(10, 5), (20, 4), (6, 7)])
def test_hermiticity(oracle_native, N, M):
    rng = np.random.default_rng(N * 31 + M)
    _, h, g = W.random_instance(1, M, N)
    D = cb.dim(N, M)
    C = W.random_coefficients(rng, D)
    E = W.random_coefficients(rng, D)
    HC = oracle_native.apply_h(N, M, h, g, C)
    HE = oracle_native.apply_h(N, M, h, g, E)
    lhs = np.vdot(E, HC)
    rhs = np.conj(np.vdot(C, HE))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_identity_one_body(oracle_native):
    N, M = 9, 4
    C, _, _ = W.random_instance(N, M, 1)
    hc = oracle_native.apply_h(N, M, np.eye(M), np.zeros((M,) * 4), C)
    assert np.allclose(hc, N * C, rtol=0, atol=1e-13)


def test_pair_counting_two_body(oracle_native):
    # g_ksql = (d_kl d_sq + d_kq d_sl)/2 makes the interaction term
    # (1/2) * N(N-1): the factor 1/2 of the paper's interaction operator
    N, M = 8, 4
    C, _, _ = W.random_instance(N, M, 2)
    d = np.eye(M)
    g = 0.5 * (np.einsum("kl,sq->ksql", d, d) + np.einsum("kq,sl->ksql", d, d))
    hc = oracle_native.apply_h(N, M, np.zeros((M, M)), g, C)
    assert np.allclose(hc, 0.5 * N * (N - 1) * C, rtol=0, atol=1e-12)


def test_single_particle_is_matrix_vector(oracle_native):
    M = 6
    C, h, g = W.random_instance(1, M, 3)
    hc = oracle_native.apply_h(1, M, h, g, C)
    assert np.allclose(hc, h @ C, rtol=0, atol=1e-14)
    rng = np.random.default_rng(0)
    hn = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    assert np.allclose(oracle_native.apply_h(1, M, hn, g, C), hn @ C, rtol=0, atol=1e-14)


def test_single_orbital(oracle_native):
    N = 37
    h = np.array([[1.25 - 0.5j]])
    g = np.array([0.75 + 0.25j]).reshape(1, 1, 1, 1)
    C = np.array([0.6 + 0.8j])
    hc = oracle_native.apply_h(N, 1, h, g, C)
    assert np.allclose(hc, (N * h[0, 0] + 0.5 * N * (N - 1) * g[0, 0, 0, 0]) * C, rtol=1e-15)


def test_noninteracting_spectrum(oracle_native):
    N, M = 3, 4
    _, h, _ = W.random_instance(N, M, 4)
    D = cb.dim(N, M)
    g = np.zeros((M,) * 4)
    H = np.stack([oracle_native.apply_h(N, M, h, g, np.eye(D)[j]) for j in range(D)], axis=1)
    eps = np.linalg.eigvalsh(h)
    expect = sorted(sum(n * e for n, e in zip(c, eps)) for c in cb.compositions(N, M))
    assert np.allclose(np.linalg.eigvalsh(H), expect, atol=1e-12)


def test_sampled_rows_equal_full(oracle_native):
    N, M = 10, 5
    C, h, g = W.random_instance(N, M, 0)
    full = oracle_native.apply_h(N, M, h, g, C)
    rows = np.array([999, 0, 5, 1000, 77], dtype=np.int64)
    assert np.array_equal(oracle_native.apply_h(N, M, h, g, C, rows), full[rows])
