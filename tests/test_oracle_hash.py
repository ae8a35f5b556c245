"""Pins for the oracle's dimension and its configuration <-> index maps
(the maps of Algorithms 1 and 2; CPU only)."""

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import combinatorics as cb
from tests.conftest import golden


def hockey_stick_index(occ):
    """Independent closed form of Eq. (TotalCost): the particles of orbital m
    are removed while the basket holds S_m, S_m - 1, ..., S_{m-1} + 1 particles
    (S_m = n_0 + ... + n_m), and sum_{s=a+1}^{b} C(s+m-1, m-1) =
    C(b+m, m) - C(a+m, m)."""
    S = np.cumsum(occ)
    return sum(math.comb(int(S[m]) + m, m) - math.comb(int(S[m - 1]) + m, m)
               for m in range(1, len(occ)))


def order_rank(occ):
    """Position of a configuration in the order the algorithms define
    (orbital M-1 most significant): the number of configurations that come
    before it, counted block by block -- for each orbital m from M-1 down,
    the configurations that agree above m and hold fewer particles in m."""
    left = sum(occ)
    rank = 0
    for m in range(len(occ) - 1, 0, -1):
        rank += sum(cb.nc(left - t, m) for t in range(occ[m]))
        left -= occ[m]
    return rank


def test_worked_example_fig_scheme2(oracle_native):
    ex = golden("hash_worked_example.json")
    N, M, occ = ex["N"], ex["M"], ex["occupation"]
    terms = [cb.nc(n, m) for n, m in ex["cost_terms"]]
    assert sum(terms) == ex["index"]
    assert cb.index_of(occ) == ex["index"]
    assert oracle_native.hash_occ(occ, N) == ex["index"]
    assert cb.config_of(ex["index"], N, M) == occ
    assert list(oracle_native.unhash(ex["index"], N, M)) == occ
    # Eq. (TotalCost) with sorted particle positions: orbital 1 once, orbital 3 twice
    assert cb.total_cost([1, 3, 3], M) == ex["index"]


@pytest.mark.parametrize("N,M,D", [(10, 5, 1001), (20, 7, 230230), (200, 5, 70058751),
                                   (50, 6, 3478761), (1000, 3, 501501), (5, 25, 118755)])
def test_dimension_closed_form(oracle_native, N, M, D):
    assert cb.dim(N, M) == D
    assert oracle_native.dim(N, M) == D
    assert D == math.comb(N + M - 1, N)


def test_dimension_edge_cases(oracle_native):
    for n in range(6):
        assert cb.nc(n, 0) == 0 and oracle_native.nc(n, 0) == 0
    for m in range(1, 7):
        assert cb.nc(0, m) == 1 and oracle_native.nc(0, m) == 1
    for n in range(8):
        assert cb.nc(n, 1) == 1 and cb.nc(n, 2) == n + 1


def test_hand_derived_order_two_particles_three_orbitals():
    # orbital M-1 most significant: sorted by (n2, n1) with n0 the remainder
    expected = [[2, 0, 0], [1, 1, 0], [0, 2, 0], [1, 0, 1], [0, 1, 1], [0, 0, 2]]
    assert [cb.config_of(i, 2, 3) for i in range(6)] == expected
    assert [cb.index_of(o) for o in expected] == list(range(6))


def test_single_particle_maps_to_its_orbital(oracle_native):
    for M in range(1, 9):
        for j in range(M):
            e = [0] * M
            e[j] = 1
            assert cb.index_of(e) == j
            assert oracle_native.hash_occ(e, 1) == j


@pytest.mark.parametrize("N,M", [(1, 1), (3, 1), (0, 4), (1, 6), (3, 5), (4, 4), (6, 3), (7, 4), (10, 5), (5, 7)])
def test_bijection_full_enumeration(oracle_native, N, M):
    if N == 0:
        pytest.skip("Algorithms 1 and 2 require N > 0")
    D = cb.dim(N, M)
    configs = list(cb.compositions(N, M))
    assert len(configs) == D
    idx = [cb.index_of(c) for c in configs]
    assert sorted(idx) == list(range(D))
    # brute force: the index is the position in the order that compares
    # n_{M-1} first, then n_{M-2}, ..., n_1
    ordered = sorted(configs, key=lambda c: tuple(reversed(c[1:])))
    assert [cb.index_of(c) for c in ordered] == list(range(D))
    for c, i in zip(configs, idx):
        assert cb.config_of(i, N, M) == c
    occ = np.array(configs, dtype=np.int32)
    assert np.array_equal(oracle_native.hash_rows(occ, N), np.array(idx))
    assert np.array_equal(oracle_native.occ_rows(N, M, np.array(idx)), occ)


@pytest.mark.parametrize("N,M", [(3, 5), (7, 4), (6, 6), (12, 3)])
def test_index_equals_closed_form_and_block_count(N, M):
    for c in cb.compositions(N, M):
        i = cb.index_of(c)
        assert hockey_stick_index(c) == i
        assert order_rank(c) == i


def test_extreme_indices(oracle_native):
    for N, M in [(10, 5), (200, 5), (50, 6)]:
        D = cb.dim(N, M)
        assert list(oracle_native.unhash(0, N, M)) == [N] + [0] * (M - 1)
        assert list(oracle_native.unhash(D - 1, N, M)) == [0] * (M - 1) + [N]
        with pytest.raises(ValueError):
            oracle_native.unhash(D, N, M)
        with pytest.raises(ValueError):
            oracle_native.unhash(-1, N, M)


def test_large_space_sampled_roundtrip(oracle_native):
    N, M = 200, 5
    D = cb.dim(N, M)
    rng = np.random.default_rng(7)
    rows = np.concatenate([rng.integers(0, D, 3000), [0, 1, D - 2, D - 1]]).astype(np.int64)
    occ = oracle_native.occ_rows(N, M, rows)
    assert np.all(occ.sum(axis=1) == N) and np.all(occ >= 0)
    assert np.array_equal(oracle_native.hash_rows(occ, N), rows)
    for o, r in zip(occ[:200], rows[:200]):
        assert hockey_stick_index(o) == r


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 12), st.integers(1, 6), st.data())
def test_roundtrip_property(N, M, data):
    cuts = sorted(data.draw(st.lists(st.integers(0, N), min_size=M - 1, max_size=M - 1)))
    bounds = [0] + cuts + [N]
    occ = [bounds[i + 1] - bounds[i] for i in range(M)]
    i = cb.index_of(occ)
    assert 0 <= i < cb.dim(N, M)
    assert cb.config_of(i, N, M) == occ
    assert hockey_stick_index(occ) == i
