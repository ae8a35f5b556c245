"""The seeded input generators: shapes, normalisation and the symmetries
the instances are documented to have, bit for bit (the energy gradient
skips the adjoint apply only for exactly Hermitian h and g)."""

import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("M", range(1, 9))
def test_random_instance_symmetries_are_exact(M):
    C, h, g = W.random_instance(4, M, 100 + M)
    assert C.shape == (W.fock_dim(4, M),) and abs(np.linalg.norm(C) - 1.0) < 1e-14
    assert np.array_equal(h, h.conj().T)
    assert np.array_equal(g, g.transpose(1, 0, 2, 3))          # k <-> s
    assert np.array_equal(g, g.transpose(0, 1, 3, 2))          # q <-> l
    assert np.array_equal(g, g.transpose(2, 3, 0, 1).conj())   # g_ksql = conj(g_qlks)
    assert np.array_equal(g, g.transpose(3, 2, 1, 0).conj())   # g_ksql = conj(g_lqsk): H = H^dagger
