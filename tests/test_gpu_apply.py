"""GPU H.C vs the oracle: relative infinity-norm error <= 1e-12."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = [(1, 1, 0), (3, 1, 1), (1, 4, 2), (2, 2, 3), (3, 5, 4), (10, 5, 0), (7, 4, 5), (5, 7, 6),
         (6, 8, 7), (12, 6, 8), (20, 3, 9), (2, 9, 10), (3, 10, 11), (300, 2, 12), (256, 3, 13),
         (40, 4, 14)]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N,M,seed", CASES)
def test_apply_matches_oracle(mc, oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    tab = mc.build_tables(N, M)
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab).cpu().numpy()
    ref = oracle_native.apply_h(N, M, h, g, C)
    assert rel_inf(hc, ref) <= TOL


@pytest.mark.parametrize("N,M", [(4, 3), (10, 5), (5, 9)])
def test_apply_general_complex_inputs(mc, oracle_native, N, M):
    """No symmetry of h or g is assumed."""
    rng = np.random.default_rng(N + M)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    D = oracle_native.dim(N, M)
    C = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    tab = mc.build_tables(N, M)
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab).cpu().numpy()
    assert rel_inf(hc, oracle_native.apply_h(N, M, h, g, C)) <= TOL


def test_apply_hermiticity_and_repeatability(mc):
    N, M = 10, 5
    C, h, g = W.random_instance(N, M, 0)
    E = W.random_coefficients(np.random.default_rng(99), C.size)
    tab = mc.build_tables(N, M)
    HC = mc.apply_H(dev(h), dev(g), dev(C), tab)
    HE = mc.apply_H(dev(h), dev(g), dev(E), tab)
    lhs = np.vdot(E, HC.cpu().numpy())
    rhs = np.conj(np.vdot(C, HE.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    HC2 = mc.apply_H(dev(h), dev(g), dev(C), tab)
    assert torch.equal(HC, HC2)


def test_apply_rejects_aliasing_and_bad_shapes(mc):
    N, M = 4, 3
    C, h, g = W.random_instance(N, M, 1)
    tab = mc.build_tables(N, M)
    c = dev(C)
    with pytest.raises(mc.MCError):
        mc.apply_H(dev(h), dev(g), c, tab, out=c)
    with pytest.raises(ValueError):
        mc.apply_H(dev(h), dev(g), c[:-1].contiguous(), tab)


def test_lieb_liniger_sampled_rows(mc, oracle_native):
    """Plane waves k = -3..3 (M = 7), N = 20 (dim 230,230), gamma = 1."""
    N, M, L = 20, 7, 1.0
    h = W.lieb_liniger_h(M, L)
    g = W.lieb_liniger_g(M, c=20.0, L=L)
    C = W.random_coefficients(np.random.default_rng(1), oracle_native.dim(N, M))
    tab = mc.build_tables(N, M)
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab).cpu().numpy()
    rows = np.unique(np.concatenate([np.random.default_rng(2).integers(0, C.size, 3000),
                                     np.arange(100), C.size - 1 - np.arange(100)]))
    ref = oracle_native.apply_h(N, M, h, g, C, rows)
    assert rel_inf(hc[rows], ref) <= TOL


def test_large_space_sampled_rows(mc, oracle_native):
    """N = 200, M = 5 (dim 70,058,751), the throughput workload."""
    N, M = 200, 5
    C, h, g = W.random_instance(N, M, 2)
    tab = mc.build_tables(N, M)
    Cd = dev(C)
    hc = mc.apply_H(dev(h), dev(g), Cd, tab)
    rng = np.random.default_rng(3)
    D = C.size
    rows = np.unique(np.concatenate([rng.integers(0, D, 2000), np.arange(128), D - 1 - np.arange(128)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    ref = oracle_native.apply_h(N, M, h, g, C, rows)
    assert rel_inf(got, ref) <= TOL
    # whole-vector property: <C|HC> is real for Hermitian H
    e = mc.zdotc(Cd, hc).item()
    assert abs(e.imag) <= 1e-12 * abs(e.real)
    del tab, hc, Cd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N,M,seed", [(1, 3, 0), (2, 2, 1), (3, 5, 4), (10, 5, 0), (7, 4, 5), (5, 7, 6),
                                      (6, 8, 7), (300, 2, 12), (40, 4, 14), (12, 6, 8), (14, 8, 10),
                                      (20, 7, 11)])
def test_apply_chained_single_jumps_matches_oracle(mc, oracle_native, N, M, seed):
    """Without the double-jump map the apply chains two single jumps."""
    C, h, g = W.random_instance(N, M, seed)
    tab = mc.build_tables(N, M, double_jumps=False)
    assert tab.t2 is None
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab).cpu().numpy()
    assert rel_inf(hc, oracle_native.apply_h(N, M, h, g, C)) <= TOL


def test_apply_chained_large_space_sampled_rows(mc, oracle_native):
    N, M = 200, 5
    C, h, g = W.random_instance(N, M, 2)
    tab = mc.build_tables(N, M, double_jumps=False)
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([rng.integers(0, C.size, 1000), np.arange(64), C.size - 1 - np.arange(64)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C, rows)) <= TOL
    del tab, hc
    torch.cuda.empty_cache()
