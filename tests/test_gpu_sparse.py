"""GPU H.C walking only nonzero constants (mc_apply_H_sparse) vs the oracle,
relative infinity-norm error <= 1e-12: the Lieb-Liniger interaction
(momentum conservation, Sec. VI), dense random g, and g with random holes."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-12


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N,M,maps", [(5, 5, True), (5, 5, False), (8, 7, True), (7, 3, False),
                                      (12, 7, False)])
def test_lieb_liniger_matches_oracle(mc, oracle_native, N, M, maps):
    h = W.lieb_liniger_h(M)
    g = W.lieb_liniger_g(M, c=20.0)
    C = W.random_coefficients(np.random.default_rng(N + M), oracle_native.dim(N, M))
    tab = mc.build_tables(N, M, form="reduced", double_jumps=maps)
    got = mc.apply_H_sparse(dev(h), dev(g), dev(C), tab).cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C)) <= TOL


def test_lieb_liniger_workload_sampled_rows(mc, oracle_native):
    """N = 20, M = 7 (dim 230,230), the Lanczos workload."""
    N, M = 20, 7
    h = W.lieb_liniger_h(M)
    g = W.lieb_liniger_g(M, c=20.0)
    C = W.random_coefficients(np.random.default_rng(3), oracle_native.dim(N, M))
    tab = mc.build_tables(N, M, form="reduced")
    got = mc.apply_H_sparse(dev(h), dev(g), dev(C), tab)
    dense_path = mc.apply_H(dev(h), dev(g), dev(C), tab)
    rows = np.unique(np.concatenate([np.random.default_rng(4).integers(0, C.size, 3000),
                                     np.arange(64), C.size - 1 - np.arange(64)]))
    ref = oracle_native.apply_h(N, M, h, g, C, rows)
    assert rel_inf(got[torch.from_numpy(rows).cuda()].cpu().numpy(), ref) <= TOL
    assert rel_inf(got.cpu().numpy(), dense_path.cpu().numpy()) <= TOL


@pytest.mark.parametrize("N,M,seed,holes", [(6, 4, 0, 0.0), (9, 5, 1, 0.0), (6, 4, 2, 0.8),
                                            (5, 6, 3, 0.9), (4, 8, 4, 0.95), (300, 2, 5, 0.5)])
def test_general_and_holed_g(mc, oracle_native, N, M, seed, holes):
    rng = np.random.default_rng(seed)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    g[rng.random(g.shape) < holes] = 0.0
    h[rng.random(h.shape) < holes] = 0.0
    C = W.random_coefficients(rng, oracle_native.dim(N, M))
    tab = mc.build_tables(N, M, form="reduced")
    got = mc.apply_H_sparse(dev(h), dev(g), dev(C), tab).cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C)) <= TOL


def test_sparse_needs_reduced_tables(mc):
    M = 3
    tab = mc.build_tables(4, M)    # paper form
    C = torch.ones(tab.dim, dtype=torch.complex128, device="cuda")
    with pytest.raises(mc.MCError):
        mc.apply_H_sparse(torch.zeros((M, M), dtype=torch.complex128, device="cuda"),
                          torch.zeros((M,) * 4, dtype=torch.complex128, device="cuda"), C, tab)
