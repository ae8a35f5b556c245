"""GPU density matrices vs the oracle (relative infinity-norm <= 1e-12),
invariants, and bitwise reproducibility of the fixed-order reductions."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-12


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N,M,seed", [(1, 3, 0), (2, 2, 1), (3, 5, 2), (10, 5, 0), (7, 4, 3),
                                      (5, 7, 4), (6, 8, 5), (300, 2, 6), (3, 10, 7)])
def test_rho_match_oracle(mc, oracle_native, N, M, seed):
    C, _, _ = W.random_instance(N, M, seed)
    tab = mc.build_tables(N, M)
    Cd = dev(C)
    r1 = mc.rho1(Cd, tab).cpu().numpy()
    assert rel_inf(r1, oracle_native.rho1(N, M, C)) <= TOL
    if M <= 8:
        r2 = mc.rho2(Cd, tab).cpu().numpy()
        assert rel_inf(r2, oracle_native.rho2(N, M, C)) <= TOL
    else:
        with pytest.raises(mc.MCError):
            mc.rho2(Cd, tab)


def test_rho_reproducible_and_consistent_with_energy(mc):
    N, M = 10, 5
    C, h, g = W.random_instance(N, M, 0)
    tab = mc.build_tables(N, M)
    Cd = dev(C)
    r1a, r1b = mc.rho1(Cd, tab), mc.rho1(Cd, tab)
    r2a, r2b = mc.rho2(Cd, tab), mc.rho2(Cd, tab)
    assert torch.equal(r1a, r1b) and torch.equal(r2a, r2b)
    HC = mc.apply_H(dev(h), dev(g), Cd, tab)
    E = mc.zdotc(Cd, HC).item()
    E2 = (torch.sum(dev(h) * r1a) + 0.5 * torch.sum(dev(g) * r2a)).item()
    assert abs(E - E2) <= 1e-12 * abs(E)


def test_autograd_size_sampled_elements(mc, oracle_native):
    """N = 50, M = 6 (dim 3,478,761): full rho1, sampled rho2 elements."""
    N, M = 50, 6
    C, _, _ = W.random_instance(N, M, 3)
    tab = mc.build_tables(N, M)
    Cd = dev(C)
    r1 = mc.rho1(Cd, tab).cpu().numpy()
    r2 = mc.rho2(Cd, tab).cpu().numpy()
    assert abs(np.trace(r1) - N) <= 1e-12 * N
    assert np.allclose(np.einsum("kssl->kl", r2), (N - 1) * r1, rtol=0, atol=1e-10)
    assert rel_inf(r1, oracle_native.rho1(N, M, C)) <= TOL
    rng = np.random.default_rng(4)
    idx = np.unique(np.concatenate([rng.integers(0, M ** 4, 12), [0, M ** 4 - 1]]))
    ref = oracle_native.rho2_elements(N, M, C, idx)
    assert np.max(np.abs(r2.reshape(-1)[idx] - ref)) <= TOL * np.max(np.abs(r2))
    del tab
    torch.cuda.empty_cache()


def test_zdotc(mc):
    rng = np.random.default_rng(8)
    for n in (1, 63, 1000, 1 << 20):
        x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        got = mc.zdotc(dev(x), dev(y)).item()
        ref = np.vdot(x, y)
        assert abs(got - ref) <= 1e-13 * np.sum(np.abs(x) * np.abs(y))
