"""GPU H.C in the case-split form (reduced tables) vs the oracle: relative
infinity-norm error <= 1e-12, with the reduced double-jump map and with
chained single jumps."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import ORDER_TOL, rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-12

# M = 1..8 (compile-time pair fold for M <= 5, pair loop for M >= 6), 16-bit
# occupations (N > 255), ragged last tiles, single-tile spaces
CASES = [(1, 1, 0), (3, 1, 1), (1, 4, 2), (2, 2, 3), (3, 5, 4), (10, 5, 0), (7, 4, 5), (5, 7, 6),
         (6, 8, 7), (12, 6, 8), (20, 3, 9), (300, 2, 12), (256, 3, 13), (40, 4, 14), (14, 8, 10),
         (20, 7, 11), (2, 3, 15)]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N,M,seed", CASES)
def test_split_apply_matches_oracle(mc, oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    ref = oracle_native.apply_h(N, M, h, g, C)
    tm = mc.build_tables(N, M, form="reduced")
    tc = mc.build_tables(N, M, form="reduced", double_jumps=False)
    assert tm.t2 is not None and tc.t2 is None
    a = mc.apply_H(dev(h), dev(g), dev(C), tm)
    b = mc.apply_H(dev(h), dev(g), dev(C), tc)
    assert rel_inf(a.cpu().numpy(), ref) <= TOL
    # both sources of the true double jumps give the same sums
    assert rel_inf(a.cpu().numpy(), b.cpu().numpy()) <= ORDER_TOL


@pytest.mark.parametrize("N,M", [(4, 3), (10, 5), (6, 6), (5, 8), (3, 2)])
def test_split_general_complex_inputs_and_adjoint(mc, oracle_native, N, M):
    """No symmetry of h or g; the adjoint is H with h -> h^dagger, g -> g^dagger."""
    rng = np.random.default_rng(N * 10 + M)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    D = oracle_native.dim(N, M)
    C = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    tab = mc.build_tables(N, M, form="reduced")
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab).cpu().numpy()
    assert rel_inf(hc, oracle_native.apply_h(N, M, h, g, C)) <= TOL
    hd = h.conj().T
    gd = np.transpose(g, (3, 2, 1, 0)).conj()
    adj = mc.apply_H_adjoint(dev(h), dev(g), dev(C), tab).cpu().numpy()
    assert rel_inf(adj, oracle_native.apply_h(N, M, hd, gd, C)) <= TOL


def test_split_agrees_with_paper_form(mc):
    N, M = 30, 5
    C, h, g = W.random_instance(N, M, 21)
    paper = mc.apply_H(dev(h), dev(g), dev(C), mc.build_tables(N, M))
    split = mc.apply_H(dev(h), dev(g), dev(C), mc.build_tables(N, M, form="reduced"))
    assert rel_inf(split.cpu().numpy(), paper.cpu().numpy()) <= TOL


@pytest.mark.parametrize("double_jumps", [True, False])
def test_split_large_space_sampled_rows(mc, oracle_native, double_jumps):
    """N = 200, M = 5 (dim 70,058,751), the throughput workload."""
    N, M = 200, 5
    C, h, g = W.random_instance(N, M, 2)
    tab = mc.build_tables(N, M, form="reduced", double_jumps=double_jumps)
    if double_jumps:
        # tiled size = entries of the reduced rows plus -1 padding
        assert tab.t2_required >= int(mc.tables_size(N, M).t2r_compact_entries)
    Cd = dev(C)
    hc = mc.apply_H(dev(h), dev(g), Cd, tab)
    rng = np.random.default_rng(3)
    D = C.size
    rows = np.unique(np.concatenate([rng.integers(0, D, 2000), np.arange(128), D - 1 - np.arange(128)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C, rows)) <= TOL
    e = mc.zdotc(Cd, hc).item()
    assert abs(e.imag) <= 1e-12 * abs(e.real)
    del tab, hc, Cd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N,M,seed", [(1, 1, 0), (2, 2, 1), (4, 3, 2), (6, 4, 3), (10, 5, 4), (5, 6, 5),
                                      (4, 7, 6), (3, 8, 7), (300, 2, 8), (40, 3, 9)])
def test_rho_on_reduced_tables_matches_oracle(mc, oracle_native, N, M, seed):
    C, _, _ = W.random_instance(N, M, seed)
    tab = mc.build_tables(N, M, form="reduced")
    Cd = dev(C)
    r2 = mc.rho2(Cd, tab).cpu().numpy()
    assert rel_inf(r2, oracle_native.rho2(N, M, C)) <= TOL
    r1 = mc.rho1(Cd, tab).cpu().numpy()
    assert rel_inf(r1, oracle_native.rho1(N, M, C)) <= TOL


def test_rho2_agrees_across_forms(mc):
    N, M = 30, 5
    C, _, _ = W.random_instance(N, M, 10)
    a = mc.rho2(dev(C), mc.build_tables(N, M)).cpu().numpy()
    b = mc.rho2(dev(C), mc.build_tables(N, M, form="reduced")).cpu().numpy()
    assert rel_inf(b, a) <= TOL


def test_rho2_without_a_map_chains_single_jumps(mc, oracle_native):
    """Tables without a double-jump map: rho2's targets m + e_q + e_l are two
    chained single jumps out of orbital 0 (Sec. IV)."""
    N, M = 6, 4
    tab = mc.build_tables(N, M, form="reduced", double_jumps=False)
    C, _, _ = W.random_instance(N, M, 5)
    r2 = mc.rho2(torch.from_numpy(C).cuda(), tab).cpu().numpy()
    assert rel_inf(r2, oracle_native.rho2(N, M, C)) <= TOL


def test_split_rejects_more_than_eight_orbitals(mc):
    N, M = 2, 9
    tab = mc.build_tables(N, M, form="reduced")
    C = torch.ones(tab.dim, dtype=torch.complex128, device="cuda")
    h = torch.zeros((M, M), dtype=torch.complex128, device="cuda")
    g = torch.zeros((M,) * 4, dtype=torch.complex128, device="cuda")
    with pytest.raises(mc.MCError):
        mc.apply_H(h, g, C, tab)


@pytest.mark.parametrize("form", ["reduced", "paper"])
def test_chained_64bit_gathers_sampled_rows(mc, oracle_native, form):
    """N = 300, M = 5: dim 348,881,876 > 2^28, so the coefficient gathers use
    64-bit addresses (chained, no double-jump map; 16-bit occupations)."""
    N, M = 300, 5
    rng = np.random.default_rng(31)
    D = oracle_native.dim(N, M)
    C = W.random_coefficients(rng, D)
    _, h, g = W.random_instance(1, M, 32)
    tab = mc.build_tables(N, M, form=form, double_jumps=False)
    hc = mc.apply_H(dev(h), dev(g), dev(C), tab)
    rows = np.unique(np.concatenate([rng.integers(0, D, 1500), np.arange(64), D - 1 - np.arange(64)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C, rows)) <= TOL
    del tab, hc
    torch.cuda.empty_cache()
