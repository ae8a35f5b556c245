"""GPU H.C with no table (mc_apply_H_direct: occupations and jump targets of
each row from its index in closed form) vs the oracle, relative
infinity-norm error <= 1e-12, and against the case-split apply on reduced
tables, which sums the same terms (in another grouping on tiles that do not
take the class-major stream)."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import ORDER_TOL, rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-12

# M = 1..8, single-tile spaces, ragged last tiles, N > 255, N = 1
CASES = [(1, 1, 0), (3, 1, 1), (1, 4, 2), (2, 2, 3), (3, 5, 4), (10, 5, 0), (7, 4, 5), (5, 7, 6),
         (6, 8, 7), (12, 6, 8), (20, 3, 9), (300, 2, 12), (256, 3, 13), (40, 4, 14), (14, 8, 10),
         (20, 7, 11), (2, 3, 15), (1, 8, 16), (63, 2, 17), (64, 2, 18)]


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N,M,seed", CASES)
def test_direct_matches_oracle_and_split(mc, oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    got = mc.apply_H_direct(dev(h), dev(g), dev(C), N, M)
    assert rel_inf(got.cpu().numpy(), oracle_native.apply_h(N, M, h, g, C)) <= TOL
    split = mc.apply_H(dev(h), dev(g), dev(C), mc.build_tables(N, M, form="reduced",
                                                               double_jumps=False))
    assert rel_inf(got.cpu().numpy(), split.cpu().numpy()) <= ORDER_TOL


@pytest.mark.parametrize("N,M", [(4, 3), (10, 5), (6, 6), (5, 8), (3, 2), (9, 7)])
def test_direct_general_complex_inputs(mc, oracle_native, N, M):
    """No symmetry of h or g, C not normalised."""
    rng = np.random.default_rng(N * 10 + M)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    D = oracle_native.dim(N, M)
    C = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    got = mc.apply_H_direct(dev(h), dev(g), dev(C), N, M).cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C)) <= TOL


def test_direct_lieb_liniger_workload(mc, oracle_native):
    """N = 20, M = 7 (dim 230,230), the plane-wave Lieb-Liniger Hamiltonian."""
    N, M = 20, 7
    h = W.lieb_liniger_h(M)
    g = W.lieb_liniger_g(M, c=20.0)
    C = W.random_coefficients(np.random.default_rng(3), oracle_native.dim(N, M))
    got = mc.apply_H_direct(dev(h), dev(g), dev(C), N, M)
    rows = np.unique(np.concatenate([np.random.default_rng(4).integers(0, C.size, 3000),
                                     np.arange(64), C.size - 1 - np.arange(64)]))
    ref = oracle_native.apply_h(N, M, h, g, C, rows)
    assert rel_inf(got[torch.from_numpy(rows).cuda()].cpu().numpy(), ref) <= TOL


def test_direct_large_space_sampled_rows(mc, oracle_native):
    """N = 200, M = 5 (dim 70,058,751), the throughput workload, in the launch
    configuration the benchmark times; equal to the reduced-map apply."""
    N, M = 200, 5
    C, h, g = W.random_instance(N, M, 2)
    Cd = dev(C)
    hc = mc.apply_H_direct(dev(h), dev(g), Cd, N, M)
    rng = np.random.default_rng(3)
    D = C.size
    rows = np.unique(np.concatenate([rng.integers(0, D, 2000), np.arange(128), D - 1 - np.arange(128)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C, rows)) <= TOL
    tab = mc.build_tables(N, M, form="reduced")
    ref = mc.apply_H(dev(h), dev(g), Cd, tab)
    assert rel_inf(hc.cpu().numpy(), ref.cpu().numpy()) <= ORDER_TOL
    del tab, ref, hc, Cd
    torch.cuda.empty_cache()


def test_direct_64bit_gathers_sampled_rows(mc, oracle_native):
    """N = 300, M = 5: dim 348,881,876 > 2^28, 64-bit coefficient gathers."""
    N, M = 300, 5
    rng = np.random.default_rng(31)
    D = oracle_native.dim(N, M)
    C = W.random_coefficients(rng, D)
    _, h, g = W.random_instance(1, M, 32)
    hc = mc.apply_H_direct(dev(h), dev(g), dev(C), N, M)
    rows = np.unique(np.concatenate([rng.integers(0, D, 1500), np.arange(64), D - 1 - np.arange(64)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C, rows)) <= TOL
    del hc
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N,M", [(65535, 2), (9000, 3), (600, 4)])
def test_direct_large_N_few_orbitals(mc, oracle_native, N, M):
    """N up to MC_MAX_N at few orbitals (no square-root table in LDS below
    M = 6, so N is bounded only by D < 2^31); sampled rows vs the oracle."""
    rng = np.random.default_rng(N + M)
    D = oracle_native.dim(N, M)
    C = W.random_coefficients(rng, D)
    _, h, g = W.random_instance(1, M, 60 + M)
    hc = mc.apply_H_direct(dev(h), dev(g), dev(C), N, M)
    rows = np.unique(np.concatenate([rng.integers(0, D, 300), np.arange(64), D - 1 - np.arange(64)]))
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, oracle_native.apply_h(N, M, h, g, C, rows)) <= TOL


def test_direct_rejects_bad_sizes(mc):
    z = lambda *s: torch.zeros(s, dtype=torch.complex128, device="cuda")
    with pytest.raises(mc.MCError):            # M > 8
        mc.apply_H_direct(z(9, 9), z(9, 9, 9, 9), z(mc.dim(1, 9)), 1, 9)
    C = z(mc.dim(4, 3))
    with pytest.raises(mc.MCError):            # output aliases the input
        mc.apply_H_direct(z(3, 3), z(3, 3, 3, 3), C, 4, 3, out=C)


@pytest.mark.parametrize("N,M,seed,k", [(10, 5, 0, 12), (6, 8, 7, 6), (20, 3, 6, 8)])
def test_direct_sil_step_matches_oracle(mc, oracle_native, N, M, seed, k):
    """A SIL step on a table-free space (DirectSpace): same result as on
    reduced tables, and the oracle's SIL step within 1e-11 (k Krylov steps
    at the 1e-12 apply bar)."""
    from oracle import propagate as pr
    C, h, g = W.random_instance(N, M, seed)
    ref, m_ref, _ = pr.sil_step(lambda v: oracle_native.apply_h(N, M, h, g, v), C, 0.02, k=k)
    got, m, _ = mc.sil_step(mc.DirectSpace(N, M), dev(h), dev(g), dev(C), 0.02, k=k)
    tab, m2, _ = mc.sil_step(mc.build_tables(N, M, form="reduced"), dev(h), dev(g), dev(C), 0.02, k=k)
    assert m == m_ref == m2
    assert rel_inf(got.cpu().numpy(), ref) <= 1e-11
    assert rel_inf(got.cpu().numpy(), tab.cpu().numpy()) <= 1e-12


def test_direct_lanczos_lieb_liniger_energies(mc):
    """Lanczos ground states of the plane-wave Lieb-Liniger ring on table-free
    spaces equal the oracle's stored energies (N = 20, M up to 7)."""
    import json
    import os
    from paper_2005_13679_amd import lanczos
    from tests.conftest import ROOT
    ref = json.load(open(os.path.join(ROOT, "tests", "golden", "ll_energies.json")))
    N, L = ref["N"], ref["L"]
    for r in ref["runs"]:
        M = r["M"]
        h, g = W.lieb_liniger_h(M, L), W.lieb_liniger_g(M, r["c"], L)
        sp = mc.DirectSpace(N, M)
        v0 = W.random_coefficients(np.random.default_rng(1000 + M), sp.dim)
        e, *_ = lanczos.ground_state(h, g, sp, dev(v0), max_iter=400, tol=1e-13)
        assert abs(e - r["E0"]) <= 1e-9 * abs(r["E0"]), (r, e)


@pytest.mark.timeout(600)
def test_direct_maximum_dimension(mc, oracle_native):
    """N = 473, M = 5: dim 2,130,031,575, the largest below 2^31 (the tables
    would need 213 GB for the single-jump map alone).  C is a closed-form
    function of the index, made on the device and copied to the host for the
    oracle; sampled rows against the oracle, the extreme rows included, and
    Hermiticity <D|HC> = conj<C|HD> over the whole space."""
    N, M = 473, 5
    D = oracle_native.dim(N, M)
    assert D == 2130031575 and D < 2 ** 31
    _, h, g = W.random_instance(1, M, 41)              # Hermitian h, symmetric g
    k = torch.arange(D, dtype=torch.float64, device="cuda")
    Cd = torch.complex(torch.cos(0.3718 * k), torch.sin(0.9127 * k + 0.25))
    del k
    C = Cd.cpu().numpy()
    hd, gd = dev(h), dev(g)
    hc = mc.apply_H_direct(hd, gd, Cd, N, M)
    rng = np.random.default_rng(43)
    rows = np.unique(np.concatenate([rng.integers(0, D, 600), np.arange(64), D - 1 - np.arange(64)]))
    ref = oracle_native.apply_h(N, M, h, g, C, rows)
    got = hc[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert rel_inf(got, ref) <= TOL
    del C
    # Hermiticity with a second vector made on the device
    k = torch.arange(D, dtype=torch.float64, device="cuda")
    Dv = torch.complex(torch.sin(0.113 * k), torch.cos(0.271 * k))
    del k
    hd_v = mc.apply_H_direct(hd, gd, Dv, N, M)
    lhs = mc.zdotc(Dv, hc).item()
    rhs = mc.zdotc(Cd, hd_v).item()
    bound = (mc.zdotc(Dv, Dv).item().real * mc.zdotc(hc, hc).item().real) ** 0.5
    assert abs(lhs - rhs.conjugate()) <= 1e-11 * bound
    del Cd, hc, Dv, hd_v
    torch.cuda.empty_cache()


@pytest.mark.parametrize("N,M,seed", [(1, 1, 0), (3, 1, 1), (1, 4, 2), (2, 2, 3), (10, 5, 0),
                                      (7, 4, 5), (5, 7, 6), (6, 8, 7), (12, 6, 8), (300, 2, 12),
                                      (40, 3, 9), (2, 3, 15)])
def test_direct_density_matrices_match_oracle(mc, oracle_native, N, M, seed):
    C, h, g = W.random_instance(N, M, seed)
    sp = mc.DirectSpace(N, M)
    r1 = mc.rho1(dev(C), sp).cpu().numpy()
    r2 = mc.rho2(dev(C), sp).cpu().numpy()
    assert rel_inf(r1, oracle_native.rho1(N, M, C)) <= TOL
    assert rel_inf(r2, oracle_native.rho2(N, M, C)) <= TOL


def test_direct_density_matrices_match_tables(mc):
    """N = 30, M = 6 (dim 324,632): table-free rho1, rho2 against the
    table-driven kernels (different summation order, same sums)."""
    N, M = 30, 6
    C, _, _ = W.random_instance(N, M, 19)
    sp, tab = mc.DirectSpace(N, M), mc.build_tables(N, M)
    for f in (mc.rho1, mc.rho2):
        assert rel_inf(f(dev(C), sp).cpu().numpy(), f(dev(C), tab).cpu().numpy()) <= TOL


def test_direct_energy_gradients(mc):
    """E = <C|HC> on a table-free space: value and every gradient (C, h, g)
    against the reduced-table run, with Hermitian inputs and with
    non-Hermitian ones (the C-gradient then takes the table-free adjoint)."""
    N, M = 12, 5
    C, h, g = W.random_instance(N, M, 71)
    out = []
    for space in (mc.DirectSpace(N, M), mc.build_tables(N, M, form="reduced")):
        Ct, ht, gt = (dev(x).requires_grad_(True) for x in (C, h, g))
        E = mc.energy(Ct, ht, gt, space)
        E.real.backward()
        out.append((E.detach(), Ct.grad, ht.grad, gt.grad))
    assert abs(out[0][0].item() - out[1][0].item()) <= ORDER_TOL * abs(out[1][0].item())
    assert rel_inf(out[0][1].cpu().numpy(), out[1][1].cpu().numpy()) <= ORDER_TOL
    for i in (2, 3):
        assert rel_inf(out[0][i].cpu().numpy(), out[1][i].cpu().numpy()) <= TOL
    rng = np.random.default_rng(72)
    hn = h + 0.3j * rng.standard_normal((M, M))
    gn = g + 0.2 * rng.standard_normal((M,) * 4)
    grads = []
    for space in (mc.DirectSpace(N, M), mc.build_tables(N, M, form="reduced")):
        Ct = dev(C).requires_grad_(True)
        mc.energy(Ct, dev(hn), dev(gn), space).real.backward()
        grads.append(Ct.grad)
    assert rel_inf(grads[0].cpu().numpy(), grads[1].cpu().numpy()) <= ORDER_TOL


@pytest.mark.parametrize("N,M", [(4, 3), (10, 5), (6, 6), (5, 8)])
def test_direct_adjoint_matches_oracle(mc, oracle_native, N, M):
    """Table-free H^dagger C with no symmetry of h or g: the oracle's H with
    h -> h^dagger, g_ksql -> conj(g_lqsk); equal to the adjoint on reduced
    tables that chain single jumps (the same terms in the same order)."""
    rng = np.random.default_rng(N * 10 + M + 1)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    D = oracle_native.dim(N, M)
    C = rng.standard_normal(D) + 1j * rng.standard_normal(D)
    adj = mc.apply_H_adjoint(dev(h), dev(g), dev(C), mc.DirectSpace(N, M))
    ref = oracle_native.apply_h(N, M, h.conj().T, np.transpose(g, (3, 2, 1, 0)).conj(), C)
    assert rel_inf(adj.cpu().numpy(), ref) <= TOL
    tab = mc.apply_H_adjoint(dev(h), dev(g), dev(C),
                             mc.build_tables(N, M, form="reduced", double_jumps=False))
    assert rel_inf(adj.cpu().numpy(), tab.cpu().numpy()) <= ORDER_TOL
    mapped = mc.apply_H_adjoint(dev(h), dev(g), dev(C), mc.build_tables(N, M, form="reduced"))
    assert rel_inf(mapped.cpu().numpy(), ref) <= TOL


def test_direct_density_matrices_reject_bad_sizes(mc):
    C = torch.zeros(mc.dim(1, 9), dtype=torch.complex128, device="cuda")
    with pytest.raises(mc.MCError):
        mc.rho1(C, mc.DirectSpace(1, 9))
