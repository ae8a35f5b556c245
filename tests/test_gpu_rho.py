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


def unique_rho2_index(M):
    """Flat indices of rho2_ksql with k <= s and q <= l (the other elements
    follow from rho_ksql = rho_skql = rho_kslq, exact for bosons)."""
    return np.array([((k * M + s) * M + q) * M + l for k in range(M) for s in range(k, M)
                     for q in range(M) for l in range(q, M)], dtype=np.int64)


def expand_rho2(M, idx, vals):
    """Full rho2 from its unique elements through the two pair symmetries."""
    full = np.full(M ** 4, np.nan + 0j)
    for t, v in zip(idx, vals):
        l = t % M
        q = (t // M) % M
        s = (t // M ** 2) % M
        k = t // M ** 3
        for a, b in ((k, s), (s, k)):
            for c, d in ((q, l), (l, q)):
                full[((a * M + b) * M + c) * M + d] = v
    assert not np.isnan(full.real).any()
    return full.reshape((M,) * 4)


@pytest.fixture(scope="module")
def autograd_size_reference(oracle_native):
    """Oracle rho1 (all 36 elements) and the 441 unique rho2 elements at
    N = 50, M = 6 (dim 3,478,761), seed 3."""
    N, M = 50, 6
    C, _, _ = W.random_instance(N, M, 3)
    idx = unique_rho2_index(M)
    print(f"[rho] oracle rho1 and {idx.size} rho2 elements at N={N}, M={M}", flush=True)
    r1 = oracle_native.rho1(N, M, C)
    r2u = oracle_native.rho2_elements(N, M, C, idx)
    return C, r1, idx, r2u


@pytest.mark.parametrize("space", ["paper", "reduced", "direct"])
def test_autograd_size_every_element(mc, autograd_size_reference, space):
    """N = 50, M = 6: rho1 in full and every unique rho2 element against the
    oracle (the oracle's largest element as the scale), and all 1296 rho2
    elements against the oracle's unique ones expanded by the pair
    symmetries; trace and partial-trace invariants."""
    N, M = 50, 6
    C, r1_ref, idx, r2u_ref = autograd_size_reference
    tab = mc.DirectSpace(N, M) if space == "direct" else mc.build_tables(N, M, form=space)
    Cd = dev(C)
    r1 = mc.rho1(Cd, tab).cpu().numpy()
    r2 = mc.rho2(Cd, tab).cpu().numpy()
    assert abs(np.trace(r1) - N) <= 1e-12 * N
    assert np.allclose(np.einsum("kssl->kl", r2), (N - 1) * r1, rtol=0, atol=1e-10)
    assert rel_inf(r1, r1_ref) <= TOL
    e_u = rel_inf(r2.reshape(-1)[idx], r2u_ref)
    e_all = rel_inf(r2, expand_rho2(M, idx, r2u_ref))
    print(f"[rho] {space}: rho2 rel err {e_u:.2e} (unique), {e_all:.2e} (all)", flush=True)
    assert e_u <= TOL and e_all <= TOL
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


KINDS = {  # space kind: (form, double-jump map); None = table-free
    "paper_map": ("paper", True),
    "reduced_map": ("reduced", True),
    "paper_chained": ("paper", False),
    "reduced_chained": ("reduced", False),
    "direct": (None, None),
}


def make_space(mc, kind, N, M):
    form, has_map = KINDS[kind]
    if form is None:
        return mc.DirectSpace(N, M)
    return mc.build_tables(N, M, form=form, double_jumps=has_map)


# one particle (rho2 = 0), two (a single N-2 configuration), one orbital,
# ragged tiles, M = 8, more than 255 particles
@pytest.mark.parametrize("N,M,seed", [(1, 4, 0), (2, 3, 1), (2, 1, 2), (5, 1, 3), (4, 6, 4),
                                      (9, 8, 5), (13, 5, 6), (300, 2, 7), (33, 3, 8), (8, 7, 9)])
@pytest.mark.parametrize("kind", list(KINDS))
def test_rho_every_space_kind(mc, oracle_native, kind, N, M, seed):
    """Eqs. rho1, rho2 through each source of targets (maps of either form,
    chained single jumps, closed form) against the oracle."""
    C, _, _ = W.random_instance(N, M, seed)
    sp = make_space(mc, kind, N, M)
    Cd = dev(C)
    r1 = mc.rho1(Cd, sp).cpu().numpy()
    r2 = mc.rho2(Cd, sp).cpu().numpy()
    assert rel_inf(r1, oracle_native.rho1(N, M, C)) <= TOL
    ref2 = oracle_native.rho2(N, M, C)
    if N < 2:
        assert not np.any(r2) and not np.any(ref2)
    assert rel_inf(r2, ref2) <= TOL


@pytest.mark.parametrize("kind", list(KINDS))
def test_rho_symmetries_exact(mc, kind):
    """rho_lk = conj(rho_kl); rho_ksql = rho_skql = rho_kslq = conj(rho_qlks),
    bit for bit; diagonal elements real."""
    N, M = 11, 6
    C, _, _ = W.random_instance(N, M, 31)
    sp = make_space(mc, kind, N, M)
    Cd = dev(C)
    r1, r2 = mc.rho1(Cd, sp), mc.rho2(Cd, sp)
    assert torch.equal(r1, r1.T.conj().resolve_conj())
    assert torch.equal(r2, r2.permute(1, 0, 2, 3).contiguous())
    assert torch.equal(r2, r2.permute(0, 1, 3, 2).contiguous())
    assert torch.equal(r2, r2.permute(2, 3, 0, 1).conj().resolve_conj().contiguous())
    assert not torch.any(torch.diagonal(r1).imag)


@pytest.mark.parametrize("kind", ["reduced_map", "direct"])
def test_rho_headline_size_invariants(mc, kind):
    """N = 200, M = 5 (dim 70,058,751), seed 2: tr rho1 = N, sum_s rho_kssl =
    (N-1) rho_kl, and E = sum h rho1 + 1/2 sum g rho2 equals <C|HC> from the
    apply on the same space (Sec. II; the apply is checked against the oracle
    at this size elsewhere)."""
    N, M = 200, 5
    C, h, g = W.random_instance(N, M, 2)
    sp = make_space(mc, kind, N, M)
    Cd, hd, gd = dev(C), dev(h), dev(g)
    r1, r2 = mc.rho1(Cd, sp), mc.rho2(Cd, sp)
    HC = mc.apply_H(hd, gd, Cd, sp)
    E = mc.zdotc(Cd, HC).item()
    E2 = (torch.sum(hd * r1) + 0.5 * torch.sum(gd * r2)).item()
    r1n, r2n = r1.cpu().numpy(), r2.cpu().numpy()
    assert abs(np.trace(r1n) - N) <= 1e-12 * N
    assert rel_inf(np.einsum("kssl->kl", r2n), (N - 1) * r1n) <= 1e-12
    assert abs(E - E2) <= 1e-12 * abs(E)
    del sp, HC
    torch.cuda.empty_cache()
