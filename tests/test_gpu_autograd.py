"""Energy functional E = <C|H C> with its hand-written backward: gradients
against central finite differences (step 1e-6) and the oracle's density
matrices; torch.autograd.gradcheck on a tiny space."""

import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def fd_check(mc, tab, C, h, g, hermitian, rng, ndir=4, eps=1e-6, kinds=None):
    """Central differences of Re E along seeded directions of C, h and g
    against Re <grad, d>.  `kinds` maps an input to its direction kinds:
    "any" (complex normal entries) or, for h, "hermitian" ((A + A^H) / 2);
    C directions are unit vectors."""
    Cd = dev(C).requires_grad_(True)
    hd = dev(h).requires_grad_(True)
    gd = dev(g).requires_grad_(True)
    E = mc.energy(Cd, hd, gd, tab, hermitian)
    E.real.backward()
    grads = {"C": Cd.grad.cpu().numpy(), "h": hd.grad.cpu().numpy(), "g": gd.grad.cpu().numpy()}
    base = {"C": C, "h": h, "g": g}

    def L(Cx, hx, gx):
        with torch.no_grad():
            return mc.energy(dev(Cx), dev(hx), dev(gx), tab, hermitian).real.item()

    kinds = kinds or {"C": ["any"], "h": ["any"], "g": ["any"]}
    for name, kind in ((n, k) for n in ("C", "h", "g") for k in kinds[n]):
        x0 = base[name]
        for _ in range(ndir):
            d = rng.standard_normal(x0.shape) + 1j * rng.standard_normal(x0.shape)
            if kind == "hermitian":
                d = 0.5 * (d + d.conj().T)
            if name == "C":
                d /= np.linalg.norm(d)
            args_p = dict(base)
            args_m = dict(base)
            args_p[name] = x0 + eps * d
            args_m[name] = x0 - eps * d
            fd = (L(args_p["C"], args_p["h"], args_p["g"]) - L(args_m["C"], args_m["h"], args_m["g"])) / (2 * eps)
            an = float(np.real(np.vdot(grads[name], d)))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (name, fd, an)
    return grads


@pytest.mark.parametrize("N,M,seed,form", [(10, 5, 0, "paper"), (6, 4, 1, "paper"),
                                           (10, 5, 0, "reduced"), (5, 6, 2, "reduced")])
def test_gradients_fd_and_density_matrices(mc, oracle_native, N, M, seed, form):
    C, h, g = W.random_instance(N, M, seed)
    tab = mc.build_tables(N, M, form=form)
    grads = fd_check(mc, tab, C, h, g, True, np.random.default_rng(seed))
    assert rel_inf(grads["h"], np.conj(oracle_native.rho1(N, M, C))) <= 1e-12
    assert rel_inf(grads["g"], 0.5 * np.conj(oracle_native.rho2(N, M, C))) <= 1e-12
    HC = oracle_native.apply_h(N, M, h, g, C)
    assert rel_inf(grads["C"], 2 * HC) <= 1e-12


@pytest.mark.parametrize("form", ["paper", "reduced"])
def test_gradients_non_hermitian(mc, form):
    N, M = 5, 3
    rng = np.random.default_rng(7)
    h = rng.standard_normal((M, M)) + 1j * rng.standard_normal((M, M))
    g = rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4)
    tab = mc.build_tables(N, M, form=form)
    C = W.random_coefficients(rng, tab.dim)
    fd_check(mc, tab, C, h, g, False, rng)


def test_gradcheck_tiny(mc):
    N, M = 3, 3
    tab = mc.build_tables(N, M)
    C, h, g = W.random_instance(N, M, 2)
    rng = np.random.default_rng(3)
    h = h + 0.3j * rng.standard_normal((M, M))       # non-Hermitian
    inputs = (dev(C).requires_grad_(True), dev(h).requires_grad_(True), dev(g).requires_grad_(True))
    f = lambda c, hh, gg: mc.energy(c, hh, gg, tab, False)
    assert torch.autograd.gradcheck(f, inputs, eps=1e-6, atol=1e-7, rtol=1e-6)


@pytest.mark.parametrize("space", ["paper", "direct"])
def test_autograd_workload(mc, oracle_native, space):
    """N = 50, M = 6 (dim 3,478,761): the h-gradient against the oracle's
    rho1, the C-gradient against 2 HC on sampled rows, and central
    differences along 8 seeded directions each of C, of h (Hermitian-
    preserving and arbitrary) and of g.  The g-gradient against every
    rho2 element is in the density-matrix tests."""
    N, M = 50, 6
    C, h, g = W.random_instance(N, M, 3)
    tab = mc.DirectSpace(N, M) if space == "direct" else mc.build_tables(N, M)
    grads = fd_check(mc, tab, C, h, g, None, np.random.default_rng(6), ndir=8,
                     kinds={"C": ["any"], "h": ["hermitian", "any"], "g": ["any"]})
    assert rel_inf(grads["h"], np.conj(oracle_native.rho1(N, M, C))) <= 1e-12
    rows = np.unique(np.concatenate([np.random.default_rng(5).integers(0, tab.dim, 4000),
                                     np.arange(64), tab.dim - 1 - np.arange(64)]))
    ref = 2 * oracle_native.apply_h(N, M, h, g, C, rows)
    assert rel_inf(grads["C"][rows], ref) <= 1e-12
    del tab
    torch.cuda.empty_cache()


@pytest.mark.parametrize("space", ["paper", "reduced", "direct"])
def test_default_arguments_detect_non_hermitian_inputs(mc, space):
    """energy(C, h, g, space) with no `hermitian` argument: non-Hermitian h
    and g must still give the right C-gradient (conj(gbar) HC + gbar H^dagger C),
    checked by central differences; Hermitian inputs are recognised."""
    N, M = 8, 4
    rng = np.random.default_rng(11)
    C, h, g = W.random_instance(N, M, 12)
    tab = mc.DirectSpace(N, M) if space == "direct" else mc.build_tables(N, M, form=space)
    assert mc.is_hermitian(dev(h), dev(g), M, torch.device("cuda"))
    hn = h + 0.4j * rng.standard_normal((M, M))
    gn = g + 0.3 * (rng.standard_normal((M,) * 4) + 1j * rng.standard_normal((M,) * 4))
    assert not mc.is_hermitian(dev(hn), dev(g), M, torch.device("cuda"))
    assert not mc.is_hermitian(dev(h), dev(gn), M, torch.device("cuda"))
    fd_check(mc, tab, C, hn, gn, None, rng, ndir=4)
