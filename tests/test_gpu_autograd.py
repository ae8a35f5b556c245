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


def fd_check(mc, tab, C, h, g, hermitian, rng, ndir=4, eps=1e-6):
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

    for name in ("C", "h", "g"):
        x0 = base[name]
        for _ in range(ndir):
            d = rng.standard_normal(x0.shape) + 1j * rng.standard_normal(x0.shape)
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


def test_autograd_workload_sampled(mc, oracle_native):
    """N = 50, M = 6 (dim 3,478,761): rho-gradients vs oracle, C-gradient vs 2HC
    on sampled rows, and finite differences along seeded directions."""
    N, M = 50, 6
    C, h, g = W.random_instance(N, M, 3)
    tab = mc.build_tables(N, M)
    Cd = dev(C).requires_grad_(True)
    hd = dev(h).requires_grad_(True)
    gd = dev(g).requires_grad_(True)
    E = mc.energy(Cd, hd, gd, tab)
    E.real.backward()
    assert rel_inf(hd.grad.cpu().numpy(), np.conj(oracle_native.rho1(N, M, C))) <= 1e-12
    rows = np.random.default_rng(5).integers(0, tab.dim, 1500)
    ref = 2 * oracle_native.apply_h(N, M, h, g, C, rows)
    assert rel_inf(Cd.grad[torch.from_numpy(rows).cuda()].cpu().numpy(), ref) <= 1e-12
    idx = np.array([0, 7, 100, 777, M ** 4 - 1])
    r2 = oracle_native.rho2_elements(N, M, C, idx)
    assert np.max(np.abs(gd.grad.reshape(-1).cpu().numpy()[idx] - 0.5 * np.conj(r2))) <= 1e-12 * np.max(np.abs(gd.grad.cpu().numpy()))
    rng = np.random.default_rng(6)
    eps = 1e-6
    for _ in range(3):
        d = W.random_coefficients(rng, tab.dim)
        with torch.no_grad():
            ep = mc.energy(dev(C + eps * d), hd, gd, tab).real.item()
            em = mc.energy(dev(C - eps * d), hd, gd, tab).real.item()
        fd = (ep - em) / (2 * eps)
        an = float(np.real(np.vdot(Cd.grad.cpu().numpy(), d)))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
    del tab
    torch.cuda.empty_cache()
