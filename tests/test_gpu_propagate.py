"""GPU Short Iterative Lanczos steps vs the oracle: the dense matrix
exponential on tiny spaces, the oracle's SIL step (same Krylov dimension) on
larger ones, and exp(-i H dt)'s invariants at N = 200, M = 5.

Tolerance: SIL products agree with the oracle's to 1e-11 relative; each of
the k <= 12 Krylov steps carries the 1e-12 H.C bar plus dot products and
Gram-Schmidt in a different order, so k * 1e-12 bounds the drift."""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense
from oracle import propagate as pr
from tests.gpu_helpers import rel_inf

pytestmark = pytest.mark.gpu

TOL = 1e-11


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("N,M,seed,form", [(3, 3, 0, "paper"), (2, 4, 1, "reduced"), (4, 2, 2, "paper"),
                                           (1, 5, 3, "reduced"), (5, 3, 4, "reduced")])
def test_full_krylov_matches_expm(mc, N, M, seed, form):
    C, h, g = W.random_instance(N, M, seed)
    H = dense.hamiltonian(N, M, h, g)
    tab = mc.build_tables(N, M, form=form)
    for dt in (0.01, 0.5):
        got, m, err = mc.sil_step(tab, dev(h), dev(g), dev(C), dt, k=C.size)
        assert rel_inf(got.cpu().numpy(), pr.expm_step(H, C, dt)) <= TOL


@pytest.mark.parametrize("N,M,seed,k,form", [(10, 5, 0, 12, "reduced"), (8, 6, 5, 10, "paper"),
                                             (20, 3, 6, 8, "reduced"), (6, 8, 7, 6, "reduced")])
def test_matches_oracle_sil(mc, oracle_native, N, M, seed, k, form):
    C, h, g = W.random_instance(N, M, seed)
    dt = 0.02
    ref, m_ref, e_ref = pr.sil_step(lambda v: oracle_native.apply_h(N, M, h, g, v), C, dt, k=k)
    tab = mc.build_tables(N, M, form=form)
    got, m, err = mc.sil_step(tab, dev(h), dev(g), dev(C), dt, k=k)
    assert m == m_ref
    assert rel_inf(got.cpu().numpy(), ref) <= TOL
    assert abs(err - e_ref) <= 1e-6 * max(e_ref, 1e-300) + 1e-15


def test_adaptive_stops_at_tolerance(mc):
    N, M = 12, 5
    C, h, g = W.random_instance(N, M, 8)
    tab = mc.build_tables(N, M, form="reduced")
    st = mc.SILStepper(tab, dev(h), dev(g), kmax=40)
    out, m, err = st.step(dev(C), 1e-3, tol=1e-12)
    assert m < 40 and err < 1e-12
    # a stepper is reusable: two half steps agree with one full step
    half, _, e1 = st.step(dev(C), 5e-4, tol=1e-13)
    two, _, e2 = st.step(half.clone(), 5e-4, tol=1e-13)
    full, _, e3 = st.step(dev(C), 1e-3, tol=1e-13)
    assert float((two - full).abs().max()) <= 1e-11


def test_large_space_invariants(mc):
    """N = 200, M = 5: norm and energy are conserved by the Krylov projection."""
    N, M = 200, 5
    C, h, g = W.random_instance(N, M, 2)
    tab = mc.build_tables(N, M, form="reduced")
    hd, gd, Cd = dev(h), dev(g), dev(C)
    out, m, err = mc.sil_step(tab, hd, gd, Cd, 2e-4, k=8)
    assert m == 8
    n0 = float(torch.linalg.vector_norm(Cd))
    n1 = float(torch.linalg.vector_norm(out))
    assert abs(n1 - n0) <= 1e-12 * n0
    e0 = mc.zdotc(Cd, mc.apply_H(hd, gd, Cd, tab)).item().real
    e1 = mc.zdotc(out, mc.apply_H(hd, gd, out, tab)).item().real
    assert abs(e1 - e0) <= 1e-11 * abs(e0)
    del tab, out, Cd
    torch.cuda.empty_cache()
