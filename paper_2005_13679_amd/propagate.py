"""Short Iterative Lanczos (SIL) time steps C(t + dt) = exp(-i H dt) C(t).

Sec. II names the SIL integrator as the time-dependent use of repeated H.C
(Park and Light's method): a Krylov basis V_k = [v_0, ..., v_{k-1}] of
(H, C/|C|) is built by Lanczos with full reorthogonalisation, the projected
tridiagonal T_k gives y = exp(-i T_k dt) e_0, and C(t + dt) ~ |C| V_k y.
The basis grows until the a-posteriori error estimate
|C| beta_k |y_{k-1}| (the weight the next Krylov vector would receive) falls
below ``tol`` or ``kmax`` is reached.

Every vector operation runs in the library's kernels (mc_apply_H, mc_zdotc,
mc_zgemv_c / mc_zgemv_sub, mc_normalize, mc_zgemv_n); the k x k exponential,
the scaling by |C| and the error estimate are the library's host routine
mc_sil_coefficients.  alpha and beta are read back after each Lanczos step
for the stopping test.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from . import api


def tridiag_expv(alphas, betas, dt: float) -> np.ndarray:
    """exp(-i T dt) e_0 for the symmetric tridiagonal T (host)."""
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if b.size < max(0, a.size - 1):
        raise ValueError("need K-1 off-diagonal entries")
    y = np.empty(2 * a.size, dtype=np.float64)
    L.check(L.load().mc_tridiag_expv(a.size, a.ctypes.data_as(ctypes.c_void_p),
                                     b.ctypes.data_as(ctypes.c_void_p), float(dt),
                                     y.ctypes.data_as(ctypes.c_void_p)), "mc_tridiag_expv")
    return y[0::2] + 1j * y[1::2]


def sil_coefficients(alphas, betas, beta_next: float, norm_c: float, dt: float):
    """(coefficients |C| exp(-i T dt) e_0 as complex128, error estimate,
    invariant-space flag) from the library (host routine)."""
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    if b.size < max(0, a.size - 1):
        raise ValueError("need K-1 off-diagonal entries")
    coef = np.empty(2 * a.size, dtype=np.float64)
    err = ctypes.c_double()
    inv = ctypes.c_int32()
    L.check(L.load().mc_sil_coefficients(a.size, a.ctypes.data_as(ctypes.c_void_p),
                                         b.ctypes.data_as(ctypes.c_void_p), float(beta_next),
                                         float(norm_c), float(dt),
                                         coef.ctypes.data_as(ctypes.c_void_p), ctypes.byref(err),
                                         ctypes.byref(inv)), "mc_sil_coefficients")
    return coef.view(np.complex128), float(err.value), bool(inv.value)


class SILStepper:
    """Reusable SIL stepper for one (tables, h, g): Krylov storage for up to
    ``kmax`` vectors is allocated once."""

    def __init__(self, tables, h, g, kmax: int = 30):
        self.t = tables
        self.dev, self.D, self.M = tables.device, tables.dim, tables.M
        self.kmax = int(max(1, min(kmax, self.D)))
        M = self.M
        self.h = api._as_dev(h, self.dev, (M, M))
        self.g = api._as_dev(g, self.dev, (M, M, M, M))
        D, k = self.D, self.kmax
        self.V = torch.empty((k + 1, D), dtype=torch.complex128, device=self.dev)
        self.w = torch.empty(D, dtype=torch.complex128, device=self.dev)
        self.c = torch.empty(k + 1, dtype=torch.complex128, device=self.dev)
        self.alpha_d = torch.empty((), dtype=torch.complex128, device=self.dev)
        self.beta_d = torch.empty((), dtype=torch.float64, device=self.dev)
        self.ws_g = torch.empty(max(16, (k + 1) * 64 * 16), dtype=torch.uint8, device=self.dev)
        self.ws_n = torch.empty((L.MC_DOT_BLOCKS + 2) * 16, dtype=torch.uint8, device=self.dev)

    def step(self, C: torch.Tensor, dt: float, tol: float = 1e-12, out: torch.Tensor | None = None,
             k: int | None = None):
        """Returns (C(t+dt), krylov_dim, error_estimate).  With ``k`` given,
        exactly k Krylov vectors are used (no early stop, unless the space is
        exhausted)."""
        dev, D = self.dev, self.D
        api._require(C, "C", torch.complex128, dev, numel=D)
        if out is None:
            out = torch.empty_like(C)
        api._require(out, "out", torch.complex128, dev, numel=D)
        lib = L.load()
        st = api._stream(dev)
        P = api._ptr
        cap = self.kmax if k is None else int(min(k, self.kmax))
        V, w, c = self.V, self.w, self.c
        with torch.cuda.device(dev):
            L.check(lib.mc_normalize(D, P(C), P(V[0]), P(self.beta_d), P(self.ws_n),
                                     self.ws_n.numel(), st), "mc_normalize")
        norm_c = float(self.beta_d.item())
        if norm_c == 0.0:
            out.copy_(C)
            return out, 0, 0.0
        alphas, betas = [], []
        coef, err, m = None, float("inf"), 0
        for j in range(cap):
            api.apply_H(self.h, self.g, V[j], self.t, out=w)
            api.zdotc(V[j], w, out=self.alpha_d)
            for _ in range(2):   # classical Gram-Schmidt, twice
                with torch.cuda.device(dev):
                    L.check(lib.mc_zgemv_c(j + 1, D, P(V), D, P(w), P(c), P(self.ws_g),
                                           self.ws_g.numel(), st), "mc_zgemv_c")
                    L.check(lib.mc_zgemv_sub(j + 1, D, P(V), D, P(c), P(w), st), "mc_zgemv_sub")
            with torch.cuda.device(dev):
                L.check(lib.mc_normalize(D, P(w), P(V[j + 1]), P(self.beta_d), P(self.ws_n),
                                         self.ws_n.numel(), st), "mc_normalize")
            alphas.append(float(self.alpha_d.real.item()))
            b = float(self.beta_d.item())
            m = j + 1
            coef, err, invariant = sil_coefficients(alphas, betas, b, norm_c, dt)
            if invariant or (k is None and err < tol):
                break
            betas.append(b)
        coef = torch.from_numpy(np.ascontiguousarray(coef)).to(dev)
        with torch.cuda.device(dev):
            L.check(lib.mc_zgemv_n(m, D, P(V), D, P(coef), P(out), st), "mc_zgemv_n")
        return out, m, err


def sil_step(tables, h, g, C: torch.Tensor, dt: float, kmax: int = 30, tol: float = 1e-12,
             k: int | None = None):
    """One SIL step; see SILStepper.step."""
    return SILStepper(tables, h, g, kmax=kmax if k is None else max(kmax, k)).step(C, dt, tol, k=k)
