"""Lanczos ground state on the GPU (Sec. VI): Krylov vectors, H.C, dot
products, reorthogonalisation and normalisation run in the library's kernels;
the alpha/beta scalars are read back each step for the tridiagonal
eigenvalue (Sturm bisection in the library) and the stopping test.

The paper caps iterations at dim/8 with full reorthogonalisation; here the
cap is ``max_iter`` and iteration stops once the lowest Ritz value changes by
less than ``tol`` (relative) for three consecutive steps.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from . import api


def tridiag_lowest(alphas, betas) -> float:
    a = np.ascontiguousarray(alphas, dtype=np.float64)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    e = ctypes.c_double()
    L.check(L.load().mc_tridiag_lowest(a.size, a.ctypes.data_as(ctypes.c_void_p),
                                       b.ctypes.data_as(ctypes.c_void_p), ctypes.byref(e)),
            "mc_tridiag_lowest")
    return float(e.value)


def ground_state(h, g, tables, v0: torch.Tensor, max_iter: int = 300, tol: float = 1e-12,
                 reorthogonalize: bool = True, sparse: bool = False):
    """Returns (E0, alphas, betas, iterations).  sparse=True applies H with
    mc_apply_H_sparse (reduced-form tables; for interactions with many
    vanishing coefficients such as the Lieb-Liniger g)."""
    dev, D = tables.device, tables.dim
    cap = int(min(max_iter, D))
    M = tables.M
    h = api._as_dev(h, dev, (M, M))
    g = api._as_dev(g, dev, (M, M, M, M))
    api._require(v0, "v0", torch.complex128, dev, numel=D)
    V = torch.empty((cap + 1 if reorthogonalize else 2, D), dtype=torch.complex128, device=dev)
    w = torch.empty(D, dtype=torch.complex128, device=dev)
    c = torch.empty(cap + 1, dtype=torch.complex128, device=dev)
    alpha_d = torch.empty((), dtype=torch.complex128, device=dev)
    beta_d = torch.empty((), dtype=torch.float64, device=dev)
    ws_g = torch.empty(max(16, (cap + 1) * 64 * 16), dtype=torch.uint8, device=dev)
    ws_n = torch.empty((L.MC_DOT_BLOCKS + 2) * 16, dtype=torch.uint8, device=dev)
    lib = L.load()
    st = api._stream(dev)
    P = api._ptr

    def normalize(src, dst):
        with torch.cuda.device(dev):
            L.check(lib.mc_normalize(D, P(src), P(dst), P(beta_d), P(ws_n), ws_n.numel(), st),
                    "mc_normalize")

    normalize(v0, V[0])
    alphas, betas = [], []
    prev, stable, e0 = None, 0, None
    for j in range(cap):
        cur = V[j] if reorthogonalize else V[j % 2]
        (api.apply_H_sparse if sparse else api.apply_H)(h, g, cur, tables, out=w)
        api.zdotc(cur, w, out=alpha_d)
        if reorthogonalize:
            for _ in range(2):   # classical Gram-Schmidt, twice
                with torch.cuda.device(dev):
                    L.check(lib.mc_zgemv_c(j + 1, D, P(V), D, P(w), P(c), P(ws_g), ws_g.numel(),
                                           st), "mc_zgemv_c")
                    L.check(lib.mc_zgemv_sub(j + 1, D, P(V), D, P(c), P(w), st), "mc_zgemv_sub")
            nxt = V[j + 1]
        else:
            prev_v = V[(j + 1) % 2] if j > 0 else None
            with torch.cuda.device(dev):
                L.check(lib.mc_lanczos_orth(D, P(w), P(cur),
                                            P(prev_v) if prev_v is not None else None,
                                            P(alpha_d), P(beta_d) if j > 0 else None, st),
                        "mc_lanczos_orth")
            nxt = V[(j + 1) % 2]
        normalize(w, nxt)
        a = float(alpha_d.real.item())
        b = float(beta_d.item())
        alphas.append(a)
        e0 = tridiag_lowest(alphas, betas)
        if prev is not None and abs(e0 - prev) <= tol * max(1.0, abs(e0)):
            stable += 1
            if stable >= 3:
                return e0, np.array(alphas), np.array(betas), j + 1
        else:
            stable = 0
        prev = e0
        if b < 1e-14:
            break
        betas.append(b)
    return e0, np.array(alphas), np.array(betas), len(alphas)
