"""Energy functional E(C, h, g) = <C|H C> as a torch.autograd.Function.

Forward: one H.C apply and a fixed-order <C|HC>.  Backward (torch's
conjugate-Wirtinger convention, upstream gradient gbar = dL/dE*):
    grad_C = conj(gbar) H C + gbar H^dagger C
    grad_h = gbar conj(rho1),           rho1_kl = <a+_k a_l>        (Eq. rho1)
    grad_g = gbar (1/2) conj(rho2),     rho2_ksql = <a+_k a+_s a_q a_l> (Eq. rho2)
since E = sum_kl h_kl rho1_kl + 1/2 sum g_ksql rho2_ksql is linear in h and g
and sesquilinear in C.  When H^dagger = H, H^dagger C is the saved H C and dC
costs no extra pass; otherwise it takes one adjoint apply.  ``hermitian=None``
(the default) decides on the device (mc_is_hermitian: h = h^dagger and
g_ksql = conj(g_lqsk) elementwise); True or False skips the check.  All
arithmetic runs in the library's kernels.
"""

from __future__ import annotations

import torch

from . import api


class Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, h, g, tables, hermitian=None):
        M = tables.M
        h = h.reshape(M, M).contiguous()
        g = g.reshape(M, M, M, M).contiguous()
        if hermitian is None:
            hermitian = api.is_hermitian(h, g, M, C.device)
        HC = api.apply_H(h, g, C, tables)
        E = api.zdotc(C, HC)
        ctx.save_for_backward(C, HC, h, g)
        ctx.tables = tables
        ctx.hermitian = bool(hermitian)
        return E

    @staticmethod
    def backward(ctx, gE):
        C, HC, h, g = ctx.saved_tensors
        tables = ctx.tables
        gE = gE.to(torch.complex128).reshape(()).contiguous()
        grad_C = grad_h = grad_g = None
        if ctx.needs_input_grad[0]:
            HdC = HC if ctx.hermitian else api.apply_H_adjoint(h, g, C, tables)
            grad_C = api.zaxpby(HC, a=gE, conj_a=True, y=HdC, b=gE)
        if ctx.needs_input_grad[1]:
            r1 = api.rho1(C, tables)
            grad_h = api.zaxpby(r1.reshape(-1), a=gE, conj_x=True).reshape(h.shape)
        if ctx.needs_input_grad[2]:
            r2 = api.rho2(C, tables)
            grad_g = api.zaxpby(r2.reshape(-1), a=gE, conj_x=True, scale=0.5).reshape(g.shape)
        return grad_C, grad_h, grad_g, None, None


def energy(C, h, g, tables, hermitian=None):
    return Energy.apply(C, h, g, tables, hermitian)
