"""torch.autograd.Function wrappers of the twisted-mass operator.

Both functions take canonical complex128 tensors on the device -- psi and
chi ``[Vh][4][3]`` (odd sites), the gauge field ``[4][V][3][3]`` -- and return
a real FP64 scalar.  Forward and backward run entirely in libtmhop's HIP
kernels: the psi-gradient is Qhat(-sign) applied to chi, the link gradient
comes from the gauge-link derivative kernel (tmh_qtm_force, Euclidean kind),
the reductions are the library's deterministic FP64 scalar products.

Gradients follow torch's convention for complex inputs and a real output:
grad = dL/dRe + i dL/dIm, i.e. dL = Re sum conj(grad) d(input).
"""

from __future__ import annotations

import torch

from . import tmhop as _t


def _prepare(lat, psi, U):
    G = _t.gauge_import(lat, U.detach())
    p = _t.spinor_import(lat, psi.detach())
    return G, p


class QtmBilinear(torch.autograd.Function):
    """L = Re <chi, Qhat(sign) psi>."""

    @staticmethod
    def forward(ctx, psi, U, chi, lat, kappa, mu, theta, sign):
        G, p = _prepare(lat, psi, U)
        c = _t.spinor_import(lat, chi.detach())
        q = lat.new_spinor()
        _t.qtm_apply(lat, q, G, p, kappa, mu, theta, sign)
        L = _t.scalar_prod_r(lat, c, q)
        ctx.lat, ctx.args = lat, (kappa, mu, tuple(theta), int(sign))
        ctx.fields = (G, p, c, q)
        return torch.tensor(L, dtype=torch.float64, device=psi.device)

    @staticmethod
    def backward(ctx, gL):
        lat = ctx.lat
        kappa, mu, theta, sign = ctx.args
        G, p, c, q = ctx.fields
        g_psi = g_U = g_chi = None
        if ctx.needs_input_grad[0]:
            r = lat.new_spinor()
            _t.qtm_apply(lat, r, G, c, kappa, mu, theta, -sign)
            g_psi = _t.spinor_export(lat, r) * gL
        if ctx.needs_input_grad[1]:
            F = lat.new_gauge(zero=True)
            _t.qtm_force(lat, F, G, c, p, kappa, mu, theta, sign, 1.0, "euclid")
            g_U = _t.gauge_export(lat, F) * gL
        if ctx.needs_input_grad[2]:
            g_chi = _t.spinor_export(lat, q) * gL
        return g_psi, g_U, g_chi, None, None, None, None, None


class QtmNorm2(torch.autograd.Function):
    """L = |Qhat(sign) psi|^2."""

    @staticmethod
    def forward(ctx, psi, U, lat, kappa, mu, theta, sign):
        G, p = _prepare(lat, psi, U)
        q = lat.new_spinor()
        _t.qtm_apply(lat, q, G, p, kappa, mu, theta, sign)
        L = _t.norm2(lat, q)
        ctx.lat, ctx.args = lat, (kappa, mu, tuple(theta), int(sign))
        ctx.fields = (G, p, q)
        return torch.tensor(L, dtype=torch.float64, device=psi.device)

    @staticmethod
    def backward(ctx, gL):
        lat = ctx.lat
        kappa, mu, theta, sign = ctx.args
        G, p, q = ctx.fields
        g_psi = g_U = None
        if ctx.needs_input_grad[0]:
            r = lat.new_spinor()
            _t.qtm_apply(lat, r, G, q, kappa, mu, theta, -sign)
            g_psi = 2.0 * _t.spinor_export(lat, r) * gL
        if ctx.needs_input_grad[1]:
            F = lat.new_gauge(zero=True)
            _t.qtm_force(lat, F, G, q, p, kappa, mu, theta, sign, 2.0, "euclid")
            g_U = _t.gauge_export(lat, F) * gL
        return g_psi, g_U, None, None, None, None, None


def qtm_bilinear(lat, chi, psi, U, kappa, mu, theta, sign=+1):
    """Re <chi, Qhat(sign) psi> as a differentiable torch scalar."""
    return QtmBilinear.apply(psi, U, chi, lat, kappa, mu, theta, sign)


def qtm_norm2(lat, psi, U, kappa, mu, theta, sign=+1):
    """|Qhat(sign) psi|^2 as a differentiable torch scalar."""
    return QtmNorm2.apply(psi, U, lat, kappa, mu, theta, sign)
