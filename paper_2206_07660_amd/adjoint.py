"""Derivatives of the GW self-energy functional G -> (Sigma_inf[G], Sigma~[G])
on the GPU, behind torch.autograd.  The chain and its derivatives run in
libgw's whole-chain calls (include/gw.h):

  forward   gw_sigma       Sigma_inf = HF[gamma(G)], P0 = Pol[G, G],
                           P~ = (I - P0)^{-1} P0 (through the bosonic
                           transforms), Sigma~ = SE[P~, G]
  JVP       gw_sigma_jvp   dSigma_inf = HF[gamma(dG)], dP0 = Pol[dG, G] + Pol[G, dG],
                           dP~(i Omega) = (I + P~) dP0(i Omega) (I + P~),
                           dSigma~ = SE[dP~, G] + SE[P~, dG]
  VJP       gw_sigma_vjp   the conjugate transposes of the same steps, in
                           reverse order.

P~ of the current G is needed by both derivatives.  By default it is kept
from the forward call for all q (nk * (ntau + nw_b) * naux^2 complex
numbers).  With per_q=True nothing is kept: the library rebuilds P~^q from G
q by q inside every call (one polarization, transform and
screened-interaction solve per q), so the memory beyond the inputs is a few
per-q buffers in the workspace; this costs one more polarization chain per
call.
"""
from __future__ import annotations

import torch

from . import gw


class SigmaDerivatives:
    """Forward evaluation that keeps what the derivatives need (per_q=False),
    or has the library recompute it per q inside each derivative call
    (per_q=True)."""

    def __init__(self, path, per_q=False):
        if getattr(path, "finite_size", None) is not None:
            raise NotImplementedError("the derivatives do not include the finite-size corrections")
        self.path = path
        self.ctx = path.ctx
        self.per_q = per_q

    def _herm(self, two_slot=False):
        herm = getattr(self.path, "hermitian", False)
        gw.gw_set_hermitian(self.ctx, herm, two_slot=herm and two_slot)

    def forward(self, G):
        """Sigma_inf[G], Sigma~[G] (new tensors) and the P~ (tau, i Omega) of G
        (None, None with per_q)."""
        c, V = self.ctx, self.path.V
        z = dict(dtype=torch.complex128, device="cuda")
        s_inf = torch.empty(c.k_shape(), **z)
        s_tau = torch.empty(c.g_shape(), **z)
        self._herm()
        if self.per_q:
            gw.gw_sigma(c, V, G, s_inf, s_tau)
            return s_inf, s_tau, None, None
        Pt_tau = torch.empty((c.nk, c.ntau, c.naux, c.naux), **z)
        P0_iw = torch.empty((c.nk, c.nw_b, c.naux, c.naux), **z)
        Pt_iw = torch.empty((c.nk, c.nw_b, c.naux, c.naux), **z)
        gw.gw_sigma(c, V, G, s_inf, s_tau, P_tau=Pt_tau, P0_iw=P0_iw, Pt_iw=Pt_iw)
        return s_inf, s_tau, Pt_tau, Pt_iw

    def jvp(self, G, Pt_tau, Pt_iw, dG, hermitian_dG=False):
        """hermitian_dG: dG is Hermitian per (tau, k), like G (e.g. the Dyson
        response to a Hermitian dSigma); with a Hermitian-mode path the two
        polarization terms are then contracted as Hermitian products."""
        c = self.ctx
        z = dict(dtype=torch.complex128, device="cuda")
        d_inf = torch.empty(c.k_shape(), **z)
        d_tau = torch.empty(c.g_shape(), **z)
        self._herm(two_slot=hermitian_dG)
        gw.gw_sigma_jvp(c, self.path.V, G, Pt_tau, Pt_iw, dG, d_inf, d_tau)
        return d_inf, d_tau

    def vjp(self, G, Pt_tau, Pt_iw, sinf_bar, stau_bar):
        c = self.ctx
        Gbar = torch.empty(c.g_shape(), dtype=torch.complex128, device="cuda")
        self._herm()
        gw.gw_sigma_vjp(c, self.path.V, G, Pt_tau, Pt_iw, sinf_bar, stau_bar, Gbar)
        return Gbar


class SigmaFunction(torch.autograd.Function):
    """(Sigma_inf, Sigma~) = SigmaFunction.apply(G, derivs); backward is the
    hand-written VJP (gw_sigma_vjp).

    When derivs.path runs the polarization in Hermitian mode (GWPath's
    default), G must be Hermitian per (tau, k); the forward checks this and
    raises ValueError otherwise (build the path with hermitian=False to
    differentiate at a general complex G).  The VJP itself holds for any G."""

    @staticmethod
    def forward(ctx, G, derivs):
        if getattr(derivs.path, "hermitian", False):
            dev = (G - G.conj().transpose(-1, -2)).abs().max().item()
            if dev > 1e-10 * max(1.0, G.abs().max().item()):
                raise ValueError(f"G is not Hermitian per (tau, k) (deviation {dev:.2e}); the path "
                                 "computes the polarization in Hermitian mode")
        s_inf, s_tau, Pt_tau, Pt_iw = derivs.forward(G.detach().contiguous())
        ctx.derivs = derivs
        ctx.save_for_backward(G.detach(), Pt_tau, Pt_iw)
        return s_inf, s_tau

    @staticmethod
    def backward(ctx, g_inf, g_tau):
        G, Pt_tau, Pt_iw = ctx.saved_tensors
        z = torch.complex128
        g_inf = torch.zeros(G.shape[1:], dtype=z, device=G.device) if g_inf is None else g_inf.contiguous()
        g_tau = torch.zeros_like(G) if g_tau is None else g_tau.contiguous()
        return ctx.derivs.vjp(G, Pt_tau, Pt_iw, g_inf, g_tau), None
