"""Derivatives of the GW self-energy functional G -> (Sigma_inf[G], Sigma~[G])
on the GPU, composed from libgw calls (see include/gw.h):

  forward   Sigma_inf = HF[gamma(G)],  P0 = Pol[G, G],  P~ = (I - P0)^{-1} P0
            (through the bosonic transforms),  Sigma~ = SE[P~, G]
  JVP       dSigma_inf = HF[gamma(dG)]   (linear)
            dP0 = Pol[dG, G] + Pol[G, dG]
            dP~(i Omega) = (I + P~) dP0(i Omega) (I + P~)
            dSigma~ = SE[dP~, G] + SE[P~, dG]
  VJP       the conjugate transposes of the same steps, in reverse order.

The screened interaction P~ of the current G is recomputed by the forward
call that the backward pass follows (it is kept from that call, not rebuilt
from the adjoint).  SigmaFunction wraps the pair for torch.autograd.
"""
from __future__ import annotations

import torch

from . import gw


class SigmaDerivatives:
    """Forward evaluation that keeps what the derivatives need."""

    def __init__(self, path):
        self.path = path
        self.ctx = path.ctx
        c = self.ctx
        z = dict(dtype=torch.complex128, device="cuda")
        self.buf_tau = torch.empty((c.nk, c.ntau, c.naux, c.naux), **z)
        self.buf_w1 = torch.empty((c.nk, c.nw_b, c.naux, c.naux), **z)
        self.buf_w2 = torch.empty((c.nk, c.nw_b, c.naux, c.naux), **z)

    def forward(self, G):
        """Sigma_inf[G], Sigma~[G] (new tensors) and the P~ (tau, i Omega) of G."""
        s_inf, s_tau = self.path.sigma(G)
        s_inf, s_tau = s_inf.clone(), s_tau.clone()
        Pt_tau = self.path.P0.clone()          # sigma() leaves P~(tau) in P0
        Pt_iw = self.path.Pw.clone()
        return s_inf, s_tau, Pt_tau, Pt_iw

    def jvp(self, G, Pt_tau, Pt_iw, dG):
        c, V = self.ctx, self.path.V
        z = dict(dtype=torch.complex128, device="cuda")
        d_inf = torch.empty(c.k_shape(), **z)
        gw.gw_hf(c, V, dG, None, d_inf)
        dP = self.buf_tau
        gw.gw_polarization2(c, V, dG, G, 0, c.nk, dP)
        gw.gw_polarization2(c, V, G, dG, 0, c.nk, dP, accumulate=True)
        gw.gw_tau_to_iw(c, gw.GW_BOSON, dP, self.buf_w1, batch=c.nk)
        gw.gw_screened_W_lin(c, Pt_iw, self.buf_w1, self.buf_w2, adjoint=False)
        gw.gw_iw_to_tau(c, gw.GW_BOSON, self.buf_w2, dP, batch=c.nk)
        d_tau = torch.empty(c.g_shape(), **z)
        gw.gw_mix(c, 1.0, None, d_tau)
        gw.gw_self_energy(c, V, G, dP, 0, c.nk, d_tau)
        gw.gw_self_energy(c, V, dG, Pt_tau, 0, c.nk, d_tau)
        return d_inf, d_tau

    def vjp(self, G, Pt_tau, Pt_iw, sinf_bar, stau_bar):
        c, V = self.ctx, self.path.V
        z = dict(dtype=torch.complex128, device="cuda")
        Gbar = torch.empty(c.g_shape(), **z)
        gw.gw_mix(c, 1.0, None, Gbar)
        Pbar = self.buf_tau
        gw.gw_self_energy_vjp(c, V, G, Pt_tau, stau_bar, 0, c.nk, Gbar, Pbar)
        gw.gw_transform_adjoint(c, gw.GW_BOSON, True, Pbar, self.buf_w1, batch=c.nk)
        gw.gw_screened_W_lin(c, Pt_iw, self.buf_w1, self.buf_w2, adjoint=True)
        gw.gw_transform_adjoint(c, gw.GW_BOSON, False, self.buf_w2, Pbar, batch=c.nk)
        gw.gw_polarization_vjp(c, V, G, Pbar, 0, c.nk, Gbar)
        gw.gw_hf_vjp(c, V, sinf_bar, Gbar)
        return Gbar


class SigmaFunction(torch.autograd.Function):
    """(Sigma_inf, Sigma~) = SigmaFunction.apply(G, derivs); backward is the
    hand-written VJP above."""

    @staticmethod
    def forward(ctx, G, derivs):
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
