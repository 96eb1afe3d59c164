"""Derivatives of the GW self-energy functional G -> (Sigma_inf[G], Sigma~[G])
on the GPU, composed from libgw calls (see include/gw.h):

  forward   Sigma_inf = HF[gamma(G)],  P0 = Pol[G, G],  P~ = (I - P0)^{-1} P0
            (through the bosonic transforms),  Sigma~ = SE[P~, G]
  JVP       dSigma_inf = HF[gamma(dG)]   (linear)
            dP0 = Pol[dG, G] + Pol[G, dG]
            dP~(i Omega) = (I + P~) dP0(i Omega) (I + P~)
            dSigma~ = SE[dP~, G] + SE[P~, dG]
  VJP       the conjugate transposes of the same steps, in reverse order.

P~ of the current G is needed by both derivatives.  By default it is kept
from the forward call for all q (nk * ntau * naux^2 complex numbers, twice).
With per_q=True nothing is kept: every derivative call loops over q and
rebuilds P~^q from G (one polarization, transform and screened-interaction
solve per q) next to the q-slices it needs, so the memory beyond the inputs
is a few per-q buffers; this costs one more polarization chain per call.
SigmaFunction wraps the pair for torch.autograd.
"""
from __future__ import annotations

import torch

from . import gw


class SigmaDerivatives:
    """Forward evaluation that keeps what the derivatives need (per_q=False),
    or recomputes it per q inside each derivative call (per_q=True)."""

    def __init__(self, path, per_q=False):
        if getattr(path, "finite_size", None) is not None:
            raise NotImplementedError("the derivatives do not include the finite-size corrections")
        self.path = path
        self.ctx = path.ctx
        self.per_q = per_q
        c = self.ctx
        z = dict(dtype=torch.complex128, device="cuda")
        nqb = 1 if per_q else c.nk
        self.buf_tau = torch.empty((nqb, c.ntau, c.naux, c.naux), **z)
        self.buf_w1 = torch.empty((nqb, c.nw_b, c.naux, c.naux), **z)
        self.buf_w2 = torch.empty((nqb, c.nw_b, c.naux, c.naux), **z)
        if per_q:
            self.pt_tau = torch.empty((1, c.ntau, c.naux, c.naux), **z)
            self.p0_w = torch.empty((1, c.nw_b, c.naux, c.naux), **z)
            self.pt_w = torch.empty((1, c.nw_b, c.naux, c.naux), **z)

    def _pt(self, G, q):
        """P~^q(tau) -> self.pt_tau and P~^q(i Omega) -> self.pt_w for one q."""
        c, V = self.ctx, self.path.V
        gw.gw_set_hermitian(c, getattr(self.path, "hermitian", False))
        gw.gw_polarization(c, V, G, q, 1, self.pt_tau)
        gw.gw_tau_to_iw(c, gw.GW_BOSON, self.pt_tau, self.p0_w, batch=1)
        gw.gw_screened_W(c, self.p0_w, self.pt_w)
        gw.gw_iw_to_tau(c, gw.GW_BOSON, self.pt_w, self.pt_tau, batch=1)

    def forward(self, G):
        """Sigma_inf[G], Sigma~[G] (new tensors) and the P~ (tau, i Omega) of G
        (None, None with per_q)."""
        if not self.per_q:
            s_inf, s_tau = self.path.sigma(G)
            s_inf, s_tau = s_inf.clone(), s_tau.clone()
            Pt_tau = self.path.P0.clone()          # sigma() leaves P~(tau) in P0
            Pt_iw = self.path.Pw.clone()
            return s_inf, s_tau, Pt_tau, Pt_iw
        c, V = self.ctx, self.path.V
        z = dict(dtype=torch.complex128, device="cuda")
        s_inf = torch.empty(c.k_shape(), **z)
        gw.gw_hf(c, V, G, None, s_inf)
        s_tau = torch.empty(c.g_shape(), **z)
        gw.gw_mix(c, 1.0, None, s_tau)
        for q in range(c.nk):
            self._pt(G, q)
            gw.gw_self_energy(c, V, G, self.pt_tau, q, 1, s_tau)
        return s_inf, s_tau, None, None

    def jvp(self, G, Pt_tau, Pt_iw, dG, hermitian_dG=False):
        """hermitian_dG: dG is Hermitian per (tau, k), like G (e.g. the Dyson
        response to a Hermitian dSigma); with a Hermitian-mode path the two
        polarization terms are then contracted as Hermitian products."""
        c, V = self.ctx, self.path.V
        herm = getattr(self.path, "hermitian", False)
        z = dict(dtype=torch.complex128, device="cuda")
        d_inf = torch.empty(c.k_shape(), **z)
        gw.gw_hf(c, V, dG, None, d_inf)
        d_tau = torch.empty(c.g_shape(), **z)
        gw.gw_mix(c, 1.0, None, d_tau)
        dP = self.buf_tau
        for q0, nq, pt_tau, pt_w in self._slices(G, Pt_tau, Pt_iw):
            gw.gw_set_hermitian(c, herm, two_slot=herm and hermitian_dG)
            gw.gw_polarization2(c, V, dG, G, q0, nq, dP)
            gw.gw_polarization2(c, V, G, dG, q0, nq, dP, accumulate=True)
            gw.gw_tau_to_iw(c, gw.GW_BOSON, dP, self.buf_w1, batch=nq)
            gw.gw_screened_W_lin(c, pt_w, self.buf_w1, self.buf_w2, adjoint=False)
            gw.gw_iw_to_tau(c, gw.GW_BOSON, self.buf_w2, dP, batch=nq)
            gw.gw_self_energy(c, V, G, dP, q0, nq, d_tau)
            gw.gw_self_energy(c, V, dG, pt_tau, q0, nq, d_tau)
        return d_inf, d_tau

    def vjp(self, G, Pt_tau, Pt_iw, sinf_bar, stau_bar):
        c, V = self.ctx, self.path.V
        z = dict(dtype=torch.complex128, device="cuda")
        Gbar = torch.empty(c.g_shape(), **z)
        gw.gw_mix(c, 1.0, None, Gbar)
        Pbar = self.buf_tau
        for q0, nq, pt_tau, pt_w in self._slices(G, Pt_tau, Pt_iw):
            gw.gw_self_energy_vjp(c, V, G, pt_tau, stau_bar, q0, nq, Gbar, Pbar)
            gw.gw_transform_adjoint(c, gw.GW_BOSON, True, Pbar, self.buf_w1, batch=nq)
            gw.gw_screened_W_lin(c, pt_w, self.buf_w1, self.buf_w2, adjoint=True)
            gw.gw_transform_adjoint(c, gw.GW_BOSON, False, self.buf_w2, Pbar, batch=nq)
            gw.gw_polarization_vjp(c, V, G, Pbar, q0, nq, Gbar)
        gw.gw_hf_vjp(c, V, sinf_bar, Gbar)
        return Gbar

    def _slices(self, G, Pt_tau, Pt_iw):
        """(q0, nq, P~(tau), P~(i Omega)) for all q at once, or q by q with
        P~^q rebuilt from G."""
        if not self.per_q:
            yield 0, self.ctx.nk, Pt_tau, Pt_iw
            return
        for q in range(self.ctx.nk):
            self._pt(G, q)
            yield q, 1, self.pt_tau, self.pt_w


class SigmaFunction(torch.autograd.Function):
    """(Sigma_inf, Sigma~) = SigmaFunction.apply(G, derivs); backward is the
    hand-written VJP above.

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
