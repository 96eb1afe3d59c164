"""scGW driver on the GPU: one Sigma[G] + Pi evaluation and the damped
fixed-point iteration of the paper's workflow (Sec. IV.A, Algorithm 1).

Every numeric step is a call into libgw (see include/gw.h); torch only holds
the device buffers.  Readings: the damped fixed point Sigma <- (1 - a) Sigma +
a Sigma[G] with a = 0.5 on both the static and the dynamic part, G_0 from H0
at the chemical potential of the target electron count, convergence measured
as the largest |Sigma[G_t] - Sigma_t| over all elements.
"""
from __future__ import annotations

import dataclasses

import torch

from . import gw


@dataclasses.dataclass
class State:
    mu: float
    sig_inf: torch.Tensor
    sig_tau: torch.Tensor
    G_tau: torch.Tensor
    G_iw: torch.Tensor
    n_e: float = 0.0
    dsig: float = float("nan")
    iteration: int = 0


class GWPath:
    """hermitian: every G given to sigma() is Hermitian per (tau, k), as any
    Green's function of Hermitian H0, S and Sigma is, and V has the pair
    relation; gw_polarization then contracts only half of each P0 matrix.
    finite_size: None, or (chi, head) with the Madelung constant chi and the
    ntau values head[i] = eps^{-1}_00(-tau_i) - 1; sigma() then adds the
    corrections of Eqs. K_corr and GW_head_corr (gw_finite_size)."""

    def __init__(self, ctx: gw.Context, V, H0, S, n_target, alpha=0.5, hermitian=True,
                 finite_size=None, want_phi=False, fixed_mu=False):
        self.ctx, self.V, self.H0, self.S = ctx, V, H0, S
        # fixed_mu: grand-canonical iteration.  After start() has found the mu
        # of n_target for G0, every Green's function is the Dyson solution at
        # that mu (no search); the electron count is reported, not imposed.
        self.fixed_mu = bool(fixed_mu)
        # want_phi: sigma() takes the screened-interaction solve through
        # gw_screened_W_phi and keeps Phi~ (Eq. tilde_Phi_GW) of that G in self.phi
        self.want_phi, self.phi = bool(want_phi), float("nan")
        self.finite_size = None if finite_size is None else (float(finite_size[0]), finite_size[1])
        self.hermitian = bool(hermitian)
        gw.gw_set_hermitian(ctx, self.hermitian)
        self.n_target, self.alpha = float(n_target), float(alpha)
        c = ctx
        z = dict(dtype=torch.complex128, device="cuda")
        self.P0 = torch.empty((c.nk, c.ntau, c.naux, c.naux), **z)      # also holds P~(tau)
        self.P0w = torch.empty((c.nk, c.nw_b, c.naux, c.naux), **z)
        self.Pw = torch.empty((c.nk, c.nw_b, c.naux, c.naux), **z)
        self.new_inf = torch.empty(c.k_shape(), **z)
        self.new_tau = torch.empty(c.g_shape(), **z)
        self.gamma = torch.empty(c.k_shape(), **z)
        self.sig_iw = torch.empty(c.giw_shape(), **z)

    # ------------------------------------------------ Sigma[G] + Pi -----
    def sigma(self, G_tau, out_inf=None, out_tau=None):
        """Sigma_inf[G] (Eqs. HF_J, HF_K) and Sigma~[G](tau) (Eqs. tilde_P0_tau ...
        tilde_sigma2), all q at once (gw_sigma); P~(tau) and P~(i Omega) of G
        stay in self.P0 and self.Pw."""
        c = self.ctx
        out_inf = self.new_inf if out_inf is None else out_inf
        out_tau = self.new_tau if out_tau is None else out_tau
        gw.gw_set_hermitian(c, self.hermitian)         # the context may be shared
        phi = gw.gw_sigma(c, self.V, G_tau, out_inf, out_tau, gamma=self.gamma, P_tau=self.P0,
                          P0_iw=self.P0w, Pt_iw=self.Pw, want_phi=self.want_phi)
        if self.want_phi:
            self.phi = phi
        if self.finite_size is not None:
            chi, head = self.finite_size
            gw.gw_finite_size(c, self.S, chi, self.gamma, out_inf, G_tau, head, out_tau)
        return out_inf, out_tau

    def green(self, sig_inf, sig_iw, mu, G_iw, G_tau):
        """G(i w) and G(tau) of the self-energy: at the mu of n_target
        (gw_find_mu from mu), or at mu itself when fixed_mu.  Returns (mu, N_e)."""
        c = self.ctx
        if not self.fixed_mu:
            return gw.gw_find_mu(c, self.H0, self.S, sig_inf, sig_iw, self.n_target, mu,
                                 G_iw=G_iw, G_tau=G_tau)
        gw.gw_dyson_G(c, self.H0, self.S, sig_inf, sig_iw, mu, G_iw)
        gw.gw_iw_to_tau(c, gw.GW_FERMION, G_iw, G_tau)
        return mu, gw.gw_density(c, G_tau, self.S, self.gamma)

    # ------------------------------------------------ scGW loop -----------
    def start(self, mu0=0.0, search=True):
        """Sigma = 0 and G0 at the mu of n_target (searched from mu0), or at mu0
        itself with search=False."""
        c = self.ctx
        z = dict(dtype=torch.complex128, device="cuda")
        st = State(mu0, torch.empty(c.k_shape(), **z), torch.empty(c.g_shape(), **z),
                   torch.empty(c.g_shape(), **z), torch.empty(c.giw_shape(), **z))
        gw.gw_mix(c, 1.0, None, st.sig_inf)
        gw.gw_mix(c, 1.0, None, st.sig_tau)
        if search:
            st.mu, st.n_e = gw.gw_find_mu(c, self.H0, self.S, None, None, self.n_target, mu0,
                                          G_iw=st.G_iw, G_tau=st.G_tau)
        else:
            gw.gw_dyson_G(c, self.H0, self.S, None, None, mu0, st.G_iw)
            gw.gw_iw_to_tau(c, gw.GW_FERMION, st.G_iw, st.G_tau)
            st.n_e = gw.gw_density(c, st.G_tau, self.S, self.gamma)
        return st

    def step(self, st: State, want_diff=True):
        """One damped scGW iteration: Sigma[G] -> mix -> tau->iw -> mu -> Dyson -> iw->tau."""
        c = self.ctx
        self.sigma(st.G_tau)
        d1 = gw.gw_mix(c, self.alpha, self.new_inf, st.sig_inf, want_diff)
        d2 = gw.gw_mix(c, self.alpha, self.new_tau, st.sig_tau, want_diff)
        gw.gw_tau_to_iw(c, gw.GW_FERMION, st.sig_tau, self.sig_iw)
        st.mu, st.n_e = self.green(st.sig_inf, self.sig_iw, st.mu, st.G_iw, st.G_tau)
        st.dsig = max(d1, d2) if want_diff else float("nan")
        st.iteration += 1
        return st

    def thermodynamics(self, st: State, phi=None):
        """Grand potential (Eq. GP) and Galitskii-Migdal energy of the state's
        self-energy at its mu (gw_thermodynamics).  phi: Phi~ of the G that
        produced the self-energy; default: the last sigma() call's (needs
        want_phi)."""
        c = self.ctx
        phi = self.phi if phi is None else float(phi)
        gw.gw_tau_to_iw(c, gw.GW_FERMION, st.sig_tau, self.sig_iw)
        return gw.gw_thermodynamics(c, self.H0, self.S, st.sig_inf, self.sig_iw, st.mu, phi)
