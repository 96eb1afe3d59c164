"""Oracle (test infrastructure only): the thermodynamics of Sec. III.C —
the grand potential of Eq. GP,

    Omega[G] = Phi[G] - Tr ln(-G^{-1}) - Tr{Sigma[G] G},
    Phi_GW = Phi_inf + Phi~  (Eq. Phi_GW),

with Phi~ of Eq. tilde_Phi_GW (oracle.gw.phi_gw), and the Galitskii-Migdal
total energy E = Tr{H0 gamma} + (1/2) Tr{Sigma G}.  Tr sums over k
((1/Nk) sum_k), over all Matsubara frequencies ((1/beta) sum_n) and over
spin-orbitals (a factor ns for the spin-restricted matrices).  Plain numpy;
shares no code with the library.

Readings (R20 of the design notes):
  * every equal-time trace takes G(0^-) = gamma (the convergence factor
    e^{i w 0+}); then Tr ln(-G^{-1}) of a free G is (1/beta) sum_a
    ln(1 + e^{-beta xi_a}) per spin, Tr{Sigma_inf G} = Tr{Sigma_inf gamma},
    and the first-order term of the Luttinger-Ward series, (1/2) Tr{Sigma G},
    is Phi_inf = +(1/2) Tr{Sigma_inf gamma}.  Eq. Phi_GW prints -(1/2)
    Tr{Sigma_inf gamma}, which is that term with the equal-time G taken at
    beta^- (= -gamma); with one convention for all of Eq. GP only the +
    sign gives the Hartree-Fock grand potential Omega_0[eps_HF] - (1/2)
    Tr{Sigma_inf gamma} and -dOmega/dmu = N at self-consistency (both pinned);
  * Tr ln(-G^{-1}) splits into the static reference G_ref^{-1} = (i w + mu) S
    - H0 - Sigma_inf, whose sum is the free-fermion closed form
    (1/beta) sum_a ln(1 + e^{-beta xi_a}) over the generalised eigenvalues xi_a
    of (H0 + Sigma_inf - mu S, S), and ln det(I - G_ref Sigma~(i w_n)) =
    ln det M(i w_n) - ln det M_ref(i w_n), M = G^{-1}, which decays as 1/w^2;
  * a Matsubara sum (1/beta) sum_n F(i w_n) of a function that decays faster
    than 1/w and has F(-i w) = conj F(i w) is read off the sparse grid as the
    symmetric average of the fitted tau function at 0+ and 0- (= -beta^-):
    (1/beta) sum_n F = -sum_n Re(r_n) Re F(i w_n), r = w Tp (the beta^- row
    of the fermionic fit); so only Re ln det = ln |det| enters;
  * Tr{Sigma G} = Tr{Sigma_inf gamma} + (1/beta) sum_n tr[Sigma~(i w_n) G(i w_n)].
"""
from __future__ import annotations

import numpy as np

from . import gw


def free_fermion_term(H, S, mu, beta):
    """(1/beta) sum_a ln(1 + e^{-beta xi_a}) per k, xi_a the eigenvalues of
    (H - mu S, S) (overflow-safe)."""
    out = np.empty(H.shape[0])
    for k in range(H.shape[0]):
        L = np.linalg.cholesky(S[k])
        Li = np.linalg.inv(L)
        xi = np.linalg.eigvalsh(Li @ (H[k] - mu * S[k]) @ Li.conj().T)
        out[k] = np.sum(np.maximum(-xi, 0.0) + np.log1p(np.exp(-beta * np.abs(xi))) / beta)
    return out


def matsubara_sum_weights(grids):
    """Weights c_n with (1/beta) sum_n F(i w_n) ~ sum_n c_n Re F(i w_n) for
    fermionic F decaying faster than 1/w: c = -Re(w Tp)."""
    return -np.real(grids.w @ grids.TFp)


def grand_potential(H0, S, Sig_inf, Sig_iw, mu, phi_tilde, grids, ns):
    """Omega and its parts, with G from the Dyson equation at mu; Sig_iw on
    the fermionic sparse set.  Returns a dict."""
    nw, nk, n, _ = Sig_iw.shape
    c = matsubara_sum_weights(grids)
    G = gw.dyson(H0, S, Sig_inf, Sig_iw, mu, grids.wF)
    gamma = gw.density_matrix(gw.to_tau(grids.TFp, G), grids.w)
    tr_ln_dyn = 0.0
    tr_sg_dyn = 0.0
    for iw in range(nw):
        for k in range(nk):
            M = (1j * grids.wF[iw] + mu) * S[k] - H0[k] - Sig_inf[k] - Sig_iw[iw, k]
            Mr = (1j * grids.wF[iw] + mu) * S[k] - H0[k] - Sig_inf[k]
            ld = np.linalg.slogdet(M)[1] - np.linalg.slogdet(Mr)[1]     # ln|det(I - G_ref Sigma~)|
            tr_ln_dyn += c[iw] * ld
            tr_sg_dyn += c[iw] * np.trace(Sig_iw[iw, k] @ G[iw, k]).real
    free = free_fermion_term(H0 + Sig_inf, S, mu, grids.beta)
    tr_ln = ns / nk * (free.sum() + tr_ln_dyn)
    tr_sinf_g = ns / nk * np.einsum("kij,kji->", Sig_inf, gamma).real
    tr_sg = tr_sinf_g + ns / nk * tr_sg_dyn
    phi_inf = 0.5 * tr_sinf_g
    e1 = ns / nk * np.einsum("kij,kji->", H0, gamma).real
    omega = phi_inf + phi_tilde - tr_ln - tr_sg
    n_e = gw.electron_count(gamma, S, ns)
    return dict(omega=omega, phi_inf=phi_inf, phi_tilde=phi_tilde, tr_ln=tr_ln, tr_sigma_g=tr_sg,
                e_one_body=e1, e_gm=e1 + 0.5 * tr_sg, n_e=n_e)
