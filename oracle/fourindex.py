"""Oracle (test infrastructure only): the four-index route for tiny inputs.

Builds the bare interaction U from V (Eq. U_decompose), the four-index bubble
Pi(tau) (Eq. P0_tau), solves W = U + (1/Nk) U Pi W (Eq. W) in pair space for
each transfer q and bosonic frequency, and evaluates Sigma~ from W~ = W - U
through Eq. tilde_sigma.  Nothing here uses the density-fitted objects P0, P~,
so agreement with the density-fitted chain pins its algebra (the Q pairing,
the 1/Nk and spin factors, and the screened-interaction solve).

Pair index for transfer q: (k, x, y) is the orbital pair with momenta
(k, k - q).  Reading R2: the bubble's two Green's functions are oriented as in
the real-space product P0(r, r'; tau) = G(r, r'; tau) G(r', r; -tau), which is
the orientation of Eq. tilde_P0_tau; with time reversal it coincides with
Eq. P0_tau as printed.  G(-tau) = -G(beta - tau) (fermionic antiperiodicity).
"""
from __future__ import annotations

import numpy as np

from .gw import mesh_tables


def _vpair(V, plus):
    """Vk[k1][k2] = V^{k1,k2}(Q) as (Q, i, j), read from the q-major storage."""
    nk = V.shape[0]
    out = np.empty((nk, nk) + V.shape[2:], V.dtype)
    for q in range(nk):
        for k in range(nk):
            out[k, plus[q, k]] = V[q, k]
    return out


def u_matrix(Vk, minus, q):
    """U_q[(k1,i,j),(k4,k,l)] = U^{k1,k1-q,k4-q,k4}_{ijkl} = sum_Q V^{k1,k1-q}_{ij}(Q) V^{k4-q,k4}_{kl}(Q)."""
    nk, _, naux, n, _ = Vk.shape
    left = np.stack([Vk[k, minus[q, k]] for k in range(nk)])       # (k1, Q, i, j)
    right = np.stack([Vk[minus[q, k], k] for k in range(nk)])      # (k4, Q, k, l)
    L = np.transpose(left, (0, 2, 3, 1)).reshape(nk * n * n, naux)
    R = np.transpose(right, (1, 0, 2, 3)).reshape(naux, nk * n * n)
    return L @ R, L, R


def pi_matrix(G_tau, minus, q, t, ns):
    """Pi_q(tau_t)[(k6,a,b),(k7,c,d)] = delta_{k6 k7} ns G^{k6}_{bc}(tau) G^{k6-q}_{da}(-tau)."""
    ntau, nk, n, _ = G_tau.shape
    P = np.zeros((nk, n, n, nk, n, n), np.complex128)
    for k6 in range(nk):
        Gp = G_tau[t, k6]                                   # G^{k6}(tau)
        Gm = -G_tau[ntau - 1 - t, minus[q, k6]]             # G^{k6-q}(-tau)
        P[k6, :, :, k6, :, :] = ns * np.einsum("bc,da->abcd", Gp, Gm)
    return P.reshape(nk * n * n, nk * n * n)


def screened_tilde_W(V, G_tau, mesh, ns, grids):
    """W~_q(i Omega_m) and W~_q(tau_i) for every q, in pair space."""
    plus, minus = mesh_tables(mesh)
    Vk = _vpair(V, plus)
    ntau, nk, n, _ = G_tau.shape
    d = nk * n * n
    Wiw = np.zeros((nk, len(grids.wB), d, d), np.complex128)
    for q in range(nk):
        U, _, _ = u_matrix(Vk, minus, q)
        Pi_tau = np.stack([pi_matrix(G_tau, minus, q, t, ns) for t in range(ntau)])
        Pi_iw = np.tensordot(grids.TB, Pi_tau, axes=(1, 0))
        for m in range(len(grids.wB)):
            W = np.linalg.solve(np.eye(d) - U @ Pi_iw[m] / nk, U)
            Wiw[q, m] = W - U
    Wtau = np.stack([np.tensordot(grids.TBp, Wiw[q], axes=(1, 0)) for q in range(nk)])
    return Wiw, Wtau


def self_energy(G_tau, Wtau, mesh):
    """Sigma~^k_{ij}(tau) = -(1/Nk) sum_q sum_{ab} G^{k-q}_{ab}(tau) W~^{k,k-q,k-q,k}_{iabj}(tau)."""
    _, minus = mesh_tables(mesh)
    ntau, nk, n, _ = G_tau.shape
    W6 = Wtau.reshape(nk, ntau, nk, n, n, nk, n, n)
    out = np.zeros_like(G_tau)
    for t in range(ntau):
        for k in range(nk):
            for q in range(nk):
                out[t, k] -= np.einsum("ab,iabj->ij", G_tau[t, minus[q, k]],
                                       W6[q, t, k, :, :, k, :, :]) / nk
    return out


def df_tilde_W(V, Pw, mesh):
    """V P~ V in the same pair space (Eq. tilde_W_DF2), for comparison."""
    plus, minus = mesh_tables(mesh)
    Vk = _vpair(V, plus)
    nk = V.shape[0]
    out = []
    for q in range(nk):
        _, L, R = u_matrix(Vk, minus, q)
        out.append(np.einsum("xQ,mQP,Py->mxy", L, Pw[q], R))
    return np.stack(out)
