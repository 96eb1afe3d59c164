"""Oracle (test infrastructure only): the Sigma[G] evaluation as plain
PyTorch CPU complex128 operations, so that autograd supplies reference
vector-Jacobian and Jacobian-vector products of G -> (Sigma_inf, Sigma~).

Same equations and readings as oracle/gw.py (Eqs. HF_J, HF_K, tilde_P0_tau
with reading R1, P0t_to_P0w, tilde_P_omega, Piw_to_Pt, tilde_sigma2); the
grid tables are passed in.  Complex gradients follow torch's convention
(for a real loss L, grad z = dL/dx + i dL/dy), i.e. the VJP of a holomorphic
map is the conjugate-transposed Jacobian applied to the cotangent.
"""
from __future__ import annotations

import numpy as np
import torch

from .gw import mesh_tables


def sigma_evaluation(V, G, TB, TBp, w, mesh, ns):
    """V [q][k][Q][i][j], G [tau][k][i][j] (torch complex128); TB, TBp, w
    torch tensors.  Returns (Sigma_inf [k][i][j], Sigma~ [tau][k][i][j])."""
    plus, minus = mesh_tables(mesh)
    nt, nk = G.shape[:2]
    naux = V.shape[2]
    # density matrix and Hartree-Fock
    gamma = -torch.einsum("t,tkij->kij", w.to(G.dtype), G)
    vQ = ns / nk * torch.einsum("kab,kQba->Q", gamma, V[0])
    sig_inf = torch.einsum("Q,kQij->kij", vQ, V[0])
    for q in range(nk):
        kq = torch.as_tensor(plus[q])
        sig_inf = sig_inf - 1.0 / nk * torch.einsum("kQia,kab,kQjb->kij", V[q], gamma[kq], V[q].conj())
    # polarization for all q and tau
    rev = torch.arange(nt - 1, -1, -1)
    P0 = []
    for q in range(nk):
        kq = torch.as_tensor(plus[q])
        X = torch.einsum("kQda,tkab->tkQdb", V[q], G[:, kq])
        Z = torch.einsum("kPcb,tkcd->tkPbd", V[q].conj(), G[rev])
        P0.append(-ns / nk * torch.einsum("tkQdb,tkPbd->tQP", X, Z))
    P0 = torch.stack(P0)
    P0w = torch.einsum("mt,qtQP->qmQP", TB, P0)
    eye = torch.eye(naux, dtype=G.dtype)
    Pw = torch.linalg.solve(eye - P0w, P0w)
    Pt = torch.einsum("tm,qmQP->qtQP", TBp, Pw)
    # self-energy
    sig = torch.zeros_like(G)
    for q in range(nk):
        kk = torch.as_tensor(minus[q])
        A = V[q][kk]                                     # A[k] = V^{k-q,k}
        B = torch.einsum("tQP,kPbj->tkQbj", Pt[q], A)
        sig = sig - 1.0 / nk * torch.einsum("kQai,tkab,tkQbj->tkij", A.conj(), G[:, kk], B)
    return sig_inf, sig


def tensors(V, grids):
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x))
    return t(V), t(grids.TB), t(grids.TBp), t(grids.w)


def vjp(V, G, Sinf_bar, Sig_bar, grids, mesh, ns):
    """G_bar = J^H (Sinf_bar, Sig_bar) by reverse-mode autograd (numpy in/out)."""
    Vt, TB, TBp, w = tensors(V, grids)
    Gt = torch.from_numpy(np.ascontiguousarray(G)).requires_grad_(True)
    si, st = sigma_evaluation(Vt, Gt, TB, TBp, w, mesh, ns)
    torch.autograd.backward([si, st], [torch.from_numpy(Sinf_bar), torch.from_numpy(Sig_bar)])
    return Gt.grad.numpy()


def jvp(V, G, dG, grids, mesh, ns):
    """(dSinf, dSig) = J dG by forward-mode autograd (numpy in/out)."""
    Vt, TB, TBp, w = tensors(V, grids)
    f = lambda g: sigma_evaluation(Vt, g, TB, TBp, w, mesh, ns)
    _, (di, ds) = torch.func.jvp(f, (torch.from_numpy(G),), (torch.from_numpy(dG),))
    return di.numpy(), ds.numpy()
