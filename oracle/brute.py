"""Oracle (test infrastructure only): literal index loops for tiny inputs.

Every sum of Eqs. HF_J, HF_K, tilde_P0_tau (reading R1) and tilde_sigma2 is
written as nested Python loops over each index, with no matrix products, so
that a transposed operand or a dropped conjugate in the vectorised oracle
shows up against these.  Meant for Nk <= 8, nao <= 3, naux <= 4, ntau <= 6.
"""
from __future__ import annotations

import numpy as np

from .gw import mesh_tables


def _vkk(V, plus, k1, k2, Q, i, j):
    """V^{k1,k2}_{ij}(Q) from the q-major storage V[q][k][Q] = V^{k,k+q}(Q)."""
    nk = V.shape[0]
    for q in range(nk):
        if plus[q, k1] == k2:
            return V[q, k1, Q, i, j]
    raise KeyError


def polarization(V, G, mesh, ns):
    plus, _ = mesh_tables(mesh)
    ntau, nk, n, _ = G.shape
    naux = V.shape[2]
    P = np.zeros((nk, ntau, naux, naux), np.complex128)
    for q in range(nk):
        for t in range(ntau):
            for Q in range(naux):
                for Qp in range(naux):
                    acc = 0j
                    for k in range(nk):
                        kq = plus[q, k]
                        for a in range(n):
                            for b in range(n):
                                for c in range(n):
                                    for d in range(n):
                                        acc += (_vkk(V, plus, k, kq, Q, d, a)
                                                * G[ntau - 1 - t, k, c, d]
                                                * G[t, kq, a, b]
                                                * _vkk(V, plus, kq, k, Qp, b, c))
                    P[q, t, Q, Qp] = -ns / nk * acc
    return P


def self_energy(V, G, Pt, mesh):
    plus, minus = mesh_tables(mesh)
    ntau, nk, n, _ = G.shape
    naux = V.shape[2]
    S = np.zeros_like(G)
    for t in range(ntau):
        for k in range(nk):
            for i in range(n):
                for j in range(n):
                    acc = 0j
                    for q in range(nk):
                        kq = minus[q, k]
                        for a in range(n):
                            for b in range(n):
                                for Q in range(naux):
                                    for Qp in range(naux):
                                        acc += (G[t, kq, a, b] * _vkk(V, plus, k, kq, Q, i, a)
                                                * Pt[q, t, Q, Qp] * _vkk(V, plus, kq, k, Qp, b, j))
                    S[t, k, i, j] = -acc / nk
    return S


def hartree_fock(V, gamma, mesh, ns):
    plus, _ = mesh_tables(mesh)
    nk, n, _ = gamma.shape
    naux = V.shape[2]
    out = np.zeros_like(gamma)
    for k in range(nk):
        for i in range(n):
            for j in range(n):
                acc = 0j
                for kp in range(nk):
                    for a in range(n):
                        for b in range(n):
                            for Q in range(naux):
                                # Hartree: ns from the spin sum sigma_1
                                acc += ns * _vkk(V, plus, k, k, Q, i, j) * gamma[kp, a, b] \
                                    * _vkk(V, plus, kp, kp, Q, b, a)
                                # exchange
                                acc -= _vkk(V, plus, k, kp, Q, i, a) * gamma[kp, a, b] \
                                    * _vkk(V, plus, kp, k, Q, b, j)
                out[k, i, j] = acc / nk
    return out
