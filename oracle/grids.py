"""Oracle (test infrastructure only): imaginary-time and Matsubara grids.

Plain, slow, obviously correct fp64 construction of the discretisation used
by the GW equations of the paper.  It is imported only by tests, by the
smoke check and by the CPU-baseline timing; the product path never runs it.

The paper expands dynamical quantities in the IR basis with sparse sampling
(Sec. IV.C).  That package is not used; tau is sampled at
Chebyshev roots instead, and a sparse Matsubara set is picked greedily.  Readings
taken (each also listed in the design notes):

* tau nodes: roots of T_n on [-1,1] mapped to [0, beta], mirrored so that
  tau_{n-1-i} = beta - tau_i; a function on [0, beta] is represented by its
  degree-(n-1) Chebyshev interpolant through these nodes.
* Fourier pair Eqs. tau_to_iw / iw_to_tau: the forward transform of the
  interpolant is exact up to quadrature (Gauss-Legendre with enough points to
  resolve exp(i nu tau)); the inverse is the least-squares fit (pseudo-inverse).
* Matsubara frequencies: fermionic omega_n = (2n+1) pi / beta, bosonic
  Omega_m = 2 m pi / beta (Sec. III, Eqs. tau_to_iw and tilde_W_DF).
* sparse sets: symmetric pairs {n, -n-1} (fermionic, ntau points) or {0} and
  {m, -m} (bosonic, ntau+1 points), chosen one pair at a time, each time the
  pair whose transform rows have the largest residual after projecting out the
  rows already chosen, among 0 <= n < 4 ntau (ties: smallest n).
* density matrix gamma = -G(beta^-) (Sec. III): value of the interpolant at
  tau = beta, i.e. the row w = 1^T C^{-1} since T_l(1) = 1.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import chebyshev as npcheb
from numpy.polynomial import legendre as nplegendre


def tau_nodes(beta: float, ntau: int):
    """Chebyshev roots, ascending; returns (tau, x) with tau = beta (1 + x) / 2."""
    i = np.arange(ntau)
    x = -np.cos((2 * i + 1) * np.pi / (2 * ntau))
    h = ntau // 2
    x[ntau - h:] = -x[:h][::-1]
    if ntau % 2 == 1:
        x[h] = 0.0
    tau = beta * (1.0 + x) / 2.0
    tau[ntau - h:] = beta - tau[:h][::-1]
    return tau, x


def matsubara(indices, beta: float, stat: str):
    """omega_n = (2n+1) pi / beta (stat 'F') or Omega_m = 2 m pi / beta ('B')."""
    n = np.asarray(indices, dtype=np.float64)
    if stat == "F":
        return (2.0 * n + 1.0) * np.pi / beta
    return 2.0 * n * np.pi / beta


def chebyshev_collocation(x, ntau):
    """C_{il} = T_l(x_i)."""
    return npcheb.chebvander(x, ntau - 1)


def fourier_moments(nu, beta: float, ntau: int):
    """M_{nl} = int_0^beta T_l(2 tau / beta - 1) exp(i nu_n tau) d tau (Eq. tau_to_iw
    applied to a Chebyshev polynomial), by Gauss-Legendre quadrature."""
    nu = np.asarray(nu, dtype=np.float64)
    nq = ntau + int(np.ceil(beta * np.max(np.abs(nu)) / 2.0)) + 200
    xg, wg = nplegendre.leggauss(nq)
    tg = beta * (1.0 + xg) / 2.0
    Tv = npcheb.chebvander(xg, ntau - 1)                       # (nq, ntau)
    E = np.exp(1j * np.outer(nu, tg)) * (wg * beta / 2.0)      # (nw, nq)
    return E @ Tv


def transform_matrix(nu, beta: float, ntau: int):
    """T_{ni}: X(i nu_n) = sum_i T_{ni} X(tau_i) for the Chebyshev interpolant."""
    _, x = tau_nodes(beta, ntau)
    C = chebyshev_collocation(x, ntau)
    return fourier_moments(nu, beta, ntau) @ np.linalg.inv(C)


def beta_minus_row(beta: float, ntau: int):
    """w with X(beta^-) = sum_i w_i X(tau_i)."""
    _, x = tau_nodes(beta, ntau)
    C = chebyshev_collocation(x, ntau)
    return np.ones(ntau) @ np.linalg.inv(C)


def select_sparse(beta: float, ntau: int, stat: str):
    """Greedy symmetric sparse Matsubara index set (see module docstring)."""
    if ntau % 2:
        raise ValueError("ntau must be even")
    cand = np.arange(0, 4 * ntau)
    if stat == "F":
        pos, neg = cand, -cand - 1
    else:
        pos, neg = cand, -cand
    Tp = transform_matrix(matsubara(pos, beta, stat), beta, ntau)
    Tn = transform_matrix(matsubara(neg, beta, stat), beta, ntau)
    basis = np.zeros((0, ntau), np.complex128)

    def add_row(basis, r):
        for _ in range(2):
            if len(basis):
                r = r - basis.T @ (basis.conj() @ r)
        return np.vstack([basis, r / np.linalg.norm(r)])

    chosen = []
    if stat == "B":
        basis = add_row(basis, Tp[0])
        chosen.append(0)
    npairs = ntau // 2
    taken = set(chosen)
    for _ in range(npairs):
        res = np.full(len(cand), -1.0)
        for c in cand:
            if c in taken:
                continue
            tot = 0.0
            for r in (Tp[c], Tn[c]):
                rr = r - basis.T @ (basis.conj() @ r) if len(basis) else r
                tot += np.vdot(rr, rr).real / np.vdot(r, r).real
            res[c] = tot
        best = res.max()
        c = int(np.nonzero(res >= best * (1.0 - 1e-9))[0][0])
        taken.add(c)
        chosen.append(c)
        basis = add_row(basis, Tp[c])
        basis = add_row(basis, Tn[c])
    s = np.array(sorted(x for x in chosen if (x > 0 or stat == "F")), dtype=np.int64)
    if stat == "F":
        return np.concatenate([-s[::-1] - 1, s])
    return np.concatenate([-s[::-1], [0], s])


class Grids:
    """All discretisation tables for one (beta, ntau)."""

    def __init__(self, beta: float, ntau: int, nF=None, nB=None):
        self.beta = float(beta)
        self.ntau = int(ntau)
        self.tau, self.x = tau_nodes(beta, ntau)
        self.nF = select_sparse(beta, ntau, "F") if nF is None else np.asarray(nF, np.int64)
        self.nB = select_sparse(beta, ntau, "B") if nB is None else np.asarray(nB, np.int64)
        self.wF = matsubara(self.nF, beta, "F")
        self.wB = matsubara(self.nB, beta, "B")
        self.TF = transform_matrix(self.wF, beta, ntau)
        self.TB = transform_matrix(self.wB, beta, ntau)
        self.TFp = np.linalg.pinv(self.TF)
        self.TBp = np.linalg.pinv(self.TB)
        self.w = beta_minus_row(beta, ntau)
