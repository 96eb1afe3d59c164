"""Oracle (test infrastructure only): the intermediate representation (IR) of
imaginary-time functions with sparse sampling on both axes (Sec. IV.C,
"Representation on the imaginary axes": the paper expands every dynamical
quantity in the IR basis, with a dimensionless cutoff lambda larger than
beta times the bandwidth, and samples it sparsely in tau and in Matsubara
frequency).  Plain numpy; shares no code with the library's builder.

Construction (reading R19 of the design notes):
  * the logistic kernel on x = 2 tau / beta - 1 and y = omega / omega_max in
    [-1, 1], lambda = beta omega_max:
        K(x, y) = exp(-lambda y (x + 1) / 2) / (1 + exp(-lambda y)),
    which is e^{-omega tau} / (1 + e^{-beta omega}) in physical units; it
    serves fermionic and bosonic functions alike (a bosonic spectral
    function enters multiplied by coth(beta omega / 2));
  * its singular-value expansion from an SVD of sqrt(w_x) K sqrt(w_y) on
    composite Gauss-Legendre rules (segments halving towards x = +-1 and
    towards y = 0); L = the number of singular values above eps times the
    largest, rounded up to even;
  * basis functions by the Nystrom extension
        u_l(x) = (1 / s_l) sum_j K(x, y_j) sqrt(w_j) v_{jl},
    so that their Matsubara transforms are closed forms:
        int_0^beta e^{i nu tau} e^{-omega tau} / (1 + e^{-beta omega}) d tau
          = -1 / (i nu - omega)                 (fermionic nu)
          = -tanh(beta omega / 2) / (i nu - omega)  (bosonic nu);
  * tau sampling points: the L roots of u_L, the first function left out
    (mirrored pairs, so tau_{L-1-i} = beta - tau_i);
  * Matsubara sampling points: symmetric pairs ({n, -n-1} fermionic; {0},
    {m, -m} bosonic) chosen greedily among |n| < 4 lambda / pi + 4 L: each
    time the pair whose rows of the transform matrix (columns scaled to unit
    norm over the candidates) keep the largest residual after the rows
    already chosen are projected out; L fermionic and L + 1 bosonic points;
  * tables: T = Uhat U(tau)^{-1}, Tp = U(tau) Uhat^+, and the density row
    w = u(beta) U(tau)^{-1} (the value at tau = beta^-).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss

NODES_PER_SEGMENT = 16


def logistic_kernel(x, y, lam):
    """K(x, y) for arrays x (rows) and y (columns), without overflow."""
    x = np.asarray(x, np.float64)[:, None]
    y = np.asarray(y, np.float64)[None, :]
    expo = np.where(y >= 0.0, -0.5 * lam * y * (x + 1.0), 0.5 * lam * y * (1.0 - x))
    return np.exp(expo) / (1.0 + np.exp(-lam * np.abs(y)))


def segments(lam):
    """Breakpoints of the composite rules: x halves towards both ends, y halves
    towards 0, down to a width below 1 / lam."""
    m = int(np.ceil(np.log2(lam))) + 2
    xs = [0.0] + [1.0 - 2.0 ** -j for j in range(1, m)] + [1.0]
    ys = [0.0] + [2.0 ** -j for j in range(m)]
    bx = np.array(sorted(set([-v for v in xs] + xs)))
    by = np.array(sorted(set([-v for v in ys] + ys)))
    return bx, by


def composite_gauss_legendre(breaks, npts):
    t, w = leggauss(npts)
    x = np.concatenate([0.5 * (b - a) * t + 0.5 * (b + a) for a, b in zip(breaks[:-1], breaks[1:])])
    ww = np.concatenate([0.5 * (b - a) * w for a, b in zip(breaks[:-1], breaks[1:])])
    return x, ww


class Basis:
    """Singular-value expansion of the logistic kernel for (lam, eps)."""

    def __init__(self, lam, eps):
        self.lam, self.eps = float(lam), float(eps)
        bx, by = segments(self.lam)
        self.breaks_x = bx
        x, wx = composite_gauss_legendre(bx, NODES_PER_SEGMENT)
        y, wy = composite_gauss_legendre(by, NODES_PER_SEGMENT)
        A = np.sqrt(wx)[:, None] * logistic_kernel(x, y, self.lam) * np.sqrt(wy)[None, :]
        _, s, vt = np.linalg.svd(A, full_matrices=False)
        L = int(np.sum(s / s[0] > self.eps))
        L += L % 2
        self.L = L
        self.s = s
        self.y = y
        # Nystrom coefficients of u_0 .. u_L (u_L gives the tau sampling points)
        self.coef = np.sqrt(wy)[:, None] * vt[:L + 1].T / s[None, :L + 1]

    def u(self, x, cols=None):
        """u_l(x) for l in cols (default 0 .. L-1), shape (len(x), ncols)."""
        c = self.coef[:, :self.L] if cols is None else self.coef[:, cols]
        return logistic_kernel(np.atleast_1d(x), self.y, self.lam) @ c

    def uhat(self, nu, beta, stat):
        """int_0^beta e^{i nu tau} u_l(2 tau / beta - 1) d tau for l < L (closed
        form of the Nystrom sum); stat 'F' or 'B'."""
        om = self.y * (self.lam / beta)
        z = 1j * np.asarray(nu, np.float64)[:, None] - om[None, :]
        f = -1.0 / z if stat == "F" else -np.tanh(0.5 * beta * om)[None, :] / z
        return f @ self.coef[:, :self.L]


def sampling_tau(basis):
    """Roots of u_L in (0, 1) by sign changes on a fine composite grid and
    bisection, mirrored to (-1, 0)."""
    g, _ = composite_gauss_legendre(basis.breaks_x, 64)
    g = np.unique(np.concatenate([g, basis.breaks_x]))
    g = g[g > 0.0]
    f = basis.u(g, [basis.L])[:, 0]
    roots = []
    for i in np.nonzero(np.sign(f[:-1]) * np.sign(f[1:]) < 0)[0]:
        a, b, fa = g[i], g[i + 1], f[i]
        for _ in range(64):
            m = 0.5 * (a + b)
            fm = basis.u([m], [basis.L])[0, 0]
            if np.sign(fm) == np.sign(fa):
                a, fa = m, fm
            else:
                b = m
        roots.append(0.5 * (a + b))
    pos = np.sort(np.array(roots))
    if 2 * len(pos) != basis.L:
        raise RuntimeError(f"found {2 * len(pos)} roots of u_L, expected {basis.L}")
    return np.concatenate([-pos[::-1], pos])


def sampling_matsubara(basis, beta, stat, count):
    """Greedy symmetric selection of `count` Matsubara indices (see module doc)."""
    N = int(np.ceil(4.0 * basis.lam / np.pi)) + 4 * basis.L
    idx = np.arange(-N, N)
    nu = (2 * idx + 1) * np.pi / beta if stat == "F" else 2 * idx * np.pi / beta
    M = basis.uhat(nu, beta, stat)
    M = M / np.linalg.norm(M, axis=0)[None, :]
    pos = {int(n): i for i, n in enumerate(idx)}
    if stat == "F":
        groups = [(n, -n - 1) for n in range(N)]
    else:
        groups = [(0,)] + [(m, -m) for m in range(1, N)]
    R = M.copy()                      # rows with the chosen directions projected out
    chosen = []
    while len(chosen) < count:
        norms = [np.sqrt(sum(np.linalg.norm(R[pos[n]]) ** 2 for n in g)) for g in groups]
        g = groups.pop(int(np.argmax(norms)))
        for n in g:
            q = R[pos[n]] / np.linalg.norm(R[pos[n]])
            R = R - np.outer(R @ q.conj(), q)
            chosen.append(n)
    return np.array(sorted(chosen), np.int64)


class IRGrids:
    """Sparse-sampling tables of the IR basis for (beta, lam, eps), with the
    attributes of oracle.grids.Grids: tau, x, nF, nB, wF, wB, TF, TB, TFp,
    TBp, w (ntau = L, nw_f = L, nw_b = L + 1)."""

    def __init__(self, beta, lam, eps):
        self.beta = float(beta)
        self.basis = b = Basis(lam, eps)
        self.ntau = L = b.L
        self.x = sampling_tau(b)
        self.tau = 0.5 * self.beta * (self.x + 1.0)
        self.nF = sampling_matsubara(b, self.beta, "F", L)
        self.nB = sampling_matsubara(b, self.beta, "B", L + 1)
        self.wF = (2 * self.nF + 1) * np.pi / self.beta
        self.wB = 2 * self.nB * np.pi / self.beta
        Ut = b.u(self.x)                              # (ntau, L)
        Uinv = np.linalg.inv(Ut)
        UhF = b.uhat(self.wF, self.beta, "F")
        UhB = b.uhat(self.wB, self.beta, "B")
        self.TF = UhF @ Uinv
        self.TB = UhB @ Uinv
        self.TFp = Ut @ np.linalg.pinv(UhF)
        self.TBp = Ut @ np.linalg.pinv(UhB)
        self.w = (b.u([1.0]) @ Uinv)[0]
