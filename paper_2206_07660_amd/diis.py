"""DIIS (Pulay extrapolation, Anderson mixing) for the scGW self-consistency.

The paper accelerates its scGW loop with a DIIS scheme for the finite-
temperature Dyson equation (Sec. IV.B).  It prints no formulas for it; the
reading here is Pulay's direct inversion in the iterative subspace on the
same unknown and residual as the Newton-Krylov solver:
    x = (Sigma_inf, Sigma~(tau)),   F(x) = Sigma_GW[G(x)] - x,
with G(x) from the Dyson equation at the chemical potential of the target
electron count (or at a fixed mu with a grand-canonical path, GWPath(fixed_mu=True)).  From the last m pairs (x_i, F_i) the coefficients c minimise
|sum_i c_i F_i|_2 under sum_i c_i = 1, and the next point is
    x_new = sum_i c_i (x_i + a F_i)  (a = 1: x_new = sum_i c_i Sigma_GW[G(x_i)]).
The residuals are Hermitian per (tau, k), so the coefficients are taken real
(the Gram matrix is Re <F_i, F_j>) and every iterate stays Hermitian.

`DIISCore` holds the history and solves the small bordered system on the host;
it works on opaque vectors through `dot`, `axpby` and `new` callables, so the
same logic runs on device buffers (libgw's gw_dot, gw_axpby) and on numpy
arrays.  `DIIS` drives it with Sigma evaluations through libgw.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np


class DIISCore:
    """History of (x_i, F_i) and the Pulay coefficients.

    dot(u, v) -> complex <u, v>;  axpby(a, x, b, y): y <- a x + b y
    (x may be None, then y <- b y);  new() -> an uninitialised vector.
    """

    def __init__(self, dot, axpby, new, depth=6, mixing=1.0, rcond=1e-12):
        if depth < 1:
            raise ValueError("DIIS depth must be at least 1")
        self.dot, self.axpby, self.new = dot, axpby, new
        self.depth, self.mixing, self.rcond = int(depth), float(mixing), float(rcond)
        self.xs, self.fs = [], []
        self.B = np.zeros((0, 0))
        self.last_coefficients = np.zeros(0)

    def __len__(self):
        return len(self.xs)

    def reset(self):
        """Forget the history (the buffers are released)."""
        self.xs, self.fs = [], []
        self.B = np.zeros((0, 0))
        self.last_coefficients = np.zeros(0)

    def push(self, x, f):
        """Append copies of x and F(x); drops the oldest pair beyond depth."""
        if len(self.xs) == self.depth:
            xo, fo = self.xs.pop(0), self.fs.pop(0)
            self.B = self.B[1:, 1:]
        else:
            xo, fo = self.new(), self.new()
        self.axpby(1.0, x, 0.0, xo)
        self.axpby(1.0, f, 0.0, fo)
        row = np.array([self.dot(g, fo).real for g in self.fs])
        n = len(self.fs)
        B = np.zeros((n + 1, n + 1))
        B[:n, :n] = self.B
        B[:n, n] = B[n, :n] = row
        B[n, n] = self.dot(fo, fo).real
        self.xs.append(xo)
        self.fs.append(fo)
        self.B = B

    def coefficients(self):
        """argmin |sum c_i F_i| with sum c_i = 1, from the bordered system
        [[B, 1], [1^T, 0]] [c; l] = [0; 1].  Pairs whose residuals are nearly
        linearly dependent on newer ones are dropped, oldest first, until the
        scaled Gram matrix is well conditioned."""
        while True:
            n = len(self.xs)
            B = self.B
            s = np.sqrt(np.maximum(np.diag(B), np.finfo(float).tiny))
            Bs = B / np.outer(s, s)                      # unit diagonal
            if n == 1 or np.linalg.cond(Bs) < 1.0 / self.rcond:
                break
            self.xs.pop(0)
            self.fs.pop(0)
            self.B = self.B[1:, 1:]
        A = np.zeros((n + 1, n + 1))
        A[:n, :n] = Bs
        A[:n, n] = A[n, :n] = 1.0 / s                    # the constraint on c = cs / s
        rhs = np.zeros(n + 1)
        rhs[n] = 1.0
        cs = np.linalg.solve(A, rhs)[:n]
        c = cs / s
        self.last_coefficients = c
        return c

    def extrapolate(self, out):
        """out <- sum_i c_i (x_i + a F_i); returns the coefficients."""
        c = self.coefficients()
        self.axpby(0.0, None, 0.0, out)
        for ci, xi, fi in zip(c, self.xs, self.fs):
            self.axpby(float(ci), xi, 1.0, out)
            self.axpby(float(ci) * self.mixing, fi, 1.0, out)
        return c


@dataclasses.dataclass
class DIISStats:
    iterations: int = 0
    evaluations: int = 0
    residuals: list = dataclasses.field(default_factory=list)


class DIIS:
    """DIIS solve of the scGW self-consistency on the GPU (all vector arithmetic
    in libgw).  The first `start_damped` iterations are plain damped steps
    x <- x + alpha F (alpha of the path), which fill the history.
    mu_window > 0: mu is the midpoint of the interval where the electron count
    is within mu_window of the target (gw_set_mu_window) instead of the root,
    which in a gapped system at low temperature is set by the grids'
    representation error of the count."""

    def __init__(self, path, depth=6, mixing=1.0, start_damped=1, mu_window=0.0):
        import torch
        from . import gw
        self.gw, self.torch = gw, torch
        self.path, self.ctx = path, path.ctx
        c = self.ctx
        self.n_inf = c.nk * c.nao * c.nao
        self.N = self.n_inf + c.ntau * self.n_inf
        z = dict(dtype=torch.complex128, device="cuda")
        self.G_iw = torch.empty(c.giw_shape(), **z)
        self.G_tau = torch.empty(c.g_shape(), **z)
        self.sig_iw = torch.empty(c.giw_shape(), **z)
        self.mu, self.n_e = 0.0, 0.0
        self.start_damped = int(start_damped)
        self.mu_window = float(mu_window)
        self.core = DIISCore(lambda u, v: gw.gw_dot(c, u, v),
                             lambda a, x, b, y: gw.gw_axpby(c, a, x, b, y),
                             self.vec, depth=depth, mixing=mixing)
        self.stats = DIISStats()

    def vec(self):
        return self.torch.empty(self.N, dtype=self.torch.complex128, device="cuda")

    def inf(self, v):
        return v[: self.n_inf].view(self.ctx.k_shape())

    def tau(self, v):
        return v[self.n_inf:].view(self.ctx.g_shape())

    def residual(self, x, F):
        """F = Sigma_GW[G(x)] - x (mu searched for the target N_e)."""
        gw, c, p = self.gw, self.ctx, self.path
        gw.gw_tau_to_iw(c, gw.GW_FERMION, self.tau(x), self.sig_iw)
        self.mu, self.n_e = p.green(self.inf(x), self.sig_iw, self.mu, self.G_iw, self.G_tau)
        p.sigma(self.G_tau, self.inf(F), self.tau(F))
        self.stats.evaluations += 1
        gw.gw_axpby(c, -1.0, x, 1.0, F)

    def solve(self, sig_inf, sig_tau, mu0, tol=1e-8, max_iter=100, log=None, deadline=None):
        """DIIS from (sig_inf, sig_tau) until max |F| < tol; returns (x, F).
        deadline: a time.perf_counter() value after which no further
        iteration is started (the last residual is returned)."""
        gw, c = self.gw, self.ctx
        self.mu = mu0
        self.core.reset()                     # a new solve starts without history
        x, F = self.vec(), self.vec()
        gw.gw_axpby(c, 1.0, sig_inf, 0.0, self.inf(x))
        gw.gw_axpby(c, 1.0, sig_tau, 0.0, self.tau(x))
        gw.gw_set_mu_window(c, self.mu_window)
        try:
            self._iterate(x, F, tol, max_iter, log, deadline)
        finally:
            gw.gw_set_mu_window(c, 0.0)
        return x, F

    def _iterate(self, x, F, tol, max_iter, log, deadline):
        gw, c = self.gw, self.ctx
        for it in range(max_iter + 1):
            self.residual(x, F)
            res = gw.gw_mix(c, 0.0, None, F, want_diff=True)          # max |F|
            self.stats.residuals.append(res)
            if log:
                log(f"[diis] iteration {it}: max|F| {res:.3e} mu {self.mu:.10f} "
                    f"history {len(self.core)}")
            if res < tol or it == max_iter:
                break
            if deadline is not None and time.perf_counter() > deadline:
                if log:
                    log("[diis] wall-clock budget reached")
                break
            self.core.push(x, F)
            if it < self.start_damped:
                gw.gw_axpby(c, self.path.alpha, F, 1.0, x)
            else:
                self.core.extrapolate(x)
                # drop the round-off part that is not Hermitian
                gw.gw_hermitize(c, self.tau(x), c.nao)
                gw.gw_hermitize(c, self.inf(x), c.nao)
            self.stats.iterations += 1
