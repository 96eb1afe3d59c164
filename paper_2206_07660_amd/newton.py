"""Newton-Krylov solve of the scGW self-consistency on the GPU.

The unknown is x = (Sigma_inf, Sigma~(tau)) and the residual is
    F(x) = Sigma_GW[G(x)] - x,
where G(x) solves the Dyson equation (Eq. Dyson) at the chemical potential
that gives the target electron count (Sec. IV.A) or, with a grand-canonical
path (GWPath(fixed_mu=True)), at a fixed mu, and Sigma_GW is the
Hartree-Fock + dynamical GW self-energy (Eqs. HF_J, HF_K, tilde_sigma2).
Each Newton step solves J_F(x) d = -F(x) with restarted GMRES; a Jacobian-
vector product is the Dyson JVP (with the mu shift that keeps N_e fixed)
followed by the hand-written JVP of Sigma_GW, so it costs about two Sigma
evaluations.  Vector arithmetic runs through libgw (gw_axpby, gw_dot); only
the small Hessenberg least-squares problem of GMRES is solved on the host.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import torch

from . import gw
from .adjoint import SigmaDerivatives


@dataclasses.dataclass
class NKStats:
    newton_steps: int = 0
    backtracks: int = 0
    mu_fallback: bool = False
    jvps: int = 0
    evaluations: int = 0
    residuals: list = dataclasses.field(default_factory=list)


class NewtonKrylov:
    def __init__(self, path, restart=20, gmres_rtol=1e-6, max_restarts=10, per_q=False, log=None,
                 fixed_mu_jvp=False):
        self.log = log            # optional progress callback, one line per JVP
        # fixed_mu_jvp: leave out the mu shift of the Dyson JVP.  In a gapped
        # system at low temperature N_e hardly depends on mu inside the gap,
        # so the shift that keeps N_e fixed is a ratio of two exponentially
        # small numbers, while G itself hardly depends on mu there either.
        self.fixed_mu_jvp = fixed_mu_jvp or getattr(path, "fixed_mu", False)
        self.last_dmu = 0.0
        self.path = path
        self.ctx = path.ctx
        self.der = SigmaDerivatives(path, per_q=per_q)
        c = self.ctx
        self.n_inf = c.nk * c.nao * c.nao
        self.N = self.n_inf + c.ntau * self.n_inf
        self.restart, self.gmres_rtol, self.max_restarts = restart, gmres_rtol, max_restarts
        z = dict(dtype=torch.complex128, device="cuda")
        self.G_iw = torch.empty(c.giw_shape(), **z)
        self.G_tau = torch.empty(c.g_shape(), **z)
        self.sig_iw = torch.empty(c.giw_shape(), **z)
        self.dG_iw = torch.empty(c.giw_shape(), **z)
        self.dG_tau = torch.empty(c.g_shape(), **z)
        self.mu = 0.0
        self.stats = NKStats()

    # views of a flat state vector
    def inf(self, v):
        return v[: self.n_inf].view(self.ctx.k_shape())

    def tau(self, v):
        return v[self.n_inf:].view(self.ctx.g_shape())

    def vec(self):
        return torch.empty(self.N, dtype=torch.complex128, device="cuda")

    def copy(self, dst, src):
        gw.gw_axpby(self.ctx, 1.0, src, 0.0, dst)

    def pack(self, s_inf, s_tau, out):
        self.copy(self.inf(out), s_inf)
        self.copy(self.tau(out), s_tau)

    def residual(self, x, F):
        """F = Sigma_GW[G(x)] - x; keeps G(x) and P~ of G(x) for the JVPs."""
        c, p = self.ctx, self.path
        gw.gw_tau_to_iw(c, gw.GW_FERMION, self.tau(x), self.sig_iw)
        self.mu, _ = p.green(self.inf(x), self.sig_iw, self.mu, self.G_iw, self.G_tau)
        s_inf, s_tau, self.Pt_tau, self.Pt_iw = self.der.forward(self.G_tau)
        self.stats.evaluations += 1
        self.pack(s_inf, s_tau, F)
        gw.gw_axpby(c, -1.0, x, 1.0, F)

    def jac_vec(self, v, out):
        """out = J_F v = dSigma_GW[dG(v)] - v at the last residual point."""
        c, p = self.ctx, self.path
        gw.gw_tau_to_iw(c, gw.GW_FERMION, self.tau(v), self.sig_iw)
        self.last_dmu = gw.gw_dyson_jvp(c, p.S, self.G_iw, self.inf(v), self.sig_iw, self.dG_iw,
                                        fixed_mu=self.fixed_mu_jvp)
        gw.gw_iw_to_tau(c, gw.GW_FERMION, self.dG_iw, self.dG_tau)
        # the Krylov directions are Hermitian up to round-off, and so is dG
        gw.gw_hermitize(c, self.dG_tau, c.nao)
        d_inf, d_tau = self.der.jvp(self.G_tau, self.Pt_tau, self.Pt_iw, self.dG_tau,
                                    hermitian_dG=True)
        self.stats.jvps += 1
        if self.log:
            self.log(f"[nk] JVP {self.stats.jvps} (dmu {self.last_dmu:.3e})")
        self.pack(d_inf, d_tau, out)
        gw.gw_axpby(c, -1.0, v, 1.0, out)

    def gmres(self, b, x):
        """Restarted GMRES(m) for J_F x = b starting from x = 0."""
        c, m = self.ctx, self.restart
        gw.gw_axpby(c, 0.0, None, 0.0, x)
        bnorm = np.sqrt(gw.gw_dot(c, b, b).real)
        if bnorm == 0.0:
            return
        V = [self.vec() for _ in range(m + 1)]
        w = self.vec()
        r = self.vec()
        for restart in range(self.max_restarts):
            # r = b - J x  (x = 0 on the first pass)
            if restart == 0:
                self.copy(r, b)
            else:
                self.jac_vec(x, r)
                gw.gw_axpby(c, 1.0, b, -1.0, r)
            beta = np.sqrt(gw.gw_dot(c, r, r).real)
            if beta <= self.gmres_rtol * bnorm:
                return
            gw.gw_axpby(c, 1.0 / beta, r, 0.0, V[0])
            H = np.zeros((m + 1, m), complex)
            cs, sn = np.zeros(m, complex), np.zeros(m, complex)
            g = np.zeros(m + 1, complex)
            g[0] = beta
            j_used = 0
            for j in range(m):
                self.jac_vec(V[j], w)
                for i in range(j + 1):                       # modified Gram-Schmidt
                    H[i, j] = gw.gw_dot(c, V[i], w)
                    gw.gw_axpby(c, -H[i, j], V[i], 1.0, w)
                H[j + 1, j] = np.sqrt(gw.gw_dot(c, w, w).real)
                if H[j + 1, j] != 0.0:
                    gw.gw_axpby(c, 1.0 / H[j + 1, j], w, 0.0, V[j + 1])
                for i in range(j):                           # apply earlier rotations
                    t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                    H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + np.conj(cs[i]) * H[i + 1, j]
                    H[i, j] = t
                den = np.sqrt(abs(H[j, j]) ** 2 + abs(H[j + 1, j]) ** 2)
                # complex Givens: [[c, s], [-conj(s), conj(c)]] maps (a, b) to (|(a, b)|, 0)
                cs[j], sn[j] = (np.conj(H[j, j]) / den, np.conj(H[j + 1, j]) / den) if den else (1.0, 0.0)
                H[j, j] = den
                H[j + 1, j] = 0.0
                g[j + 1] = -np.conj(sn[j]) * g[j]
                g[j] = cs[j] * g[j]
                j_used = j + 1
                if abs(g[j + 1]) <= self.gmres_rtol * bnorm:
                    break
            y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
            for i in range(j_used):
                gw.gw_axpby(c, y[i], V[i], 1.0, x)
            if abs(g[j_used]) <= self.gmres_rtol * bnorm:
                return

    def solve(self, sig_inf, sig_tau, mu0, tol=1e-8, max_steps=20, log=None, forcing=None,
              max_backtracks=3, deadline=None):
        """Newton-Krylov from (sig_inf, sig_tau); returns (x, F) flat vectors.

        forcing: None keeps the GMRES relative tolerance fixed; "ew" uses the
        Eisenstat-Walker choice 2 forcing term eta_k = 0.9 (|F_k| / |F_{k-1}|)^2
        (2-norms), safeguarded by 0.9 eta_{k-1}^2 and clipped to [gmres_rtol, 0.5],
        so that early steps are solved loosely and late ones tightly.

        A step that raises max |F| is halved (up to max_backtracks times, one
        residual evaluation each) before the next Newton step is taken.  If
        no halving helps, the solve returns to the previous point and, the
        first time, continues with the mu shift left out of the JVP (see
        fixed_mu_jvp); a second failure ends the solve there.
        deadline: a time.perf_counter() value after which no further Newton
        step is started (the last residual is returned)."""
        c = self.ctx
        self.mu = mu0
        x, F, d = self.vec(), self.vec(), self.vec()
        self.pack(sig_inf, sig_tau, x)
        rtol0 = self.gmres_rtol
        eta, fn_prev = 0.5, None
        res_prev, lam, nback = None, 1.0, 0
        try:
            for it in range(max_steps + 1):
                self.residual(x, F)
                res = gw.gw_mix(c, 0.0, None, F, want_diff=True)      # max |F|
                if log:
                    log(f"[nk] step {it}: max|F| {res:.3e} mu {self.mu:.10f} jvps {self.stats.jvps}"
                        + (f" (step x {lam:g})" if lam != 1.0 else ""))
                if res_prev is not None and res > res_prev:
                    if nback < max_backtracks:
                        lam *= 0.5                                # x = x_old + lam d
                        gw.gw_axpby(c, -lam, d, 1.0, x)
                        nback += 1
                        self.stats.backtracks += 1
                        continue
                    gw.gw_axpby(c, -lam, d, 1.0, x)               # back to x_old
                    if self.fixed_mu_jvp:
                        if log:
                            log("[nk] no descent along the Newton step; stopping at the previous point")
                        self.residual(x, F)
                        break
                    if log:
                        log("[nk] no descent along the Newton step; continuing with the mu shift "
                            "left out of the JVP")
                    self.fixed_mu_jvp = True
                    self.stats.mu_fallback = True
                    res_prev, lam, nback = None, 1.0, 0
                    continue
                self.stats.residuals.append(res)
                res_prev, lam, nback = res, 1.0, 0
                if res < tol or it == max_steps:
                    break
                if deadline is not None and time.perf_counter() > deadline:
                    if log:
                        log("[nk] wall-clock budget reached")
                    break
                if forcing == "ew":
                    fn = float(np.sqrt(gw.gw_dot(c, F, F).real))
                    if fn_prev is not None:
                        e = 0.9 * (fn / fn_prev) ** 2
                        safe = 0.9 * eta * eta
                        eta = max(e, safe) if safe > 0.1 else e
                    eta = min(max(eta, rtol0), 0.5)
                    fn_prev = fn
                    self.gmres_rtol = eta
                gw.gw_axpby(c, -1.0, F, 0.0, F)                  # right-hand side -F
                self.gmres(F, d)
                # the Newton step of a Hermitian residual is Hermitian; drop the
                # round-off part that is not, which the Hermitian-mode forward
                # and the real-differentiable mu constraint would not follow
                gw.gw_hermitize(c, d, c.nao)
                gw.gw_axpby(c, 1.0, d, 1.0, x)
                self.stats.newton_steps += 1
        finally:
            self.gmres_rtol = rtol0
        return x, F
