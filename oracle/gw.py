"""Oracle (test infrastructure only): plain fp64 CPU form of the GW hot path.

Each function writes out one equation of the paper (Yeh, Iskakov, Zgid, Gull,
"Fully self-consistent finite-temperature GW in Gaussian Bloch orbitals for
solids") with explicit loops over q, k and tau and numpy matmul/einsum/solve
inside.  It is imported only by tests, by the smoke check and by the CPU
baseline timing; the product path never runs it, and it shares no code with
the HIP library.

Layouts (complex128, row-major):
  G, Sigma~      [tau][k][i][j]
  V              [q][k][Q][i][j]  = V^{k, k+q}_{ij}(Q)
  P0, P (tau)    [q][tau][Q][Q']
  H0, S, gamma   [k][i][j]

Readings of the paper used here (also listed in the design notes):
  R1  Eq. tilde_P0_tau: G(-tau) of the bosonic bubble is G(beta - tau) on the
      stored [0, beta] grid with the overall sign fixed so that the bubble
      screens: P0(tau) = -(ns/Nk) sum_k tr[V G^{k+q}(tau) V' G^k(beta - tau)].
  R3  spin-restricted: ns = 2 multiplies P0, the Hartree term and N_e; the
      exchange term and Sigma~ carry no spin sum.
  R5  the "unitary matrix" of Eq. tilde_P_omega is the identity.
  R6  P~ is computed as solve(I - P0, P0), never by summing the series.
  R9  mu: bisection on N_e(mu) = N_target, bracket expanded from mu0 +/- 1,
      stopped when the bracket is below 1e-13 Ha.
  R10 scGW: damped fixed point Sigma <- (1 - a) Sigma + a Sigma[G], a = 0.5,
      on both the static and the dynamic part; G_0 from H0 at the mu that
      gives N_target.
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- mesh ------
def mesh_tables(mesh):
    """plus[q, k] = k + q, minus[q, k] = k - q on the Gamma-centred mesh."""
    n1, n2, n3 = mesh
    idx = np.array([(a, b, c) for a in range(n1) for b in range(n2) for c in range(n3)])

    def flat(p):
        return ((p[..., 0] % n1) * n2 + p[..., 1] % n2) * n3 + p[..., 2] % n3

    plus = flat(idx[:, None, :] + idx[None, :, :])
    minus = flat(idx[None, :, :] - idx[:, None, :])
    return plus, minus


# ------------------------------------------------ non-interacting G (Eq. G) --
def fermi_tau(xi, tau, beta):
    """g(xi, tau) = -exp(-xi tau) / (1 + exp(-beta xi)), evaluated without overflow."""
    xi = np.broadcast_to(np.asarray(xi, np.float64)[None, :], (len(tau), len(xi)))
    tau = np.broadcast_to(np.asarray(tau, np.float64)[:, None], xi.shape)
    expo = np.where(xi >= 0, -xi * tau, xi * (beta - tau))      # never positive
    return -np.exp(expo) / (1.0 + np.exp(-beta * np.abs(xi)))


def g0_tau(H0, S, mu, beta, tau):
    """G0^k(tau) of the one-body Hamiltonian (Eqs. G and Dyson with Sigma = 0).

    With H0 C = S C eps and C^dagger S C = I, G0(i w) = C (i w + mu - eps)^{-1} C^dagger,
    so G0(tau) = C diag(g(eps - mu, tau)) C^dagger."""
    nk, n, _ = H0.shape
    out = np.empty((len(tau), nk, n, n), np.complex128)
    for k in range(nk):
        L = np.linalg.cholesky(S[k])
        Li = np.linalg.inv(L)
        e, U = np.linalg.eigh(Li @ H0[k] @ Li.conj().T)
        C = Li.conj().T @ U
        g = fermi_tau(e - mu, tau, beta)                       # (ntau, n)
        out[:, k] = np.einsum("ia,ta,ja->tij", C, g, C.conj())
    return out


# ------------------------------------------------ density, N_e (Sec. III) ----
def density_matrix(G_tau, w):
    """gamma^k = -G^k(beta^-) from the interpolant through the tau nodes."""
    return -np.einsum("t,tkij->kij", w, G_tau)


def electron_count(gamma, S, ns):
    """N_e = (ns / Nk) sum_k tr[gamma^k S^k]."""
    nk = gamma.shape[0]
    return ns / nk * np.einsum("kij,kji->", gamma, S).real


# ---------------------------------------------------- HF (Eqs. HF_J, HF_K) ---
def hartree_fock(V, gamma, mesh, ns):
    """Sigma_inf^k = J^k + K^k, with V^{k,k+q}(Q) = V[q][k][Q] and
    V^{k+q,k}(Q) = V[q][k][Q]^dagger:
    J^k = sum_Q v_Q V^{kk}(Q), v_Q = (ns/Nk) sum_k' tr[gamma^k' V^{k'k'}(Q)];
    K^k = -(1/Nk) sum_q sum_Q V^{k,k+q}(Q) gamma^{k+q} V^{k+q,k}(Q)."""
    plus, _ = mesh_tables(mesh)
    nk, n, _ = gamma.shape
    naux = V.shape[2]
    vQ = np.zeros(naux, np.complex128)
    for kp in range(nk):
        vQ += ns / nk * np.einsum("ab,Qba->Q", gamma[kp], V[0, kp])
    J = np.einsum("Q,kQij->kij", vQ, V[0])
    K = np.zeros_like(gamma)
    for k in range(nk):
        for q in range(nk):
            A = V[q, k]                                             # (Q, i, a)
            T = (A.reshape(naux * n, n) @ gamma[plus[q, k]]).reshape(naux, n, n)   # (Q, i, b)
            Tf = np.swapaxes(T, 0, 1).reshape(n, naux * n)          # (i, (Q b))
            K[k] -= 1.0 / nk * (Tf @ np.swapaxes(np.conj(A), 1, 2).reshape(naux * n, n))
    return J + K


# ------------------------------------------ polarization (Eq. tilde_P0_tau) --
def polarization(V, G_tau, mesh, ns, qs=None, taus=None):
    """P0^q_{QQ'}(tau_i) = -(ns/Nk) sum_k sum_{abcd} V^{k,k+q}_{da}(Q) G^{k+q}_{ab}(tau_i)
    V^{k+q,k}_{bc}(Q') G^k_{cd}(beta - tau_i)  (reading R1).

    Loops over q and tau.  For each k, X(Q) = V^{k,k+q}(Q) G^{k+q}(tau) and
    Z(Q') = V^{k+q,k}(Q') G^k(beta - tau); the sum over (k, d, b) of
    X_{db}(Q) Z_{bd}(Q') is one matmul of X flattened over (k, d, b) with Z
    transposed to (k, d, b)."""
    plus, _ = mesh_tables(mesh)
    ntau, nk, n, _ = G_tau.shape
    naux = V.shape[2]
    qs = list(range(nk)) if qs is None else list(qs)
    taus = list(range(ntau)) if taus is None else list(taus)
    out = np.zeros((len(qs), len(taus), naux, naux), np.complex128)
    for iq, q in enumerate(qs):
        A = V[q].reshape(nk, naux * n, n)                               # (k, (Q d), a)
        Ah = np.conj(np.swapaxes(V[q], 2, 3)).reshape(nk, naux * n, n)  # V^{k+q,k}(Q') as (k, (Q' b), c)
        for it, t in enumerate(taus):
            X = np.matmul(A, G_tau[t, plus[q]]).reshape(nk, naux, n, n)            # (k, Q, d, b)
            Z = np.matmul(Ah, G_tau[ntau - 1 - t]).reshape(nk, naux, n, n)         # (k, Q', b, d)
            Xf = np.swapaxes(X, 0, 1).reshape(naux, nk * n * n)                    # (Q, (k d b))
            Zf = np.swapaxes(np.swapaxes(Z, 2, 3), 0, 1).reshape(naux, nk * n * n)  # (Q', (k d b))
            out[iq, it] = -ns / nk * (Xf @ Zf.T)
    return out


# ------------------------------------- Fourier transforms (Eqs. 9, 10, P0t..) --
def to_iw(T, X_tau):
    """X(i nu_n) = sum_i T_{ni} X(tau_i) on the leading axis."""
    return np.tensordot(T, X_tau, axes=(1, 0))


def to_tau(Tp, X_iw):
    """X(tau_i) = sum_n Tp_{in} X(i nu_n) on the leading axis (least-squares fit)."""
    return np.tensordot(Tp, X_iw, axes=(1, 0))


# --------------------------------------- screened interaction (Eq. tilde_P_omega)
def screened_W(P0_iw):
    """P~(i Omega) = [I - P0(i Omega)]^{-1} P0(i Omega) for every leading index."""
    n = P0_iw.shape[-1]
    flat = P0_iw.reshape(-1, n, n)
    out = np.empty_like(flat)
    eye = np.eye(n)
    for b in range(flat.shape[0]):
        out[b] = np.linalg.solve(eye - flat[b], flat[b])
    return out.reshape(P0_iw.shape)


# ----------------------------------------- self-energy (Eq. tilde_sigma2) ----
def self_energy(V, G_tau, Pt_tau, mesh, qs=None, out=None):
    """Sigma~^k_{ij}(tau) += -(1/Nk) sum_q sum_{ab} sum_{QQ'} G^{k-q}_{ab}(tau)
    V^{k,k-q}_{ia}(Q) P~^q_{QQ'}(tau) V^{k-q,k}_{bj}(Q').

    V^{k-q,k}(Q) = V[q][k-q][Q]; V^{k,k-q}(Q) is its conjugate transpose.
    Pt_tau[iq] belongs to q = qs[iq].  Loops over q and tau; with p = k - q
    running over the slab: B_{bj}(Q) = sum_Q' P~_{QQ'} V^{p,p+q}_{bj}(Q') for
    all p at once (one matmul), L_{ib}(Q) = sum_a V^{p+q,p}_{ia}(Q)
    G^p_{ab}(tau), and Sigma~^{p+q} -= (1/Nk) sum_{Q,b} L_{ib}(Q) B_{bj}(Q)."""
    plus, _ = mesh_tables(mesh)
    ntau, nk, n, _ = G_tau.shape
    naux = V.shape[2]
    qs = range(nk) if qs is None else qs
    out = np.zeros_like(G_tau) if out is None else out
    for iq, q in enumerate(qs):
        Vs = np.swapaxes(V[q], 0, 1).reshape(naux, nk * n * n)          # (Q', (p b j))
        Ac = np.conj(np.swapaxes(V[q], 2, 3)).reshape(nk, naux * n, n)  # V^{p+q,p}(Q) as (p, (Q i), a)
        for t in range(ntau):
            B = (Pt_tau[iq, t] @ Vs).reshape(naux, nk, n, n)                        # (Q, p, b, j)
            L = np.matmul(Ac, G_tau[t]).reshape(nk, naux, n, n)                     # (p, Q, i, b)
            Lf = np.swapaxes(L, 1, 2).reshape(nk, n, naux * n)                      # (p, i, (Q b))
            Bf = np.swapaxes(B, 0, 1).reshape(nk, naux * n, n)                      # (p, (Q b), j)
            out[t, plus[q]] -= 1.0 / nk * np.matmul(Lf, Bf)
    return out


# ---------------------------------------------------- Dyson (Eq. Dyson) ------
def dyson(H0, S, Sig_inf, Sig_iw, mu, wF):
    """G^k(i w_n) = [(i w_n + mu) S^k - H0^k - Sigma_inf^k - Sigma~^k(i w_n)]^{-1}."""
    nw, nk, n, _ = Sig_iw.shape
    G = np.empty(Sig_iw.shape, np.complex128)
    for iw in range(nw):
        for k in range(nk):
            M = (1j * wF[iw] + mu) * S[k] - H0[k] - Sig_inf[k] - Sig_iw[iw, k]
            G[iw, k] = np.linalg.inv(M)
    return G


def count_from_iw(G_iw, S, grids, ns):
    """N_e of G given on the fermionic sparse set."""
    return electron_count(density_matrix(to_tau(grids.TFp, G_iw), grids.w), S, ns)


def find_mu(H0, S, Sig_inf, Sig_iw, n_target, grids, ns, mu0=0.0, tol=1e-13, maxit=400,
            window=0.0):
    """Chemical potential with N_e(mu) = n_target (Sec. IV.A; reading R9).
    window > 0 (Sec. IV.A adjusts mu until the count meets a threshold): mu0
    itself when its count is within w of the target, else the midpoint of
    the interval of mu where it is, i.e. of the roots of N_e = n_target - w
    and n_target + w; w = min(window, n_target / 2, (ns nao - n_target) / 2)."""
    def ne(mu):
        return count_from_iw(dyson(H0, S, Sig_inf, Sig_iw, mu, grids.wF), S, grids, ns)

    def root(target):
        lo, hi = mu0 - 1.0, mu0 + 1.0
        step = 1.0
        while ne(lo) > target:
            step *= 2.0
            lo -= step
        step = 1.0
        while ne(hi) < target:
            step *= 2.0
            hi += step
        it = 0
        while hi - lo > tol and it < maxit:
            mid = 0.5 * (lo + hi)
            if ne(mid) < target:
                lo = mid
            else:
                hi = mid
            it += 1
        return 0.5 * (lo + hi)

    if window > 0.0:
        w = min(window, 0.5 * n_target, 0.5 * (ns * H0.shape[-1] - n_target))
        if abs(ne(mu0) - n_target) <= w:
            mu = mu0
        else:
            mu = 0.5 * (root(n_target - w) + root(n_target + w))
    else:
        mu = root(n_target)
    G_iw = dyson(H0, S, Sig_inf, Sig_iw, mu, grids.wF)
    return mu, G_iw, count_from_iw(G_iw, S, grids, ns)


# ------------------------------------------------ finite-size corrections ---
def finite_size_corrections(S, gamma, G_tau, chi, head):
    """Eq. K_corr: Delta_HF^k = -chi S^k gamma^k S^k, and Eq. GW_head_corr:
    Delta_GW^k(tau_i) = -chi head[i] S^k G^k(tau_i) S^k with head[i] =
    eps^{-1}_{00}(-tau_i) - 1 (Sec. III.D; chi and the dielectric head are
    inputs)."""
    d_hf = np.stack([-chi * S[k] @ gamma[k] @ S[k] for k in range(S.shape[0])])
    d_gw = np.empty_like(G_tau)
    for i in range(G_tau.shape[0]):
        for k in range(S.shape[0]):
            d_gw[i, k] = -chi * head[i] * (S[k] @ G_tau[i, k] @ S[k])
    return d_hf, d_gw


# --------------------------------------------------- Luttinger-Ward part ---
def phi_gw(P0w, grids, nk):
    """Eq. tilde_Phi_GW: (1/(2 Nk)) sum_q (1/beta) sum_n tr{ln[I - P0^q(i W_n)]
    + P0^q(i W_n)} over all bosonic frequencies.  Phi is real and F(-iW) is the
    conjugate of F(iW), so only Re F = ln|det(I - P0)| + Re tr P0 enters.  The
    Matsubara sum (1/beta) sum_n F(iW_n) is the value at tau = 0 of the bosonic
    function whose transform F is; on the sparse set it is read off the
    least-squares fit TBp and the interpolant's value at tau = 0, which by the
    mirrored nodes is the beta^- row reversed: weights Re(w[::-1] @ TBp)."""
    cw = np.real(grids.w[::-1] @ grids.TBp)
    total = 0.0
    for q in range(P0w.shape[0]):
        for n in range(P0w.shape[1]):
            P = P0w[q, n]
            sign, logdet = np.linalg.slogdet(np.eye(P.shape[0]) - P)
            total += cw[n] * (logdet + np.trace(P).real)
    return total / (2.0 * nk)


# ----------------------------------------- one Sigma[G] + Pi evaluation ------
def sigma_evaluation(V, G_tau, grids, mesh, ns):
    """Sigma_inf[G] and Sigma~[G](tau): Eqs. HF_J/HF_K and the chain
    tilde_P0_tau -> P0t_to_P0w -> tilde_P_omega -> Piw_to_Pt -> tilde_sigma2."""
    gamma = density_matrix(G_tau, grids.w)
    sig_inf = hartree_fock(V, gamma, mesh, ns)
    P0 = polarization(V, G_tau, mesh, ns)                   # [q][tau]
    P0w = np.stack([to_iw(grids.TB, P0[q]) for q in range(P0.shape[0])])
    Pw = screened_W(P0w)
    Pt = np.stack([to_tau(grids.TBp, Pw[q]) for q in range(P0.shape[0])])
    sig_tau = self_energy(V, G_tau, Pt, mesh)
    return sig_inf, sig_tau, dict(P0=P0, P0w=P0w, Pw=Pw, Pt=Pt, gamma=gamma)


# ---------------------------------------------- damped scGW (Sec. IV.A) ------
def scgw(H0, S, V, grids, mesh, ns, n_target, n_iter, alpha=0.5, mu0=0.0):
    """Damped fixed-point scGW (reading R10).  Returns the history of
    (mu, Sigma_inf, Sigma~(tau), G(tau)) after each iteration, index 0 = start.
    n_target None keeps mu = mu0 fixed (no search; the grand-canonical
    iteration that thermodynamic derivatives at fixed mu need)."""
    nk, n, _ = H0.shape
    ntau = grids.ntau
    sig_inf = np.zeros((nk, n, n), np.complex128)
    sig_tau = np.zeros((ntau, nk, n, n), np.complex128)
    sig_iw = to_iw(grids.TF, sig_tau)
    if n_target is None:
        mu, G_iw = mu0, dyson(H0, S, sig_inf, sig_iw, mu0, grids.wF)
    else:
        mu, G_iw, _ = find_mu(H0, S, sig_inf, sig_iw, n_target, grids, ns, mu0)
    G_tau = to_tau(grids.TFp, G_iw)
    hist = [(mu, sig_inf.copy(), sig_tau.copy(), G_tau.copy())]
    for _ in range(n_iter):
        s_inf, s_tau, _ = sigma_evaluation(V, G_tau, grids, mesh, ns)
        sig_inf = (1.0 - alpha) * sig_inf + alpha * s_inf
        sig_tau = (1.0 - alpha) * sig_tau + alpha * s_tau
        sig_iw = to_iw(grids.TF, sig_tau)
        if n_target is None:
            G_iw = dyson(H0, S, sig_inf, sig_iw, mu, grids.wF)
        else:
            mu, G_iw, _ = find_mu(H0, S, sig_inf, sig_iw, n_target, grids, ns, mu)
        G_tau = to_tau(grids.TFp, G_iw)
        hist.append((mu, sig_inf.copy(), sig_tau.copy(), G_tau.copy()))
    return hist
