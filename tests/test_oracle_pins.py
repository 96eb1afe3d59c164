"""Pins for the CPU oracle: closed forms, brute force, the four-index route,
invariants.  None of these compares the oracle with itself; each checks it
against something the paper or the mathematics fixes."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2206_07660_amd import inputs as inp
from oracle import brute, fourindex, gw
from oracle import grids as og

NS = 2


def _setup(mesh=(2, 2, 1), nao=2, naux=3, ntau=6, beta=5.0, seed=3, mu=0.1, s_kind="identity"):
    wl = inp.small_workload(mesh=mesh, nao=nao, naux=naux, ntau=ntau, beta=beta, seed=seed,
                            s_kind=s_kind)
    g = og.Grids(beta, ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    G = gw.g0_tau(H0, S, mu, beta, g.tau)
    return wl, g, H0, S, V, G


# ------------------------------------------------------------------ grids ---
def _poly_ft(m, nu, beta):
    """int_0^beta tau^m exp(i nu tau) d tau, m = 0, 1, 2 (closed forms)."""
    if nu == 0.0:
        return beta ** (m + 1) / (m + 1)
    z = 1j * nu
    e = np.exp(z * beta)
    i0 = (e - 1.0) / z
    if m == 0:
        return i0
    i1 = beta * e / z - i0 / z
    if m == 1:
        return i1
    return beta ** 2 * e / z - 2.0 * i1 / z


@pytest.mark.parametrize("beta,ntau", [(50.0, 24), (100.0, 60)])
def test_transform_exact_on_polynomials(beta, ntau):
    g = og.Grids(beta, ntau)
    for T, w in ((g.TF, g.wF), (g.TB, g.wB)):
        for m in range(3):
            got = T @ (g.tau ** m)
            ref = np.array([_poly_ft(m, nu, beta) for nu in w])
            assert np.abs(got - ref).max() <= 1e-12 * beta ** (m + 1)


def test_fermionic_constant_column():
    # int_0^beta exp(i w_n tau) = -2 / (i w_n); bosonic: beta delta_{m0}
    g = og.Grids(50.0, 24)
    assert np.abs(g.TF @ np.ones(24) + 2.0 / (1j * g.wF)).max() < 1e-12 * 50.0
    ref = np.where(g.nB == 0, 50.0, 0.0)
    assert np.abs(g.TB @ np.ones(24) - ref).max() < 1e-11


def test_grid_structure():
    for beta, ntau in [(50.0, 24), (100.0, 60)]:
        g = og.Grids(beta, ntau)
        assert np.abs(g.tau + g.tau[::-1] - beta).max() < 1e-12 * beta
        assert np.all(np.diff(g.tau) > 0)
        assert len(g.nF) == ntau and len(g.nB) == ntau + 1
        assert np.array_equal(g.nF, -g.nF[::-1] - 1)
        assert np.array_equal(g.nB, -g.nB[::-1])
        # least-squares inverse is a left inverse (full column rank)
        assert np.abs(g.TFp @ g.TF - np.eye(ntau)).max() < 1e-10
        assert np.abs(g.TBp @ g.TB - np.eye(ntau)).max() < 1e-10
        # beta^- row reproduces polynomials at tau = beta
        for m in range(4):
            assert abs(g.w @ (g.tau / beta) ** m - 1.0) < 1e-12
        assert np.linalg.cond(g.TF) < 1e4 and np.linalg.cond(g.TB) < 1e4


def test_transform_of_exponential_matches_pole():
    # G(tau) = -exp(-xi tau)/(1+exp(-beta xi)) has G(i w) = 1/(i w - xi)
    beta, ntau = 10.0, 40
    g = og.Grids(beta, ntau)
    for xi in (-0.7, 0.2, 1.3):
        gt = gw.fermi_tau([xi], g.tau, beta)[:, 0]
        assert np.abs(g.TF @ gt - 1.0 / (1j * g.wF - xi)).max() < 1e-12
        assert np.abs(g.TFp @ (1.0 / (1j * g.wF - xi)) - gt).max() < 1e-11


# ------------------------------------------------------------- G0 and N_e ---
@pytest.mark.parametrize("s_kind", ["identity", "random"])
def test_g0_matches_matrix_exponentials(s_kind):
    wl, g, H0, S, V, G = _setup(nao=4, s_kind=s_kind, beta=8.0, ntau=10)
    mu = 0.1
    for k in range(wl.nk):
        Sh = sla.sqrtm(S[k])
        Shi = np.linalg.inv(Sh)
        Hp = Shi @ H0[k] @ Shi - mu * np.eye(wl.nao)
        inv_occ = np.linalg.inv(np.eye(wl.nao) + sla.expm(-wl.beta * Hp))
        for t, tau in enumerate(g.tau):
            ref = -Shi @ sla.expm(-tau * Hp) @ inv_occ @ Shi
            assert np.abs(G[t, k] - ref).max() < 1e-12


def test_noninteracting_electron_count_and_mu():
    wl, g, H0, S, V, G = _setup(nao=4, beta=10.0, ntau=40, mu=0.05)
    eps = np.stack([np.linalg.eigvalsh(H0[k]) for k in range(wl.nk)])

    def n_exact(mu):
        return NS / wl.nk * np.sum(1.0 / (1.0 + np.exp(wl.beta * (eps - mu))))

    ne = gw.electron_count(gw.density_matrix(G, g.w), S, NS)
    assert abs(ne - n_exact(0.05)) < 1e-12
    z = np.zeros((wl.nk, wl.nao, wl.nao), complex)
    zw = np.zeros((wl.ntau, wl.nk, wl.nao, wl.nao), complex)
    target = 3.3
    mu, Giw, n_out = gw.find_mu(H0, S, z, zw, target, g, NS)
    assert abs(n_out - target) <= 1e-9
    assert abs(n_exact(mu) - target) < 1e-9
    # Dyson with Sigma = 0 reproduces the closed-form G0 on the nodes
    G0 = gw.g0_tau(H0, S, mu, wl.beta, g.tau)
    assert np.abs(gw.to_tau(g.TFp, Giw) - G0).max() < 1e-11


def _gapped(nk=2, beta=50.0, ntau=100, seed=9):
    """H0^k = U_k diag(-0.8, -0.6, -0.6, 0.5) U_k^dagger (a 1.1 Ha gap, the
    occupied edge twice degenerate), S = I."""
    rng = np.random.default_rng(seed)
    eps = np.array([-0.8, -0.6, -0.6, 0.5])
    H0 = np.empty((nk, 4, 4), complex)
    for k in range(nk):
        q, r = np.linalg.qr(rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4)))
        H0[k] = (q * eps) @ q.conj().T
    S = np.broadcast_to(np.eye(4, dtype=complex), (nk, 4, 4)).copy()
    return H0, S, eps, og.Grids(beta, ntau)


def test_mu_window_midpoint_noninteracting():
    """window: from a start outside it, mu is the midpoint of the interval where the closed-form count
    (ns/Nk) sum f(eps - mu) is within the window of the target (roots found
    by brentq on the exact Fermi sum).  Mid-gap the exact count differs from
    the target by far less than the grid count's representation error, so
    the root of the grid count is far from the exact root while the window
    midpoint is not."""
    from scipy.optimize import brentq
    beta = 50.0
    H0, S, eps, g = _gapped(beta=beta)
    nk = H0.shape[0]
    z = np.zeros((nk, 4, 4), complex)
    zw = np.zeros((g.wF.size, nk, 4, 4), complex)

    def n_exact(mu):
        return NS * np.sum(1.0 / (1.0 + np.exp(beta * (eps - mu))))

    target, w = 6.0, 1e-6
    lo = brentq(lambda m: n_exact(m) - (target - w), -0.6, 0.5, xtol=1e-15)
    hi = brentq(lambda m: n_exact(m) - (target + w), -0.6, 0.5, xtol=1e-15)
    root = brentq(lambda m: n_exact(m) - target, -0.6, 0.5, xtol=1e-15)
    assert abs(n_exact(0.35) - target) > 1e-4              # a start outside the window
    mu, Giw, n = gw.find_mu(H0, S, z, zw, target, g, NS, 0.35, window=w)
    mu_root, _, _ = gw.find_mu(H0, S, z, zw, target, g, NS, 0.35)
    print("window midpoint", mu, 0.5 * (lo + hi), "root", mu_root, root)
    # the grid count's representation error (about 2e-10 here) moves the
    # window edges by about that over the slope beta * w
    assert abs(mu - 0.5 * (lo + hi)) < 1e-4
    assert abs(mu_root - root) > 100 * abs(mu - 0.5 * (lo + hi))
    assert abs(n - target) <= w
    # a start inside the window is kept as it is
    for mu0 in (0.0, -0.2):
        assert abs(n_exact(mu0) - target) < 1e-7
        assert gw.find_mu(H0, S, z, zw, target, g, NS, mu0, window=w)[0] == mu0


def _s_eigen(H0, S, mu):
    """S-orthonormal eigenvectors C (C^dagger S C = I) and xi = eps - mu per k."""
    out = []
    for k in range(H0.shape[0]):
        e, C = sla.eigh(H0[k], S[k])
        out.append((e - mu, C))
    return out


def test_finite_size_hf_shifts_occupations():
    """Eq. K_corr with gamma = C diag(f) C^dagger (closed form): the generalised
    eigenvalues of (H0 + Delta_HF, S) are eps_a - chi f_a, since
    (H0 - chi S gamma S) C = S C (diag(eps) - chi diag(f))."""
    wl, g, H0, S, V, G = _setup(nao=5, beta=8.0, ntau=10, s_kind="overlap")
    mu, chi = 0.1, 0.37
    gam = np.empty_like(H0)
    want = []
    for k, (xi, C) in enumerate(_s_eigen(H0, S, mu)):
        f = 1.0 / (1.0 + np.exp(wl.beta * xi))
        gam[k] = (C * f) @ C.conj().T
        want.append(np.sort(xi + mu - chi * f))
    d_hf, _ = gw.finite_size_corrections(S, gam, G, chi, np.zeros(wl.ntau))
    for k in range(wl.nk):
        got = sla.eigh(H0[k] + d_hf[k], S[k], eigvals_only=True)
        assert np.abs(np.sort(got) - want[k]).max() < 1e-12


def test_finite_size_head_is_diagonal_in_the_eigenbasis():
    """Eq. GW_head_corr at G = G0 (closed form): C^dagger Delta_GW(tau) C =
    chi head(tau) diag(g_a(tau)), g_a(tau) = exp(-xi_a tau) / (1 + exp(-beta xi_a)),
    because G0 = -C diag(g) C^dagger and C^dagger S C = I."""
    wl, g, H0, S, V, G = _setup(nao=5, beta=8.0, ntau=10, s_kind="overlap")
    mu, chi = 0.1, 0.37
    head = -0.4 * (np.exp(-0.9 * g.tau) + np.exp(-0.9 * (wl.beta - g.tau)))
    _, d_gw = gw.finite_size_corrections(S, np.zeros_like(H0), G, chi, head)
    for k, (xi, C) in enumerate(_s_eigen(H0, S, mu)):
        for i, tau in enumerate(g.tau):
            ga = np.exp(-xi * tau) / (1.0 + np.exp(-wl.beta * xi))
            M = C.conj().T @ d_gw[i, k] @ C
            assert np.abs(M - np.diag(chi * head[i] * ga)).max() < 1e-12


# ------------------------------------------------ brute force (tiny sizes) ---
def test_bruteforce_polarization_selfenergy_hf():
    wl, g, H0, S, V, G = _setup()
    P0 = gw.polarization(V, G, wl.mesh, NS)
    assert np.abs(P0 - brute.polarization(V, G, wl.mesh, NS)).max() < 1e-15
    sinf, stau, d = gw.sigma_evaluation(V, G, g, wl.mesh, NS)
    assert np.abs(stau - brute.self_energy(V, G, d["Pt"], wl.mesh)).max() < 1e-15
    assert np.abs(sinf - brute.hartree_fock(V, d["gamma"], wl.mesh, NS)).max() < 1e-15
    assert np.abs(P0).max() > 1e-3 and np.abs(stau).max() > 1e-4   # not vacuous


def test_bruteforce_general_nonhermitian_G():
    # the index structure must hold for any G, not only Hermitian ones
    wl, g, H0, S, V, G = _setup(mesh=(3, 1, 1))
    rng = np.random.default_rng(9)
    G = G + 0.05 * inp.circular_gaussian(rng, G.shape, 1.0)
    P0 = gw.polarization(V, G, wl.mesh, NS)
    assert np.abs(P0 - brute.polarization(V, G, wl.mesh, NS)).max() < 1e-15
    # Hermiticity of P0 (test_invariants) comes from that of G: it is lost here
    assert np.abs(P0 - np.conj(np.swapaxes(P0, -1, -2))).max() > 1e-6
    Pt = inp.circular_gaussian(rng, P0.shape, 0.1)
    assert np.abs(gw.self_energy(V, G, Pt, wl.mesh)
                  - brute.self_energy(V, G, Pt, wl.mesh)).max() < 1e-15


# --------------------------------------------------- four-index route ------
@pytest.mark.parametrize("mesh", [(2, 2, 1), (3, 1, 1)])
def test_four_index_screened_interaction(mesh):
    wl, g, H0, S, V, G = _setup(mesh=mesh)
    sinf, stau, d = gw.sigma_evaluation(V, G, g, wl.mesh, NS)
    Wiw, Wtau = fourindex.screened_tilde_W(V, G, wl.mesh, NS, g)
    assert np.abs(Wiw - fourindex.df_tilde_W(V, d["Pw"], wl.mesh)).max() < 1e-14
    assert np.abs(fourindex.self_energy(G, Wtau, wl.mesh) - stau).max() < 1e-14
    assert np.abs(Wiw).max() > 1e-3


# ------------------------------------------------------ scalar closed form ---
@pytest.mark.parametrize("eps,mu,v", [(0.3, 0.1, 0.4), (-0.2, 0.05, 0.7)])
def test_scalar_chain_closed_form(eps, mu, v):
    beta, ntau = 10.0, 24
    g = og.Grids(beta, ntau)
    mesh = (1, 1, 1)
    H0 = np.full((1, 1, 1), eps, complex)
    S = np.ones((1, 1, 1), complex)
    V = np.full((1, 1, 1, 1, 1), v, complex)
    G = gw.g0_tau(H0, S, mu, beta, g.tau)
    xi = eps - mu
    f = 1.0 / (1.0 + np.exp(beta * xi))
    a = NS * v * v * beta * f * (1 - f)
    sinf, stau, d = gw.sigma_evaluation(V, G, g, mesh, NS)
    assert np.abs(d["P0"] + NS * v * v * f * (1 - f)).max() < 1e-15
    ref_w = np.where(g.nB == 0, -a, 0.0)
    assert np.abs(d["P0w"][0, :, 0, 0] - ref_w).max() < 1e-13
    assert np.abs(d["Pt"] + a / (beta * (1 + a))).max() < 1e-12
    ref_sigma = NS * v ** 4 * f * (1 - f) / (1 + a) * G
    assert np.abs(stau - ref_sigma).max() < 1e-13
    gamma = d["gamma"][0, 0, 0]
    assert abs(gamma - f) < 1e-12
    assert abs(sinf[0, 0, 0] - (NS - 1) * v * v * gamma) < 1e-15
    # Eq. tilde_Phi_GW: only W = 0 carries P0, so Phi~ = (ln(1 + a) - a) / (2 beta)
    assert abs(gw.phi_gw(d["P0w"], g, 1) - (np.log1p(a) - a) / (2 * beta)) < 1e-13


def test_phi_gw_second_order_limit():
    """Eq. tilde_Phi_GW for small P0 is -(1/4) Tr{P0^2} (the paper's expansion),
    with Tr{P0^2} = (1/Nk) sum_q int_0^beta tr[P0^q(tau) P0^q(beta - tau)] d tau
    taken by Chebyshev integration of the interpolant on the tau nodes: an
    independent route to the Matsubara-weight quadrature of phi_gw."""
    wl, g, H0, S, V, G = _setup(mesh=(2, 1, 1), nao=3, naux=4, ntau=24, beta=5.0)
    # interpolatory integration weights: int_0^beta T_l(2 tau / beta - 1) = beta/(1 - l^2), l even
    Cm = np.cos(np.outer(np.arccos(g.x), np.arange(wl.ntau)))
    il = np.array([wl.beta / (1.0 - l * l) if l % 2 == 0 else 0.0 for l in range(wl.ntau)])
    wint = il @ np.linalg.inv(Cm)
    ratios = []
    for s in (3e-2, 1e-2, 3e-3):
        _, _, d = gw.sigma_evaluation(V * s / 0.1, G, g, wl.mesh, NS)
        P0 = d["P0"]
        tr2 = sum(wint @ np.array([np.trace(P0[q, i] @ P0[q, wl.ntau - 1 - i]).real
                                   for i in range(wl.ntau)]) for q in range(wl.nk)) / wl.nk
        ratios.append(gw.phi_gw(d["P0w"], g, wl.nk) / (-0.25 * tr2))
    print("Phi~ / (-Tr P0^2 / 4):", ratios)
    # the ratio tends to 1 with corrections of order P0, i.e. as s^2 (about a
    # tenth per step here), above a floor of about 4e-5 from the two
    # quadratures on 24 nodes
    dev_ = [abs(r - 1.0) for r in ratios]
    assert dev_[2] < 5e-4
    assert dev_[0] > 6 * dev_[1] and dev_[1] > 6 * dev_[2]


@pytest.mark.parametrize("ntau", [16, 24])
def test_phi_derivability(ntau):
    """Sigma~ = delta Phi~ / delta G (Sec. III.C): along a smooth direction dG,
    d/dh Phi~[G + h dG] = Tr{Sigma~ dG} = -(ns/Nk) sum_k int_0^beta
    tr[Sigma~^k(tau) dG^k(beta - tau)] d tau (the fermionic Matsubara sum of
    a product in tau, with Sigma~ per spin and the trace over spin-orbitals).
    Central differences of phi_gw against the oracle's own self-energy,
    integrated by Chebyshev weights on the nodes: this ties the signs and
    factors of the polarization, the screened-interaction solve and the
    self-energy contraction to the Luttinger-Ward functional."""
    beta = 5.0
    wl = inp.small_workload(mesh=(2, 1, 1), nao=3, naux=4, ntau=ntau, beta=beta, seed=3)
    g = og.Grids(beta, ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), 3.0 * inp.make_V(wl)
    G = gw.g0_tau(H0, S, 0.1, beta, g.tau)
    rng = np.random.default_rng(4)
    Hp = inp.random_hermitian_tau(rng, 1, wl.nk, wl.nao, 0.3)[0]
    dG = gw.g0_tau(H0 + Hp, S, 0.1, beta, g.tau) - G

    def phi(Gx):
        return gw.phi_gw(gw.sigma_evaluation(V, Gx, g, wl.mesh, NS)[2]["P0w"], g, wl.nk)

    h = 1e-5
    fd = (phi(G + h * dG) - phi(G - h * dG)) / (2 * h)
    _, stau, _ = gw.sigma_evaluation(V, G, g, wl.mesh, NS)
    Cm = np.cos(np.outer(np.arccos(g.x), np.arange(ntau)))
    il = np.array([beta / (1.0 - l * l) if l % 2 == 0 else 0.0 for l in range(ntau)])
    wint = il @ np.linalg.inv(Cm)
    pred = -NS / wl.nk * sum(wint[i] * np.trace(stau[i, k] @ dG[ntau - 1 - i, k]).real
                             for i in range(ntau) for k in range(wl.nk))
    print("d Phi~ / dh", fd, "Tr{Sigma~ dG}", pred)
    assert abs(pred) > 1e-3
    assert abs(fd - pred) < 1e-7 * abs(pred)


# ---------------------------------------------------------------- invariants -
def test_invariants():
    wl, g, H0, S, V, G = _setup(mesh=(3, 1, 1), nao=3, naux=4, ntau=12, beta=10.0)
    plus, minus = gw.mesh_tables(wl.mesh)
    sinf, stau, d = gw.sigma_evaluation(V, G, g, wl.mesh, NS)
    P0, P0w, Pt = d["P0"], d["P0w"], d["Pt"]
    herm = lambda x: np.abs(x - np.conj(np.swapaxes(x, -1, -2))).max()
    assert herm(G) < 1e-15 and herm(P0) < 1e-15 and herm(Pt) < 1e-13
    assert herm(stau) < 1e-14 and herm(sinf) < 1e-15
    # P0^q(beta - tau) = [P0^{-q}(tau)]^T
    for q in range(wl.nk):
        mq = minus[q, 0]
        assert np.abs(P0[q, ::-1] - np.swapaxes(P0[mq], -1, -2)).max() < 1e-15
    # static bubble screens: P0(i Omega_0) is negative semidefinite
    m0 = int(np.nonzero(g.nB == 0)[0][0])
    for q in range(wl.nk):
        assert np.linalg.eigvalsh(P0w[q, m0]).max() < 1e-14
    # causality of Sigma~(i w_n): anti-Hermitian part <= 0 for w_n > 0
    siw = gw.to_iw(g.TF, stau)
    for n in np.nonzero(g.wF > 0)[0]:
        for k in range(wl.nk):
            ah = (siw[n, k] - siw[n, k].conj().T) / 2j
            assert np.linalg.eigvalsh(ah).max() < 1e-12


def _time_reversal_symmetric(wl, H0, V):
    """H0(-k) = H0(k)^*, V^{-k1,-k2}(Q) = V^{k1,k2}(Q)^* (time reversal), keeping
    V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger: average over the group generated by the
    two involutions."""
    plus, minus = gw.mesh_tables(wl.mesh)
    nk = wl.nk
    neg = minus[:, 0]                                        # index of -k
    H = H0.copy()
    for k in range(nk):
        if neg[k] == k:
            H[k] = H0[k].real
        elif k < neg[k]:
            H[neg[k]] = np.conj(H0[k])
    Vf = np.empty((nk, nk) + V.shape[2:], np.complex128)     # Vf[k1, k2] = V^{k1,k2}
    for q in range(nk):
        for k in range(nk):
            Vf[k, plus[q, k]] = V[q, k]
    dag = lambda X: np.conj(np.swapaxes(X, -1, -2))
    A = dag(np.swapaxes(Vf, 0, 1))                           # (V^{k2,k1})^dagger
    B = np.conj(Vf[np.ix_(neg, neg)])                        # conj V^{-k1,-k2}
    AB = dag(np.swapaxes(B, 0, 1))
    W = 0.25 * (Vf + A + B + AB)
    V2 = np.empty_like(V)
    for q in range(nk):
        for k in range(nk):
            V2[q, k] = W[k, plus[q, k]]
    return H, V2


def test_bosonic_symmetry_plain_form_with_time_reversal():
    """Reading R14: with time-reversal-symmetric H0 and V the bubble obeys the
    plain bosonic symmetry P0^q(beta - tau) = P0^q(tau); without time reversal
    only the general identity P0^q(beta - tau) = [P0^{-q}(tau)]^T holds."""
    wl, g, H0, S, V, G = _setup(mesh=(4, 2, 1), nao=3, naux=4, ntau=12, beta=10.0)
    H, V2 = _time_reversal_symmetric(wl, H0, V)
    plus, minus = gw.mesh_tables(wl.mesh)
    neg = minus[:, 0]
    # the construction keeps the pair relation and adds time reversal
    for q in range(wl.nk):
        for k in range(wl.nk):
            k2 = plus[q, k]
            q2 = minus[k2, k]                                 # slab of V^{k2,k}: k + q2 = k
            assert np.abs(V2[q2, k2] - np.conj(np.swapaxes(V2[q, k], -1, -2))).max() < 1e-15
            assert np.abs(V2[neg[q], neg[k]] - np.conj(V2[q, k])).max() < 1e-15
    G2 = gw.g0_tau(H, S, 0.1, wl.beta, g.tau)
    P_tr = gw.polarization(V2, G2, wl.mesh, NS)
    P_gen = gw.polarization(V, G, wl.mesh, NS)
    scale = np.abs(P_tr).max()
    assert scale > 1e-3
    assert np.abs(P_tr[:, ::-1] - P_tr).max() < 1e-14 * scale
    # without time reversal the plain form fails and the general one holds
    assert np.abs(P_gen[:, ::-1] - P_gen).max() > 1e-6 * np.abs(P_gen).max()
    for q in range(wl.nk):
        assert np.abs(P_gen[q, ::-1] - np.swapaxes(P_gen[neg[q]], -1, -2)).max() < 1e-15


def test_momentum_shift_covariance():
    wl, g, H0, S, V, G = _setup(mesh=(3, 1, 1))
    plus, minus = gw.mesh_tables(wl.mesh)
    k0 = 1
    perm = np.array([plus[k0, k] for k in range(wl.nk)])      # k -> k + k0
    G2 = np.empty_like(G)
    G2[:, perm] = G
    V2 = np.empty_like(V)
    V2[:, perm] = V
    _, s1, d1 = gw.sigma_evaluation(V, G, g, wl.mesh, NS)
    _, s2, d2 = gw.sigma_evaluation(V2, G2, g, wl.mesh, NS)
    assert np.abs(d1["P0"] - d2["P0"]).max() < 1e-15
    assert np.abs(s2[:, perm] - s1).max() < 1e-15


def test_single_transfer_vertex():
    wl, g, H0, S, V, G = _setup(mesh=(3, 1, 1))
    q0 = 1
    V1 = np.zeros_like(V)
    V1[q0] = V[q0]
    P0 = gw.polarization(V1, G, wl.mesh, NS)
    for q in range(wl.nk):
        if q != q0:
            assert np.abs(P0[q]).max() == 0.0
    assert np.abs(P0[q0]).max() > 1e-3


# ------------------------------------------------------------- fixed point ---
def test_fixed_point_independent_of_start():
    wl, g, H0, S, V, G = _setup(mesh=(2, 1, 1), nao=2, naux=3, ntau=12, beta=10.0)
    target = 2.0
    h1 = gw.scgw(H0, S, V, g, wl.mesh, NS, target, 40, alpha=0.5, mu0=0.0)
    H0b = H0 + 0.05 * np.eye(wl.nao)[None]           # different starting Hamiltonian
    h2 = gw.scgw(H0b, S, V, g, wl.mesh, NS, target, 2, alpha=0.5, mu0=0.3)
    # continue from the second start with the true H0
    mu, sinf, stau, Gt = h2[-1]
    for _ in range(40):
        s_inf, s_tau, _ = gw.sigma_evaluation(V, Gt, g, wl.mesh, NS)
        sinf = 0.5 * sinf + 0.5 * s_inf
        stau = 0.5 * stau + 0.5 * s_tau
        mu, Giw, _ = gw.find_mu(H0, S, sinf, gw.to_iw(g.TF, stau), target, g, NS, mu)
        Gt = gw.to_tau(g.TFp, Giw)
    assert np.abs(stau - h1[-1][2]).max() < 1e-8
    assert np.abs(sinf - h1[-1][1]).max() < 1e-8
    assert np.abs(h1[-1][2] - h1[-2][2]).max() < 1e-8


# ------------------------------------------------------------- Lindhard -----
def test_lindhard_bubble_in_eigenbases():
    """Non-interacting bubble on the bosonic grid against its closed form: in
    the eigenbases of H0, P0^q(i Omega_m) = -(ns/Nk) sum_k sum_{a in k+q,
    b in k} Vt(Q)_{ba} Vt'(Q')_{ab} (f_a - f_b) / (i Omega_m - xi_a + xi_b),
    with beta f (1 - f) (the limit of the fraction) where xi_a = xi_b and
    Omega_m = 0.  Pins Eq. tilde_P0_tau (with reading R1) and the bosonic
    transform together; the only error is the tau-grid representation."""
    wl = inp.small_workload(mesh=(2, 1, 1), nao=3, naux=4, ntau=40, beta=6.0, seed=17)
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    mu = 0.1
    G = gw.g0_tau(H0, S, mu, wl.beta, g.tau)
    P0w = gw.to_iw(g.TB, np.moveaxis(gw.polarization(V, G, wl.mesh, NS), 1, 0))  # [m][q][Q][Q']
    plus, _ = gw.mesh_tables(wl.mesh)
    eig = [np.linalg.eigh(H0[k]) for k in range(wl.nk)]
    ref = np.zeros_like(P0w)
    for q in range(wl.nk):
        for k in range(wl.nk):
            kq = plus[q, k]
            eb, Ub = eig[k]
            ea, Ua = eig[kq]
            xb, xa = eb - mu, ea - mu
            fb, fa = 1 / (1 + np.exp(wl.beta * xb)), 1 / (1 + np.exp(wl.beta * xa))
            Vt = np.einsum("bi,Qij,ja->Qba", Ub.conj().T, V[q, k], Ua)          # V^{k,k+q}(Q) in eigenbases
            Vtp = np.conj(np.swapaxes(Vt, 1, 2))                                # V^{k+q,k}(Q') = V^{k,k+q}(Q')^H
            for m, Om in enumerate(g.wB):
                d = 1j * Om - xa[None, :] + xb[:, None]                         # [b][a]
                num = fa[None, :] - fb[:, None]
                frac = np.where(np.abs(d) > 1e-12, num / np.where(np.abs(d) > 1e-12, d, 1.0),
                                wl.beta * fa[None, :] * (1 - fa[None, :]))
                ref[m, q] += -(NS / wl.nk) * np.einsum("Qba,Pab,ba->QP", Vt, Vtp, frac)
    err = np.abs(P0w - ref).max()
    print("Lindhard max err", err, "scale", np.abs(ref).max())
    assert err < 1e-10 * max(1.0, np.abs(ref).max()) and np.abs(ref).max() > 1e-3


# ----------------------------------------------------- two-pole Dyson -------
@pytest.mark.parametrize("eps,s,c,mu", [(0.3, 0.2, 0.15, 0.1), (-0.4, -0.1, 0.3, 0.05)])
def test_two_pole_dyson_and_fit(eps, s, c, mu):
    """One orbital with Sigma_inf = s and Sigma~(i w) = c / (i w - xi), xi =
    eps - mu: G(z) = (z - xi) / ((z - z+)(z - z-)) with z+- = xi + s/2 +-
    sqrt(s^2/4 + c), so G(tau) = -sum_+- Z+- e^{-z tau} / (1 + e^{-beta z})
    with Z+- = (z+- - xi) / (z+- - z-+).  Pins the Dyson solve on the sparse
    Matsubara set and the least-squares fit back to tau."""
    beta, ntau = 10.0, 40
    g = og.Grids(beta, ntau)
    xi = eps - mu
    H0 = np.full((1, 1, 1), eps, complex)
    S = np.ones((1, 1, 1), complex)
    sinf = np.full((1, 1, 1), s, complex)
    siw = (c / (1j * g.wF - xi)).reshape(-1, 1, 1, 1)
    Giw = gw.dyson(H0, S, sinf, siw, mu, g.wF)
    r = np.sqrt(s * s / 4 + c)
    zp, zm = xi + s / 2 + r, xi + s / 2 - r
    Zp, Zm = (zp - xi) / (zp - zm), (zm - xi) / (zm - zp)
    ref_iw = Zp / (1j * g.wF - zp) + Zm / (1j * g.wF - zm)
    assert np.abs(Giw[:, 0, 0, 0] - ref_iw).max() < 1e-14
    Gt = gw.to_tau(g.TFp, Giw)[:, 0, 0, 0]
    # fermi_tau(z) = -e^{-z tau} / (1 + e^{-beta z})
    ref_t = Zp * gw.fermi_tau([zp], g.tau, beta)[:, 0] + Zm * gw.fermi_tau([zm], g.tau, beta)[:, 0]
    assert np.abs(Gt - ref_t).max() < 1e-10
