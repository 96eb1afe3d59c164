"""GPU parity: every libgw call against the CPU oracle on the same seeded
inputs, at a size that spans several MFMA tiles with ragged tails
(2x2x2 mesh, nao 10, naux 70, ntau 20 in tau chunks of 7).

Tolerance: 1e-10 max-abs for the fp64 path (the target stated for the
fp64 GW path), on quantities of order 1e-3 .. 1."""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
NS = 2


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def small():
    from paper_2206_07660_amd import gw
    wl = inp.small_workload(mesh=(2, 2, 2), nao=10, naux=70, ntau=20, beta=20.0, seed=7)
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    mu0 = 0.05
    G = ogw.g0_tau(H0, S, mu0, wl.beta, g.tau)
    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=NS, tau_chunk=7)
    d = dict(wl=wl, g=g, H0=H0, S=S, V=V, G=G, mu0=mu0, ctx=ctx,
             dH0=dev(H0), dS=dev(S), dV=dev(V), dG=dev(G))
    yield d
    ctx.close()


def test_context_grids_match_oracle(small):
    c, g = small["ctx"], small["g"]
    assert np.array_equal(c.grids["nF"], g.nF) and np.array_equal(c.grids["nB"], g.nB)
    assert np.abs(c.grids["TF"] - g.TF).max() < 1e-11


def test_polarization(small):
    from paper_2206_07660_amd import gw
    c = small["ctx"]
    P = torch.empty((c.nk, c.ntau, c.naux, c.naux), dtype=torch.complex128, device="cuda")
    gw.gw_polarization(c, small["dV"], small["dG"], 0, c.nk, P)
    ref = ogw.polarization(small["V"], small["G"], small["wl"].mesh, NS)
    err = np.abs(host(P) - ref).max()
    print("polarization max err", err, "scale", np.abs(ref).max())
    assert err < TOL and np.abs(ref).max() > 1e-3
    # q sub-range equals the matching slice
    P2 = torch.empty((2, c.ntau, c.naux, c.naux), dtype=torch.complex128, device="cuda")
    gw.gw_polarization(c, small["dV"], small["dG"], 3, 2, P2)
    assert torch.equal(P2, P[3:5])
    # deterministic: a second run is bitwise identical
    P3 = torch.empty_like(P)
    gw.gw_polarization(c, small["dV"], small["dG"], 0, c.nk, P3)
    assert torch.equal(P, P3)
    # nq = 0 is a no-op
    gw.gw_polarization(c, small["dV"], small["dG"], 0, 0, P3[:0])


def test_polarization_hermitian_mode(small):
    """gw_set_hermitian: upper tiles contracted, lower ones filled by
    conjugation; same values as the oracle and the general mode (G here is
    the Hermitian non-interacting G(tau))."""
    from paper_2206_07660_amd import gw
    c = small["ctx"]
    P = torch.empty((c.nk, c.ntau, c.naux, c.naux), dtype=torch.complex128, device="cuda")
    Pg = torch.empty_like(P)
    gw.gw_polarization(c, small["dV"], small["dG"], 0, c.nk, Pg)
    gw.gw_set_hermitian(c, True)
    try:
        P.fill_(float("nan"))
        gw.gw_polarization(c, small["dV"], small["dG"], 0, c.nk, P)
        # q sub-range in the same mode
        P2 = torch.empty((3, c.ntau, c.naux, c.naux), dtype=torch.complex128, device="cuda")
        gw.gw_polarization(c, small["dV"], small["dG"], 2, 3, P2)
    finally:
        gw.gw_set_hermitian(c, False)
    ref = ogw.polarization(small["V"], small["G"], small["wl"].mesh, NS)
    Ph = host(P)
    assert np.isfinite(Ph).all()
    assert np.abs(Ph - ref).max() < TOL
    assert np.abs(Ph - host(Pg)).max() < 1e-13
    # lower triangle is exactly the conjugate of the upper one
    low = np.tril_indices(c.naux, -1)
    PhT = np.conj(np.swapaxes(Ph, -1, -2))
    assert np.array_equal(Ph[..., low[0], low[1]], PhT[..., low[0], low[1]])
    assert torch.equal(P2, P[2:5])


def test_two_slot_polarization_hermitian_mode(small):
    """GW_HERM_TWO_SLOT: P0[Ga, Gb] + P0[Gb, Ga] for Hermitian Ga, Gb from
    the upper tiles (with accumulation) equals the general two-slot result
    and the oracle's (the JVP of the polarization along a Hermitian dG)."""
    from paper_2206_07660_amd import gw
    c, wl = small["ctx"], small["wl"]
    rng = np.random.default_rng(12)
    Gb_h = inp.random_hermitian_tau(rng, wl.ntau, wl.nk, wl.nao, 0.05)
    Ga, Gb = small["dG"], dev(Gb_h)
    shp = (c.nk, c.ntau, c.naux, c.naux)
    Pg = torch.empty(shp, dtype=torch.complex128, device="cuda")
    Ph = torch.empty_like(Pg)
    gw.gw_polarization2(c, small["dV"], Ga, Gb, 0, c.nk, Pg)
    gw.gw_polarization2(c, small["dV"], Gb, Ga, 0, c.nk, Pg, accumulate=True)
    gw.gw_set_hermitian(c, False, two_slot=True)
    try:
        gw.gw_polarization2(c, small["dV"], Ga, Gb, 0, c.nk, Ph)
        gw.gw_polarization2(c, small["dV"], Gb, Ga, 0, c.nk, Ph, accumulate=True)
    finally:
        gw.gw_set_hermitian(c, False)
    assert np.abs(host(Ph) - host(Pg)).max() < 1e-13
    # oracle: P0 is bilinear in its two G slots (brute-force pinned), so the
    # sum of both orders is the derivative of P0[G] along Gb
    h = 1e-3
    ref = (ogw.polarization(small["V"], small["G"] + h * Gb_h, wl.mesh, NS)
           - ogw.polarization(small["V"], small["G"] - h * Gb_h, wl.mesh, NS)) / (2 * h)
    assert np.abs(host(Ph) - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("stat", [0, 1])
def test_transforms(small, stat):
    from paper_2206_07660_amd import gw
    c, g = small["ctx"], small["g"]
    rng = np.random.default_rng(3)
    nw = c.nw_f if stat == 0 else c.nw_b
    T, Tp = (g.TF, g.TFp) if stat == 0 else (g.TB, g.TBp)
    X = inp.circular_gaussian(rng, (3, c.ntau, 5, 11), 1.0)
    Y = torch.empty((3, nw, 5, 11), dtype=torch.complex128, device="cuda")
    gw.gw_tau_to_iw(c, stat, dev(X), Y, batch=3)
    ref = np.stack([ogw.to_iw(T, X[b]) for b in range(3)])
    assert np.abs(host(Y) - ref).max() < 1e-10 * np.abs(ref).max()
    Z = torch.empty((3, c.ntau, 5, 11), dtype=torch.complex128, device="cuda")
    gw.gw_iw_to_tau(c, stat, Y, Z, batch=3)
    ref2 = np.stack([ogw.to_tau(Tp, ref[b]) for b in range(3)])
    assert np.abs(host(Z) - ref2).max() < 1e-10 * np.abs(ref2).max()
    assert np.abs(host(Z) - X).max() < 1e-9        # least-squares fit inverts exactly


def test_screened_W(small):
    from paper_2206_07660_amd import gw
    c = small["ctx"]
    rng = np.random.default_rng(4)
    P0 = inp.circular_gaussian(rng, (2, c.nw_b, c.naux, c.naux), 0.3 / np.sqrt(c.naux))
    out = torch.empty_like(dev(P0))
    gw.gw_screened_W(c, dev(P0), out)
    ref = ogw.screened_W(P0)
    err = np.abs(host(out) - ref).max()
    print("screened_W max err", err)
    assert err < TOL


def test_screened_W_singular(small):
    from paper_2206_07660_amd import gw
    c = small["ctx"]
    P0 = np.zeros((1, c.nw_b, c.naux, c.naux), np.complex128)
    P0[0, 3] = np.eye(c.naux)                       # I - P0 = 0 for one frequency
    out = torch.empty_like(dev(P0))
    with pytest.raises(gw.GwError) as e:
        gw.gw_screened_W(c, dev(P0), out)
    assert e.value.status == gw.GW_ERR_SINGULAR


def test_self_energy(small):
    from paper_2206_07660_amd import gw
    c = small["ctx"]
    rng = np.random.default_rng(5)
    A = inp.circular_gaussian(rng, (c.nk, c.ntau, c.naux, c.naux), 0.02)
    Pt = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
    S = torch.empty(c.g_shape(), dtype=torch.complex128, device="cuda")
    gw.gw_mix(c, 1.0, None, S)
    gw.gw_self_energy(c, small["dV"], small["dG"], dev(Pt), 0, c.nk, S)
    ref = ogw.self_energy(small["V"], small["G"], Pt, small["wl"].mesh)
    err = np.abs(host(S) - ref).max()
    print("self_energy max err", err, "scale", np.abs(ref).max())
    assert err < TOL and np.abs(ref).max() > 1e-4
    # accumulation over q-batches equals the single pass
    S2 = torch.zeros_like(S)
    dPt = dev(Pt)
    gw.gw_self_energy(c, small["dV"], small["dG"], dPt[:5].contiguous(), 0, 5, S2)
    gw.gw_self_energy(c, small["dV"], small["dG"], dPt[5:].contiguous(), 5, 3, S2)
    assert np.abs(host(S2) - ref).max() < TOL


def test_density_and_hf(small):
    from paper_2206_07660_amd import gw
    c, g = small["ctx"], small["g"]
    gam = torch.empty(c.k_shape(), dtype=torch.complex128, device="cuda")
    n = gw.gw_density(c, small["dG"], small["dS"], gam)
    ref_g = ogw.density_matrix(small["G"], g.w)
    assert np.abs(host(gam) - ref_g).max() < TOL
    assert abs(n - ogw.electron_count(ref_g, small["S"], NS)) < 1e-11
    sinf = torch.empty(c.k_shape(), dtype=torch.complex128, device="cuda")
    gw.gw_hf(c, small["dV"], small["dG"], None, sinf)
    ref = ogw.hartree_fock(small["V"], ref_g, small["wl"].mesh, NS)
    err = np.abs(host(sinf) - ref).max()
    print("hf max err", err, "scale", np.abs(ref).max())
    assert err < TOL


def _random_sigma(c, g, seed):
    rng = np.random.default_rng(seed)
    sinf = inp.random_hermitian_tau(rng, 1, c.nk, c.nao, 0.05)[0]
    stau = inp.random_hermitian_tau(rng, c.ntau, c.nk, c.nao, 0.01)
    return sinf, ogw.to_iw(g.TF, stau)


def test_dyson(small):
    from paper_2206_07660_amd import gw
    c, g = small["ctx"], small["g"]
    sinf, siw = _random_sigma(c, g, 6)
    Giw = torch.empty(c.giw_shape(), dtype=torch.complex128, device="cuda")
    gw.gw_dyson_G(c, small["dH0"], small["dS"], dev(sinf), dev(siw), 0.1, Giw)
    ref = ogw.dyson(small["H0"], small["S"], sinf, siw, 0.1, g.wF)
    err = np.abs(host(Giw) - ref).max()
    print("dyson max err", err)
    assert err < TOL
    # NULL self-energies mean zero
    gw.gw_dyson_G(c, small["dH0"], small["dS"], None, None, 0.1, Giw)
    ref0 = ogw.dyson(small["H0"], small["S"], 0 * sinf, 0 * siw, 0.1, g.wF)
    assert np.abs(host(Giw) - ref0).max() < TOL


@pytest.mark.parametrize("with_sigma", [False, True])
def test_find_mu(small, with_sigma):
    from paper_2206_07660_amd import gw
    c, g, wl = small["ctx"], small["g"], small["wl"]
    sinf, siw = _random_sigma(c, g, 7)
    if not with_sigma:
        sinf, siw = 0 * sinf, 0 * siw
    Giw = torch.empty(c.giw_shape(), dtype=torch.complex128, device="cuda")
    Gt = torch.empty(c.g_shape(), dtype=torch.complex128, device="cuda")
    mu, n = gw.gw_find_mu(c, small["dH0"], small["dS"], dev(sinf), dev(siw), wl.n_target, 0.0,
                          G_iw=Giw, G_tau=Gt)
    mu_r, Giw_r, n_r = ogw.find_mu(small["H0"], small["S"], sinf, siw, wl.n_target, g, NS, 0.0)
    print("find_mu", mu, mu_r, n, n_r)
    assert abs(n - wl.n_target) <= 1e-9
    assert abs(mu - mu_r) < 1e-11
    assert np.abs(host(Gt) - ogw.to_tau(g.TFp, Giw_r)).max() < TOL


def test_find_mu_window(small):
    """gw_set_mu_window: the given mu when its count is within the window,
    else the midpoint of the mu interval where it is, as in the oracle (the
    same decision on both sides); 0 restores the root."""
    from paper_2206_07660_amd import gw
    c, g, wl = small["ctx"], small["g"], small["wl"]
    sinf, siw = _random_sigma(c, g, 7)
    Giw = torch.empty(c.giw_shape(), dtype=torch.complex128, device="cuda")
    Gt = torch.empty(c.g_shape(), dtype=torch.complex128, device="cuda")
    try:
        kept = []
        for w, mu0 in ((1e-9, 0.0), (1e-3, 0.0), (0.5, 0.0), (0.5, 0.3)):
            gw.gw_set_mu_window(c, w)
            mu, n = gw.gw_find_mu(c, small["dH0"], small["dS"], dev(sinf), dev(siw), wl.n_target, mu0,
                                  G_iw=Giw, G_tau=Gt)
            mu_o, Giw_o, n_o = ogw.find_mu(small["H0"], small["S"], sinf, siw, wl.n_target, g, NS, mu0,
                                           window=w)
            print("mu window", w, mu0, mu, mu_o, n, n_o)
            kept.append(mu == mu0)
            assert (mu == mu0) == (mu_o == mu0)
            assert abs(mu - mu_o) < 1e-10
            assert abs(n - wl.n_target) <= w + 1e-12
            assert np.abs(host(Gt) - ogw.to_tau(g.TFp, Giw_o)).max() < TOL
        assert not kept[0] and kept[2]        # searched from outside, kept inside
        with pytest.raises(gw.GwError):
            gw.gw_set_mu_window(c, -1.0)
    finally:
        gw.gw_set_mu_window(c, 0.0)


def test_finite_size_corrections(small):
    """gw_finite_size (Eqs. K_corr, GW_head_corr) against the oracle, added in
    place onto existing self-energies, with each term alone and with a
    non-orthogonal S; argument errors leave the outputs untouched."""
    from paper_2206_07660_amd import gw
    c, g, wl = small["ctx"], small["g"], small["wl"]
    rng = np.random.default_rng(41)
    gam = inp.circular_gaussian(rng, c.k_shape(), 0.3)
    base_inf = inp.circular_gaussian(rng, c.k_shape(), 0.2)
    base_tau = inp.circular_gaussian(rng, c.g_shape(), 0.2)
    head = -0.3 * (np.exp(-0.7 * g.tau) + np.exp(-0.7 * (wl.beta - g.tau)))
    B = inp.circular_gaussian(rng, c.k_shape(), 0.1)
    S = np.eye(c.nao) + B + np.conj(np.swapaxes(B, -1, -2))        # Hermitian, not orthogonal
    chi = 0.29
    r_hf, r_gw = ogw.finite_size_corrections(S, gam, small["G"], chi, head)
    si, st = dev(base_inf), dev(base_tau)
    gw.gw_finite_size(c, dev(S), chi, dev(gam), si, small["dG"], head, st)
    e1 = np.abs(host(si) - (base_inf + r_hf)).max()
    e2 = np.abs(host(st) - (base_tau + r_gw)).max()
    print("finite-size corrections max err", e1, e2)
    assert e1 < TOL and e2 < TOL
    # each term alone
    si, st = dev(base_inf), dev(base_tau)
    gw.gw_finite_size(c, dev(S), chi, gamma=dev(gam), Sig_inf=si)
    gw.gw_finite_size(c, dev(S), chi, G_tau=small["dG"], head=head, Sig_tau=st)
    assert np.abs(host(si) - (base_inf + r_hf)).max() < TOL
    assert np.abs(host(st) - (base_tau + r_gw)).max() < TOL
    # argument errors are found before anything is written
    st = dev(base_tau)
    with pytest.raises(gw.GwError):
        gw.gw_finite_size(c, small["dS"], chi, G_tau=small["dG"], head=np.full(wl.ntau, np.nan), Sig_tau=st)
    with pytest.raises(gw.GwError):
        gw.gw_finite_size(c, small["dS"], float("inf"), gamma=dev(gam), Sig_inf=dev(base_inf))
    assert np.array_equal(host(st), base_tau)


def test_sigma_chain_with_finite_size_corrections(small):
    """GWPath(finite_size=(chi, head)): the Sigma evaluation plus both
    corrections, with gamma of the same G, against the oracle."""
    from paper_2206_07660_amd.scgw import GWPath
    c, g, wl = small["ctx"], small["g"], small["wl"]
    head = -0.3 * (np.exp(-0.7 * g.tau) + np.exp(-0.7 * (wl.beta - g.tau)))
    path = GWPath(c, small["dV"], small["dH0"], small["dS"], wl.n_target, finite_size=(0.29, head))
    sinf, stau = path.sigma(small["dG"])
    r_inf, r_tau, d = ogw.sigma_evaluation(small["V"], small["G"], g, wl.mesh, NS)
    c_hf, c_gw = ogw.finite_size_corrections(small["S"], d["gamma"], small["G"], 0.29, head)
    e1 = np.abs(host(sinf) - (r_inf + c_hf)).max()
    e2 = np.abs(host(stau) - (r_tau + c_gw)).max()
    print("chain with corrections", e1, e2, np.abs(c_hf).max(), np.abs(c_gw).max())
    assert e1 < TOL and e2 < TOL and np.abs(c_hf).max() > 1e-2
    from paper_2206_07660_amd.adjoint import SigmaDerivatives
    with pytest.raises(NotImplementedError):
        SigmaDerivatives(path)


def test_screened_W_phi(small):
    """gw_screened_W_phi: the same P~ as gw_screened_W and Eq. tilde_Phi_GW as
    the oracle (slogdet on the CPU vs the LU diagonal on the GPU); q ranges add."""
    from paper_2206_07660_amd import gw
    c, g, wl = small["ctx"], small["g"], small["wl"]
    _, _, d = ogw.sigma_evaluation(small["V"], small["G"], g, wl.mesh, NS)
    P0w = dev(d["P0w"])
    Pt = torch.empty_like(P0w)
    Pt2 = torch.empty_like(P0w)
    phi = gw.gw_screened_W_phi(c, P0w, Pt)
    gw.gw_screened_W(c, P0w, Pt2)
    ref = ogw.phi_gw(d["P0w"], g, wl.nk)
    print("Phi~", phi, ref, "rel", abs(phi - ref) / abs(ref))
    assert torch.equal(Pt, Pt2)
    # the weights come from grid tables built independently on each side
    # (agreeing to 1e-13 .. 1e-11), so the fp64 bound of the path applies
    assert abs(phi - ref) < TOL * max(1.0, abs(ref)) and abs(ref) > 1e-6
    a = gw.gw_screened_W_phi(c, P0w[:3].contiguous(), Pt[:3].contiguous())
    b = gw.gw_screened_W_phi(c, P0w[3:].contiguous(), Pt[3:].contiguous())
    assert abs(a + b - phi) < 1e-13 * max(1.0, abs(phi))
    # the scGW path keeps Phi~ of the G it evaluates
    from paper_2206_07660_amd.scgw import GWPath
    path = GWPath(c, small["dV"], small["dH0"], small["dS"], wl.n_target, want_phi=True)
    path.sigma(small["dG"])
    assert abs(path.phi - ref) < TOL * max(1.0, abs(ref))


def test_sigma_evaluation_chain(small):
    from paper_2206_07660_amd.scgw import GWPath
    c, g, wl = small["ctx"], small["g"], small["wl"]
    path = GWPath(c, small["dV"], small["dH0"], small["dS"], wl.n_target)
    sinf, stau = path.sigma(small["dG"])
    r_inf, r_tau, _ = ogw.sigma_evaluation(small["V"], small["G"], g, wl.mesh, NS)
    e1, e2 = np.abs(host(sinf) - r_inf).max(), np.abs(host(stau) - r_tau).max()
    print("chain errors", e1, e2, "scales", np.abs(r_inf).max(), np.abs(r_tau).max())
    assert e1 < TOL and e2 < TOL


def test_scgw_iterations(small):
    from paper_2206_07660_amd.scgw import GWPath
    c, g, wl = small["ctx"], small["g"], small["wl"]
    path = GWPath(c, small["dV"], small["dH0"], small["dS"], wl.n_target)
    st = path.start(0.0)
    hist = ogw.scgw(small["H0"], small["S"], small["V"], g, wl.mesh, NS, wl.n_target, 3)
    assert abs(st.mu - hist[0][0]) < 1e-11
    for it in range(1, 4):
        path.step(st)
        mu_r, sinf_r, stau_r, G_r = hist[it]
        print("iteration", it, st.mu, mu_r, st.dsig)
        assert abs(st.mu - mu_r) < 1e-10
        assert np.abs(host(st.sig_inf) - sinf_r).max() < TOL
        assert np.abs(host(st.sig_tau) - stau_r).max() < TOL
        assert np.abs(host(st.G_tau) - G_r).max() < TOL
        assert abs(st.n_e - wl.n_target) <= 1e-9


def test_scalar_closed_form_on_gpu():
    # Nk = nao = naux = 1: the whole chain has a closed form (no oracle involved)
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.scgw import GWPath
    beta, ntau, eps, mu, v = 10.0, 24, 0.3, 0.1, 0.4
    c = gw.Context((1, 1, 1), 1, 1, ntau, beta, ns=NS)
    tau = c.grids["tau"]
    xi = eps - mu
    f = 1.0 / (1.0 + np.exp(beta * xi))
    G = (-np.exp(-xi * tau) * (1 - f)).reshape(ntau, 1, 1, 1).astype(np.complex128)
    V = np.full((1, 1, 1, 1, 1), v, np.complex128)
    H0 = np.full((1, 1, 1), eps, np.complex128)
    path = GWPath(c, dev(V), dev(H0), dev(np.ones((1, 1, 1), complex)), 1.0)
    sinf, stau = path.sigma(dev(G))
    a = NS * v * v * beta * f * (1 - f)
    assert np.abs(host(path.P0w)[0, :, 0, 0] - np.where(c.grids["nB"] == 0, -a, 0.0)).max() < 1e-13
    assert np.abs(host(stau) - NS * v ** 4 * f * (1 - f) / (1 + a) * G).max() < 1e-13
    gamma = -(c.grids["w"] @ G[:, 0, 0, 0])
    assert abs(host(sinf)[0, 0, 0] - (NS - 1) * v * v * gamma) < 1e-15
    c.close()


def test_workspace_too_small(small):
    import ctypes
    from paper_2206_07660_amd import gw
    c = small["ctx"]
    L = gw.load()
    buf = torch.empty(4096, dtype=torch.uint8, device="cuda")
    assert L.gw_set_workspace(c.h, ctypes.c_void_p(buf.data_ptr()), 4096, 7) == gw.GW_OK
    P = torch.empty((1, c.ntau, c.naux, c.naux), dtype=torch.complex128, device="cuda")
    with pytest.raises(gw.GwError) as e:
        gw.gw_polarization(c, small["dV"], small["dG"], 0, 1, P)
    assert e.value.status == gw.GW_ERR_WORKSPACE
    # restore the context's own workspace
    base = (c.workspace.data_ptr() + 255) & ~255
    need = c.workspace.numel() - 256
    assert L.gw_set_workspace(c.h, ctypes.c_void_p(base), need, c.tau_chunk) == gw.GW_OK


def test_descriptor_bounds_whole_path(small, monkeypatch):
    """With GW_DEBUG_BOUNDS=1 every GEMM descriptor of the forward chain (all
    precisions, Hermitian mode on and off), the transforms and the derivative
    calls is proven on the host to stay inside its operands; a failure would
    surface as a GwError."""
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.adjoint import SigmaDerivatives
    from paper_2206_07660_amd.scgw import GWPath
    monkeypatch.setenv("GW_DEBUG_BOUNDS", "1")
    wl = small["wl"]
    for precision in ("fp64", "fp32", "bf16x3"):
        c = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=NS, tau_chunk=7,
                       precision=precision)
        try:
            V = small["dV"] if precision == "fp64" else small["dV"].to(torch.complex64)
            for herm in (False, True):
                path = GWPath(c, V, small["dH0"], small["dS"], wl.n_target, hermitian=herm)
                s_inf, s_tau = path.sigma(small["dG"])
                assert torch.isfinite(s_tau).all()
                der = SigmaDerivatives(path)
                si, st, Pt, Pw = der.forward(small["dG"])
                der.jvp(small["dG"], Pt, Pw, small["dG"])
                der.vjp(small["dG"], Pt, Pw, si, st)
            st = path.start(small["mu0"])
            path.step(st)
            torch.cuda.synchronize()
        finally:
            c.close()
