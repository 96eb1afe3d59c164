"""The differentiation workload ad-3x3x3 (Nk 27, nao 16, naux 150, ntau 60,
beta 100, fp64) against the oracle at its full shape:

* one Sigma[G] + Pi evaluation (Eqs. HF_J, HF_K, tilde_P0_tau ...
  tilde_sigma2) to 1e-10;
* the whole-chain JVP (gw_sigma_jvp) against central differences of the
  oracle's forward with h = 1e-6, element by element (to 2e-6 relative: the
  differences carry the oracle's rounding divided by 2h);
* the whole-chain VJP (gw_sigma_vjp) against the same differences through
  the scalar L = Re <R, Sigma[G]>: dL = Re <G_bar, dG>;
* the dot-product identity <R, J dG> = <J^H R, dG> on the GPU alone;
* P~ rebuilt per q inside the derivative calls gives the stored-P~ result;
* Phi~ (Eq. tilde_Phi_GW) of the GPU path at G +/- h dG against the oracle's.

The oracle runs twice (at G + h dG and G - h dG); Sigma[G] is their mean,
which differs from the exact value by O(h^2 |Sigma''|), far below 1e-10.
naux 150 = 2 x 64 + 22 gives ragged tiles in every contraction.
"""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1500)]

H = 1e-6


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def oracle_sigma(V, G, g, mesh, ns, tag):
    """oracle.gw.sigma_evaluation written out step by step, q by q, with a
    progress line every few q (the full shape takes about a minute)."""
    nk = G.shape[1]
    gamma = ogw.density_matrix(G, g.w)
    sig_inf = ogw.hartree_fock(V, gamma, mesh, ns)
    P0 = np.empty((nk, G.shape[0], V.shape[2], V.shape[2]), np.complex128)
    for q in range(nk):
        P0[q] = ogw.polarization(V, G, mesh, ns, qs=[q])[0]
        if q % 9 == 8:
            print(f"[ad3] oracle {tag}: polarization q {q + 1}/{nk}", flush=True)
    P0w = np.stack([ogw.to_iw(g.TB, P0[q]) for q in range(nk)])
    Pw = ogw.screened_W(P0w)
    Pt = np.stack([ogw.to_tau(g.TBp, Pw[q]) for q in range(nk)])
    sig_tau = np.zeros_like(G)
    for q in range(nk):
        ogw.self_energy(V, G, Pt[q:q + 1], mesh, qs=[q], out=sig_tau)
        if q % 9 == 8:
            print(f"[ad3] oracle {tag}: self-energy q {q + 1}/{nk}", flush=True)
    return sig_inf, sig_tau, ogw.phi_gw(P0w, g, nk)


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ad3():
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.adjoint import SigmaDerivatives
    from paper_2206_07660_amd.scgw import GWPath
    wl = inp.WORKLOADS["ad-3x3x3"]
    print("[ad3] building inputs", flush=True)
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    mu = -0.05                                   # inside the gap of the four occupied bands
    G = ogw.g0_tau(H0, S, mu, wl.beta, g.tau)
    rng = np.random.default_rng([wl.seed, 71])
    Hp = inp.random_hermitian_tau(rng, 1, wl.nk, wl.nao, 0.05)[0]
    dG = ogw.g0_tau(H0 + Hp, S, mu, wl.beta, g.tau) - G      # Hermitian, smooth in tau
    R_inf = inp.circular_gaussian(rng, (wl.nk, wl.nao, wl.nao), 1.0)
    R_tau = inp.circular_gaussian(rng, G.shape, 1.0)
    ref = {}
    for sgn in (+1, -1):
        ref[sgn] = oracle_sigma(V, G + sgn * H * dG, g, wl.mesh, wl.ns, "+h" if sgn > 0 else "-h")
    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns)
    path = GWPath(ctx, dev(V), dev(H0), dev(S), wl.n_target, want_phi=True)
    der = SigmaDerivatives(path)
    yield dict(wl=wl, g=g, V=V, G=G, dG=dG, R_inf=R_inf, R_tau=R_tau, ref=ref, ctx=ctx,
               path=path, der=der)
    ctx.close()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_sigma_evaluation_matches_oracle(ad3):
    d = ad3
    print("[ad3] GPU evaluation", flush=True)
    s_inf, s_tau = d["path"].sigma(dev(d["G"]))
    r_inf = 0.5 * (d["ref"][1][0] + d["ref"][-1][0])
    r_tau = 0.5 * (d["ref"][1][1] + d["ref"][-1][1])
    e_inf = np.abs(host(s_inf) - r_inf).max()
    e_tau = np.abs(host(s_tau) - r_tau).max()
    print(f"ad-3x3x3 chain: max|dSigma_inf| {e_inf:.2e} max|dSigma~| {e_tau:.2e} "
          f"(|Sigma~| {np.abs(r_tau).max():.3f})")
    assert e_inf < 1e-10 and e_tau < 1e-10
    assert np.abs(r_tau).max() > 1e-3


def test_jvp_and_vjp_against_oracle_differences(ad3):
    d = ad3
    G, dG = dev(d["G"]), dev(d["dG"])
    print("[ad3] GPU forward, JVP and VJP", flush=True)
    s_inf, s_tau, Pt, Pw = d["der"].forward(G)
    j_inf, j_tau = d["der"].jvp(G, Pt, Pw, dG, hermitian_dG=True)
    Gb = d["der"].vjp(G, Pt, Pw, dev(d["R_inf"]), dev(d["R_tau"]))
    (pi, pt, _), (mi, mt, _) = d["ref"][1], d["ref"][-1]
    fd_inf, fd_tau = (pi - mi) / (2 * H), (pt - mt) / (2 * H)
    e_inf, e_tau = _rel(host(j_inf), fd_inf), _rel(host(j_tau), fd_tau)
    # dL along dG for L = Re <R, Sigma[G]>: the oracle's differences vs the VJP
    fd_L = (np.vdot(d["R_inf"], fd_inf) + np.vdot(d["R_tau"], fd_tau)).real
    vjp_L = np.vdot(host(Gb), d["dG"]).real
    # dot-product identity on the GPU alone
    lhs = np.vdot(d["R_inf"], host(j_inf)) + np.vdot(d["R_tau"], host(j_tau))
    rhs = np.vdot(host(Gb), d["dG"])
    print(f"ad-3x3x3 JVP vs oracle FD: rel {e_inf:.2e} {e_tau:.2e}; "
          f"VJP dL {vjp_L:.12e} vs FD {fd_L:.12e}; dot {abs(lhs - rhs) / abs(lhs):.2e}")
    # the oracle's differences carry its rounding over 2h: about 1e-7 relative
    # at this shape (h = 1e-6 and 1e-5 differences agree to 2e-7)
    assert e_inf < 2e-6 and e_tau < 2e-6
    assert abs(vjp_L - fd_L) < 2e-6 * abs(fd_L)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_per_q_recompute_matches_stored(ad3):
    from paper_2206_07660_amd.adjoint import SigmaDerivatives
    d = ad3
    G, dG = dev(d["G"]), dev(d["dG"])
    s_inf, s_tau, Pt, Pw = d["der"].forward(G)
    a_inf, a_tau = d["der"].jvp(G, Pt, Pw, dG, hermitian_dG=True)
    a_bar = d["der"].vjp(G, Pt, Pw, dev(d["R_inf"]), dev(d["R_tau"]))
    dq = SigmaDerivatives(d["path"], per_q=True)
    q_inf, q_tau, _, _ = dq.forward(G)
    b_inf, b_tau = dq.jvp(G, None, None, dG, hermitian_dG=True)
    b_bar = dq.vjp(G, None, None, dev(d["R_inf"]), dev(d["R_tau"]))
    assert _rel(host(q_tau), host(s_tau)) < 1e-13 and _rel(host(q_inf), host(s_inf)) < 1e-13
    assert _rel(host(b_tau), host(a_tau)) < 1e-12 and _rel(host(b_inf), host(a_inf)) < 1e-12
    assert _rel(host(b_bar), host(a_bar)) < 1e-12


def test_phi_matches_oracle(ad3):
    d = ad3
    vals = {}
    for sgn in (+1, -1):
        d["path"].sigma(dev(d["G"] + sgn * H * d["dG"]))
        vals[sgn] = d["path"].phi
    for sgn in (+1, -1):
        ref = d["ref"][sgn][2]
        print(f"Phi~ GPU {vals[sgn]:.15e} oracle {ref:.15e}")
        assert abs(vals[sgn] - ref) < 1e-10 * abs(ref)
    fd_gpu = (vals[1] - vals[-1]) / (2 * H)
    fd_ref = (d["ref"][1][2] - d["ref"][-1][2]) / (2 * H)
    print(f"d Phi~ / dh: GPU {fd_gpu:.10e} oracle {fd_ref:.10e}")
    assert abs(fd_gpu - fd_ref) < 1e-4 * abs(fd_ref)
