"""Mixed-precision paths (complex fp32 MFMA contractions, or split-bf16
bf16x3 / bf16x6 for the two large ones; fp64 transforms, solves and mu)
against the fp64 oracle.  The stated bound is 1e-6 Ha on the max-abs error of Sigma =
Sigma_inf + Sigma~; the error of G after one Dyson step is bounded by what
such a Sigma error can do to first order (1e-6 max ||G(i w)||_2^2), that of a
band-edge proxy (eigenvalues of H0 + Sigma_inf + Herm Sigma~(i w_0), highest
occupied and lowest empty level over k) by the same 1e-6 Ha."""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIGMA_BOUND = 1e-6


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def band_edges(H0, sinf, siw0, n_occ):
    e = np.stack([np.linalg.eigvalsh(H0[k] + sinf[k] + 0.5 * (siw0[k] + siw0[k].conj().T))
                  for k in range(H0.shape[0])])
    return e[:, n_occ - 1].max(), e[:, n_occ].min()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("name", ["tiny-2x2x2", "ragged"])
def test_mixed_sigma_error(name, precision):
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.scgw import GWPath
    if name == "ragged":
        wl = inp.small_workload(mesh=(2, 2, 2), nao=10, naux=70, ntau=20, beta=20.0, seed=7)
    else:
        wl = inp.WORKLOADS[name]
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    G = ogw.g0_tau(H0, S, wl.mu0, wl.beta, g.tau)
    c = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, precision=precision,
                   tau_chunk=7 if name == "ragged" else None)
    path = GWPath(c, dev(V.astype(np.complex64)), dev(H0), dev(S), wl.n_target)
    sinf, stau = path.sigma(dev(G))
    r_inf, r_tau, d = ogw.sigma_evaluation(V, G, g, wl.mesh, wl.ns)
    e_inf = np.abs(sinf.cpu().numpy() - r_inf).max()
    e_tau = np.abs(stau.cpu().numpy() - r_tau).max()
    # G after one Dyson step with the mixed Sigma vs with the fp64 one
    siw = ogw.to_iw(g.TF, stau.cpu().numpy())
    siw_r = ogw.to_iw(g.TF, r_tau)
    Giw = torch.empty(c.giw_shape(), dtype=torch.complex128, device="cuda")
    gw.gw_dyson_G(c, dev(H0), dev(S), sinf, dev(siw), wl.mu0, Giw)
    G_r = ogw.dyson(H0, S, r_inf, siw_r, wl.mu0, g.wF)
    e_g = np.abs(Giw.cpu().numpy() - G_r).max()
    n0 = int(np.argmin(np.abs(g.wF - g.wF[g.wF > 0].min())))
    n_occ = int(round(wl.n_target / wl.ns))
    vb, cb = band_edges(H0, sinf.cpu().numpy(), siw[n0], n_occ)
    vb_r, cb_r = band_edges(H0, r_inf, siw_r[n0], n_occ)
    print(f"{name} {precision}: max|dSigma_inf| {e_inf:.2e}  max|dSigma~| {e_tau:.2e}  max|dG| {e_g:.2e}  "
          f"band edges {abs(vb - vb_r):.2e} {abs(cb - cb_r):.2e}  (|Sigma~| {np.abs(r_tau).max():.3f})")
    # G = (M - Sigma)^{-1} moves by G dSigma G to first order: a Sigma error of
    # SIGMA_BOUND in operator norm moves G by at most SIGMA_BOUND ||G||_2^2
    g_norm2 = max(np.linalg.norm(G_r[n, k], 2) ** 2 for n in range(G_r.shape[0]) for k in range(G_r.shape[1]))
    print(f"  G bound {SIGMA_BOUND * g_norm2:.2e} (max ||G(i w)||_2^2 = {g_norm2:.1f})")
    assert e_inf < SIGMA_BOUND and e_tau < SIGMA_BOUND
    assert e_g < SIGMA_BOUND * g_norm2
    assert abs(vb - vb_r) < SIGMA_BOUND and abs(cb - cb_r) < SIGMA_BOUND
    assert e_tau > 0.0                      # it really ran in reduced precision
    c.close()
