"""Pins for the oracle's intermediate-representation grids (oracle/ir.py,
Sec. IV.C): closed-form transforms of single poles in both statistics, the
orthonormality of the Nystrom basis, the analytic Matsubara transforms of
the basis functions against direct quadrature, the sampling points, a
multi-band G0 at beta 200, the density row against the Fermi function, and
the scalar closed form of the whole Sigma chain on these grids."""
import numpy as np
import pytest

from oracle import gw
from oracle import ir

CASES = [(100.0, 500.0, 1e-10), (200.0, 1000.0, 1e-12)]


@pytest.fixture(scope="module", params=CASES, ids=["b100-l500-e10", "b200-l1000-e12"])
def grid(request):
    beta, lam, eps = request.param
    return ir.IRGrids(beta, lam, eps), eps


def _fermion_pole(xi, tau, beta):
    return -np.exp(np.where(xi >= 0, -xi * tau, xi * (beta - tau))) / (1.0 + np.exp(-beta * abs(xi)))


def _boson_pole(xi, tau, beta):
    """B(tau) = -e^{-xi tau} / (1 - e^{-beta xi}), whose transform is 1 / (i Omega - xi)."""
    if xi >= 0:
        return -np.exp(-xi * tau) / (-np.expm1(-beta * xi))
    return np.exp(xi * (beta - tau)) / (-np.expm1(beta * xi))


def test_single_pole_transforms(grid):
    g, eps = grid
    beta, wmax = g.beta, g.basis.lam / g.beta
    ef = eb = ebb = eff = 0.0
    for xi in np.linspace(-0.95 * wmax, 0.95 * wmax, 57):
        G = _fermion_pole(xi, g.tau, beta)
        exact = 1.0 / (1j * g.wF - xi)
        ef = max(ef, np.abs(g.TF @ G - exact).max())
        eff = max(eff, np.abs(g.TFp @ exact - G).max())
        if abs(xi) > 1e-12:
            B = _boson_pole(xi, g.tau, beta)
            exb = 1.0 / (1j * g.wB - xi)
            eb = max(eb, np.abs(g.TB @ B - exb).max() / np.abs(exb).max())
            ebb = max(ebb, np.abs(g.TBp @ exb - B).max() / np.abs(B).max())
    print(f"L {g.ntau}: fermionic {ef:.1e} / fit {eff:.1e}, bosonic {eb:.1e} / fit {ebb:.1e}")
    assert ef < 20 * eps and eb < 20 * eps
    assert eff < 200 * eps and ebb < 200 * eps


def test_basis_orthonormal(grid):
    """The Nystrom functions are orthonormal on [-1, 1] up to the rounding of
    the small singular vectors in double precision, about 1e-16 s_0 / s_l
    (a wrong scale or a transposed factor is off by O(1))."""
    g, _ = grid
    x, w = ir.composite_gauss_legendre(g.basis.breaks_x, 48)
    U = g.basis.u(x)
    gram = U.T @ (w[:, None] * U)
    s = g.basis.s[:g.ntau] / g.basis.s[0]
    bound = 100 * 2.2e-16 / np.minimum.outer(s, s)
    assert np.all(np.abs(gram - np.eye(g.ntau)) < bound)
    assert np.abs(gram - np.eye(g.ntau))[:10, :10].max() < 1e-12


def test_matsubara_transform_against_quadrature(grid):
    """uhat (closed form of the Nystrom sum) against int_0^beta e^{i nu tau} u_l
    d tau by composite Gauss-Legendre in tau.  The Nystrom sum of u_l cancels
    down from terms of size s_0 / s_l, so two evaluation routes agree to about
    1e-16 s_0 / s_l (1e-10 for the leading functions); a wrong sign, factor or
    statistics in the closed form is off by O(1)."""
    g, _ = grid
    beta = g.beta
    x, w = ir.composite_gauss_legendre(g.basis.breaks_x, 64)
    tau, wt = 0.5 * beta * (x + 1.0), 0.5 * beta * w
    U = g.basis.u(x)
    for stat, nn in (("F", np.array([-3, 0, 1, 7, 40])), ("B", np.array([-2, 0, 1, 9, 33]))):
        nu = (2 * nn + 1) * np.pi / beta if stat == "F" else 2 * nn * np.pi / beta
        quad = (np.exp(1j * np.outer(nu, tau)) * wt[None, :]) @ U
        closed = g.basis.uhat(nu, beta, stat)
        sl = g.basis.s[:g.ntau] / g.basis.s[0]
        bound = np.maximum(1e-10, 200 * 2.2e-16 / sl) * np.abs(closed).max(axis=0)
        assert np.all(np.abs(quad - closed).max(axis=0) < bound), stat


def test_sampling_points(grid):
    g, _ = grid
    L = g.ntau
    assert L % 2 == 0 and len(g.nF) == L and len(g.nB) == L + 1
    assert np.abs(g.tau + g.tau[::-1] - g.beta).max() < 1e-12 * g.beta
    assert np.all(np.diff(g.tau) > 0) and g.tau[0] > 0 and g.tau[-1] < g.beta
    uL = g.basis.u(g.x, [L])[:, 0]
    scale = np.abs(g.basis.u(np.linspace(-1, 1, 2001), [L])).max()
    # roots to the rounding level of u_L's Nystrom sum (1e-16 s_0 / s_L)
    assert np.abs(uL).max() < 100 * 2.2e-16 * g.basis.s[0] / g.basis.s[L] * scale
    assert np.array_equal(g.nF, -g.nF[::-1] - 1) and np.array_equal(g.nB, -g.nB[::-1])
    assert np.linalg.cond(g.basis.u(g.x)) < 1e3


def test_multiband_g0_and_density_at_beta_200():
    """G0 of random bands within 0.9 omega_max at beta 200: the transform of
    its nodes equals C (i w - eps)^{-1} C^dagger, the fit returns the nodes,
    and the density row gives the Fermi occupations."""
    g = ir.IRGrids(200.0, 1000.0, 1e-12)
    rng = np.random.default_rng(3)
    n = 6
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    C, _ = np.linalg.qr(Z)
    e = rng.uniform(-4.5, 4.5, n)
    H = (C * e) @ C.conj().T
    G = gw.g0_tau(H[None], np.eye(n)[None], 0.0, g.beta, g.tau)[:, 0]
    Giw = np.einsum("nt,tij->nij", g.TF, G)
    exact = np.stack([(C / (1j * w - e)) @ C.conj().T for w in g.wF])
    back = np.einsum("tn,nij->tij", g.TFp, exact)
    occ = -np.einsum("t,tij->ij", g.w, G)
    f = 1.0 / (1.0 + np.exp(g.beta * e))
    print("G0(i w)", np.abs(Giw - exact).max(), "fit", np.abs(back - G).max())
    assert np.abs(Giw - exact).max() < 1e-10
    assert np.abs(back - G).max() < 1e-10
    assert np.abs(occ - (C * f) @ C.conj().T).max() < 1e-10


def test_scalar_chain_closed_form_on_ir_grids():
    """Nk = nao = naux = 1 (the scalar chain of the design notes): P0(tau) is
    the constant -ns v^2 f (1 - f), P0(i Omega_m) = -a delta_{m0} with
    a = ns v^2 beta f (1 - f), and Sigma~(tau) = ns v^4 f (1 - f) / (1 + a)
    G0(tau), to the representation error of the IR grids."""
    g = ir.IRGrids(50.0, 200.0, 1e-12)
    ns, v, eps_, mu = 2, 0.3, 0.2, 0.0
    xi = eps_ - mu
    f = 1.0 / (1.0 + np.exp(g.beta * xi))
    G = _fermion_pole(xi, g.tau, g.beta).reshape(-1, 1, 1, 1).astype(np.complex128)
    V = np.full((1, 1, 1, 1, 1), v, np.complex128)
    sinf, stau, d = gw.sigma_evaluation(V, G, g, (1, 1, 1), ns)
    a = ns * v * v * g.beta * f * (1 - f)
    assert np.abs(d["P0"][0, :, 0, 0] + ns * v * v * f * (1 - f)).max() < 1e-14
    assert np.abs(d["P0w"][0, :, 0, 0] - np.where(g.nB == 0, -a, 0.0)).max() < 1e-9 * a
    assert np.abs(stau[:, 0, 0, 0] - ns * v ** 4 * f * (1 - f) / (1 + a) * G[:, 0, 0, 0]).max() < 1e-10
    assert abs(sinf[0, 0, 0] - (ns - 1) * v * v * f) < 1e-10


def test_size_grows_with_cutoff_and_precision():
    L = {(lam, eps): ir.Basis(lam, eps).L for lam in (100.0, 1000.0) for eps in (1e-8, 1e-12)}
    assert L[(100.0, 1e-8)] < L[(1000.0, 1e-8)] < L[(1000.0, 1e-12)]
    assert L[(100.0, 1e-8)] < L[(100.0, 1e-12)]
    s = ir.Basis(1000.0, 1e-12).s
    assert np.all(np.diff(s[:80]) < 0)


def test_sigma_chain_same_on_ir_and_chebyshev_grids():
    """The whole Sigma chain from the same G0 on IR grids and on a Chebyshev
    grid fine enough to be exact here: Sigma_inf and Sigma~(i w_n) at the
    lowest Matsubara frequencies agree (each grid evaluates its own tau
    representation at those frequencies)."""
    from oracle import grids as og
    from paper_2206_07660_amd import inputs as inp
    wl = inp.small_workload(mesh=(2, 1, 1), nao=3, naux=6, ntau=40, beta=10.0, seed=17)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    mu = 0.1
    cheb = og.Grids(wl.beta, 40)
    irg = ir.IRGrids(wl.beta, 60.0, 1e-12)
    out = {}
    nn = np.arange(-4, 4)
    nu = (2 * nn + 1) * np.pi / wl.beta
    for name, g in (("cheb", cheb), ("ir", irg)):
        G = gw.g0_tau(H0, S, mu, wl.beta, g.tau)
        sinf, stau, _ = gw.sigma_evaluation(V, G, g, wl.mesh, wl.ns)
        if name == "cheb":
            T = og.transform_matrix(nu, wl.beta, 40)
        else:
            T = g.basis.uhat(nu, wl.beta, "F") @ np.linalg.inv(g.basis.u(g.x))
        out[name] = (sinf, np.tensordot(T, stau, axes=(1, 0)))
    d_inf = np.abs(out["cheb"][0] - out["ir"][0]).max()
    d_iw = np.abs(out["cheb"][1] - out["ir"][1]).max()
    print(f"IR ({irg.ntau} nodes) vs Chebyshev (40): Sigma_inf {d_inf:.1e}, Sigma~(i w) {d_iw:.1e} "
          f"(|Sigma~(i w)| {np.abs(out['cheb'][1]).max():.3f})")
    assert d_inf < 1e-10 and d_iw < 1e-9
