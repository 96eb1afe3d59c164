"""Pins for the oracle's grand potential and Galitskii-Migdal energy
(oracle/thermo.py, Sec. III.C, Eqs. GP, Phi_GW, tilde_Phi_GW): the free-fermion
and Hartree-Fock limits in closed form, every term of the scalar chain
(Nk = nao = naux = 1) in closed form, and the thermodynamic identity
-dOmega/dmu = N of a Phi-derivable theory at self-consistency."""
import numpy as np
import pytest

from oracle import grids as og
from oracle import gw
from oracle import thermo
from paper_2206_07660_amd import inputs as inp

NS = 2


def _fermi(x, beta):
    return 0.5 * (1.0 - np.tanh(0.5 * beta * x))


def _omega0(x, beta):
    """-(1/beta) ln(1 + e^{-beta x}), overflow-safe."""
    return -(np.maximum(-x, 0.0) + np.log1p(np.exp(-beta * np.abs(x))) / beta)


def _eig(H, S):
    L = np.linalg.cholesky(S)
    Li = np.linalg.inv(L)
    e, U = np.linalg.eigh(Li @ H @ Li.conj().T)
    return e, Li.conj().T @ U


def test_free_fermion_grand_potential():
    wl = inp.small_workload(mesh=(2, 1, 1), nao=4, naux=3, ntau=40, beta=20.0, seed=5, s_kind="random")
    g = og.Grids(wl.beta, wl.ntau)
    H0, S = inp.make_H0(wl), inp.make_S(wl)
    zi = np.zeros_like(H0)
    zw = np.zeros((wl.ntau, wl.nk, wl.nao, wl.nao), np.complex128)

    def om(mu):
        return thermo.grand_potential(H0, S, zi, zw, mu, 0.0, g, NS)

    mu, h = 0.05, 1e-4
    r = om(mu)
    eps = np.concatenate([_eig(H0[k], S[k])[0] for k in range(wl.nk)])
    assert abs(r["omega"] - NS / wl.nk * _omega0(eps - mu, wl.beta).sum()) < 1e-13
    assert abs(r["n_e"] - NS / wl.nk * _fermi(eps - mu, wl.beta).sum()) < 1e-9
    dmu = (om(mu + h)["omega"] - om(mu - h)["omega"]) / (2 * h)
    assert abs(-dmu - r["n_e"]) < 1e-7
    assert r["tr_sigma_g"] == 0.0 and r["phi_inf"] == 0.0


def test_hartree_fock_limit():
    """Sigma~ = 0, Phi~ = 0: Omega = Omega_0[eps_HF] - (1/2) Tr{Sigma_inf rho}
    and E = Tr{H0 rho} + (1/2) Tr{Sigma_inf rho}, rho = C f C^dagger from the
    eigenvectors of (H0 + Sigma_inf, S)."""
    wl = inp.small_workload(mesh=(2, 1, 1), nao=4, naux=3, ntau=40, beta=20.0, seed=6, s_kind="random")
    g = og.Grids(wl.beta, wl.ntau)
    H0, S = inp.make_H0(wl), inp.make_S(wl)
    rng = np.random.default_rng(7)
    Sinf = inp.random_hermitian_tau(rng, 1, wl.nk, wl.nao, 0.3)[0]
    zw = np.zeros((wl.ntau, wl.nk, wl.nao, wl.nao), np.complex128)
    mu = 0.1
    r = thermo.grand_potential(H0, S, Sinf, zw, mu, 0.0, g, NS)
    om0 = x_s = x_h = 0.0
    for k in range(wl.nk):
        e, C = _eig(H0[k] + Sinf[k], S[k])
        rho = (C * _fermi(e - mu, wl.beta)) @ C.conj().T
        om0 += _omega0(e - mu, wl.beta).sum()
        x_s += np.trace(Sinf[k] @ rho).real
        x_h += np.trace(H0[k] @ rho).real
    f = NS / wl.nk
    assert abs(r["omega"] - (f * om0 - 0.5 * f * x_s)) < 1e-9
    assert abs(r["e_gm"] - (f * x_h + 0.5 * f * x_s)) < 1e-9
    assert abs(r["phi_inf"] - 0.5 * f * x_s) < 1e-9


@pytest.mark.parametrize("eps_,mu,v", [(0.3, 0.0, 0.4), (-0.2, 0.1, 0.7)])
def test_scalar_chain_thermodynamics(eps_, mu, v):
    """Nk = nao = naux = 1, Sigma from the chain at G0: Sigma~(i w) =
    C / (i w - xi) with C = ns v^4 f (1 - f) / (1 + a), a = ns v^2 beta f (1 - f),
    Sigma_inf = d = (ns - 1) v^2 f.  G has poles z = xi + d/2 +/- sqrt(d^2/4 + C)
    with weights Z = (z - xi) / (z - z'), so
      Tr ln(-G^{-1}) = ns [w(z+) + w(z-) - w(xi)],   w(x) = ln(1 + e^{-beta x}) / beta,
      Tr{Sigma G}    = ns [d gamma_G + C (f(z+) - f(z-)) / (z+ - z-)],
      gamma_G = sum Z f(z),  Phi~ = (ln(1 + a) - a) / (2 beta)."""
    beta, ntau = 20.0, 40
    g = og.Grids(beta, ntau)
    xi = eps_ - mu
    f = _fermi(xi, beta)
    G0 = (-np.exp(-xi * g.tau) * (1 - f) if xi >= 0 else -np.exp(xi * (beta - g.tau)) * f)
    G0 = G0.reshape(ntau, 1, 1, 1).astype(np.complex128)
    V = np.full((1, 1, 1, 1, 1), v, np.complex128)
    H0 = np.full((1, 1, 1), eps_, np.complex128)
    S = np.ones((1, 1, 1), np.complex128)
    sinf, stau, d = gw.sigma_evaluation(V, G0, g, (1, 1, 1), NS)
    phi = gw.phi_gw(d["P0w"], g, 1)
    siw = gw.to_iw(g.TF, stau)
    r = thermo.grand_potential(H0, S, sinf, siw, mu, phi, g, NS)
    a = NS * v * v * beta * f * (1 - f)
    C = NS * v ** 4 * f * (1 - f) / (1 + a)
    dd = (NS - 1) * v * v * f
    root = np.sqrt(0.25 * dd * dd + C)
    zp, zm = xi + 0.5 * dd + root, xi + 0.5 * dd - root
    w = lambda x: -_omega0(x, beta)
    Zp, Zm = (zp - xi) / (zp - zm), (zm - xi) / (zm - zp)
    gam = Zp * _fermi(zp, beta) + Zm * _fermi(zm, beta)
    tr_ln = NS * (w(zp) + w(zm) - w(xi))
    tr_sg = NS * (dd * gam + C * (_fermi(zp, beta) - _fermi(zm, beta)) / (zp - zm))
    phi_c = (np.log1p(a) - a) / (2 * beta)
    assert abs(sinf[0, 0, 0] - dd) < 1e-13
    assert abs(phi - phi_c) < 1e-12
    assert abs(r["tr_ln"] - tr_ln) < 1e-11
    assert abs(r["tr_sigma_g"] - tr_sg) < 1e-11
    assert abs(r["phi_inf"] - 0.5 * NS * dd * gam) < 1e-11
    assert abs(r["omega"] - (0.5 * NS * dd * gam + phi_c - tr_ln - tr_sg)) < 1e-11
    assert abs(r["e_gm"] - (NS * eps_ * gam + 0.5 * tr_sg)) < 1e-11


def _converged(wl, g, H0, S, V, mu):
    hist = gw.scgw(H0, S, V, g, wl.mesh, NS, None, 120, mu0=mu)
    (_, si0, st0, _), (_, si1, st1, G1) = hist[-2], hist[-1]
    assert max(np.abs(si1 - si0).max(), np.abs(st1 - st0).max()) < 1e-12
    _, _, d = gw.sigma_evaluation(V, G1, g, wl.mesh, NS)
    return si1, gw.to_iw(g.TF, st1), gw.phi_gw(d["P0w"], g, wl.nk)


def test_particle_number_is_minus_dOmega_dmu_at_self_consistency():
    """At the fixed-mu fixed point of the Phi-derivable GW functional,
    -dOmega/dmu equals the electron count; with the opposite sign of the
    static term (Eq. Phi_GW as printed) it does not."""
    wl = inp.small_workload(mesh=(2, 1, 1), nao=2, naux=3, ntau=30, beta=10.0, seed=8, sigma=0.4)
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    mu, h = 0.05, 1e-4
    res, flip = {}, {}
    for m in (mu - h, mu, mu + h):
        si, siw, phi = _converged(wl, g, H0, S, V, m)
        r = thermo.grand_potential(H0, S, si, siw, m, phi, g, NS)
        res[m] = r
        flip[m] = r["omega"] - 2.0 * r["phi_inf"]            # Phi_inf -> -(1/2) Tr{Sigma_inf gamma}
    n = res[mu]["n_e"]
    d = -(res[mu + h]["omega"] - res[mu - h]["omega"]) / (2 * h)
    d_flip = -(flip[mu + h] - flip[mu - h]) / (2 * h)
    print(f"N {n:.10f}  -dOmega/dmu {d:.10f}  with the printed sign {d_flip:.6f}  "
          f"(Tr Sigma_inf gamma {2 * res[mu]['phi_inf']:.4f})")
    assert abs(d - n) < 1e-6
    assert abs(d_flip - n) > 1e-3
