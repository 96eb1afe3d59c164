"""Pins for the oracle's differentiable twin (oracle/gw_torch.py): its forward
equals the pinned numpy oracle, its JVP matches central finite differences
of the numpy oracle, and its VJP is the adjoint of its JVP (dot-product test)."""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw
from oracle import gw_torch as ogt

NS = 2


@pytest.fixture(scope="module")
def case():
    wl = inp.small_workload(mesh=(2, 2, 1), nao=3, naux=5, ntau=8, beta=8.0, seed=11)
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    G = ogw.g0_tau(H0, S, 0.05, wl.beta, g.tau)
    rng = np.random.default_rng(12)
    dG = inp.random_hermitian_tau(rng, wl.ntau, wl.nk, wl.nao, 0.05)
    return wl, g, V, G, dG, rng


def _dot(a, b):
    return np.vdot(a.ravel(), b.ravel())


def test_twin_forward_matches_oracle(case):
    wl, g, V, G, dG, rng = case
    import torch
    si, st = ogt.sigma_evaluation(*[torch.from_numpy(x) for x in (V, G)][:1],
                                  torch.from_numpy(G), *ogt.tensors(V, g)[1:], wl.mesh, NS)
    r_inf, r_tau, _ = ogw.sigma_evaluation(V, G, g, wl.mesh, NS)
    assert np.abs(si.numpy() - r_inf).max() < 1e-14
    assert np.abs(st.numpy() - r_tau).max() < 1e-14


def test_jvp_matches_finite_differences(case):
    wl, g, V, G, dG, rng = case
    di, ds = ogt.jvp(V, G, dG, g, wl.mesh, NS)
    h = 1e-6
    p_inf, p_tau, _ = ogw.sigma_evaluation(V, G + h * dG, g, wl.mesh, NS)
    m_inf, m_tau, _ = ogw.sigma_evaluation(V, G - h * dG, g, wl.mesh, NS)
    fd_inf, fd_tau = (p_inf - m_inf) / (2 * h), (p_tau - m_tau) / (2 * h)
    assert np.abs(di - fd_inf).max() < 1e-8 * np.abs(fd_inf).max()
    assert np.abs(ds - fd_tau).max() < 1e-7 * np.abs(fd_tau).max()
    assert np.abs(fd_tau).max() > 1e-4


def test_vjp_is_adjoint_of_jvp(case):
    wl, g, V, G, dG, rng = case
    Sb_inf = inp.circular_gaussian(rng, (wl.nk, wl.nao, wl.nao), 1.0)
    Sb_tau = inp.circular_gaussian(rng, G.shape, 1.0)
    Gb = ogt.vjp(V, G, Sb_inf, Sb_tau, g, wl.mesh, NS)
    di, ds = ogt.jvp(V, G, dG, g, wl.mesh, NS)
    lhs = _dot(Sb_inf, di) + _dot(Sb_tau, ds)
    rhs = _dot(Gb, dG)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
