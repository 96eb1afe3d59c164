"""Parity at the full Si-like shape (4x4x4 mesh, nao 26, naux 250, ntau 100,
beta 100) in the launch configuration bench.py uses (all tau in one chunk),
on outputs the oracle can compute one by one: P0^q(tau) for sampled (q, tau)
and the single-q self-energy contribution for sampled (tau, k)."""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def big():
    from paper_2206_07660_amd import gw
    wl = inp.WORKLOADS["si-4x4x4"]
    q = 5
    slab = inp.make_V_slab(wl, q)
    V = torch.zeros((wl.nk, wl.nk, wl.naux, wl.nao, wl.nao), dtype=torch.complex128, device="cuda")
    V[q].copy_(torch.from_numpy(slab))
    rng = np.random.default_rng([wl.seed, 55])
    G = inp.random_hermitian_tau(rng, wl.ntau, wl.nk, wl.nao, 0.1)
    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, max_nq=1)
    Vh = np.zeros((wl.nk,) + slab.shape, np.complex128)
    Vh[q] = slab
    yield dict(wl=wl, q=q, V=V, Vh=Vh, G=G, dG=torch.from_numpy(G).cuda(), ctx=ctx, rng=rng)
    ctx.close()


def test_polarization_sampled(big):
    from paper_2206_07660_amd import gw
    wl, c = big["wl"], big["ctx"]
    assert c.tau_chunk == wl.ntau          # the chunking bench.py runs with
    P = torch.empty((1, wl.ntau, wl.naux, wl.naux), dtype=torch.complex128, device="cuda")
    gw.gw_polarization(c, big["V"], big["dG"], big["q"], 1, P)
    taus = [0, 37, 99]
    ref = ogw.polarization(big["Vh"], big["G"], wl.mesh, wl.ns, qs=[big["q"]], taus=taus)
    got = P.cpu().numpy()[0, taus]
    err = np.abs(got - ref[0]).max()
    print("full-size P0 err", err, "scale", np.abs(ref).max())
    assert err < TOL and np.abs(ref).max() > 1e-4
    # a property at every tau: P0^q(tau) is Hermitian for Hermitian G
    Pa = P.cpu().numpy()[0]
    assert np.abs(Pa - np.conj(np.swapaxes(Pa, -1, -2))).max() < 1e-13


def test_polarization_sampled_hermitian_mode(big):
    """The mode the scGW driver and bench.py run: only the tiles on and above
    the diagonal are contracted, the rest is filled by conjugation."""
    from paper_2206_07660_amd import gw
    wl, c = big["wl"], big["ctx"]
    P = torch.empty((1, wl.ntau, wl.naux, wl.naux), dtype=torch.complex128, device="cuda")
    gw.gw_set_hermitian(c, True)
    try:
        gw.gw_polarization(c, big["V"], big["dG"], big["q"], 1, P)
    finally:
        gw.gw_set_hermitian(c, False)
    taus = [0, 37, 99]
    ref = ogw.polarization(big["Vh"], big["G"], wl.mesh, wl.ns, qs=[big["q"]], taus=taus)
    got = P.cpu().numpy()[0, taus]
    err = np.abs(got - ref[0]).max()
    print("full-size P0 err (Hermitian mode)", err)
    assert err < TOL


def test_self_energy_sampled(big):
    from paper_2206_07660_amd import gw
    wl, c = big["wl"], big["ctx"]
    Pt = inp.random_hermitian_tau(big["rng"], wl.ntau, 1, wl.naux, 0.01)   # [tau][1][Q][Q']
    Pt = np.ascontiguousarray(np.swapaxes(Pt, 0, 1))                       # [1][tau][Q][Q']
    S = torch.zeros((wl.ntau, wl.nk, wl.nao, wl.nao), dtype=torch.complex128, device="cuda")
    gw.gw_self_energy(c, big["V"], big["dG"], torch.from_numpy(Pt).cuda(), big["q"], 1, S)
    taus = [3, 50]
    Gs = big["G"][taus]
    ref = ogw.self_energy(big["Vh"], Gs, Pt[:, taus], wl.mesh, qs=[big["q"]])
    got = S.cpu().numpy()[taus]
    err = np.abs(got - ref).max()
    print("full-size Sigma err", err, "scale", np.abs(ref).max())
    assert err < TOL and np.abs(ref).max() > 1e-6
