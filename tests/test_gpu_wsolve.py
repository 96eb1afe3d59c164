"""The screened-interaction solve (Eq. tilde_P_omega, P~ = (I - P0)^{-1} P0 by
the blocked LU of gw_screened_W) at the auxiliary-basis sizes of the
si-4x4x4 (naux 250, 8 panels of 32 columns) and si-5x5x5 (naux 300, 10
panels) workloads, on a physical P0(i Omega) of one q: the transform of a
negative semidefinite, bosonic-symmetric P0(tau) = -sum_r B_r B_r^H
(e^{-e_r tau} + e^{-e_r (beta - tau)}) / 2 with random vectors B_r, built on
the CPU.  Compared with the oracle's numpy solve of every matrix."""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def physical_p0_iw(grids, naux, rank, seed, scale):
    rng = np.random.default_rng([seed, 41])
    B = inp.circular_gaussian(rng, (rank, naux), 1.0)
    e = rng.uniform(0.2, 3.0, size=rank)
    tau, beta = grids.tau, grids.beta
    f = 0.5 * (np.exp(-np.outer(tau, e)) + np.exp(-np.outer(beta - tau, e)))       # (ntau, rank)
    P = -np.einsum("tr,ra,rb->tab", f, B, B.conj())
    P *= scale / np.abs(np.linalg.eigvalsh(ogw.to_iw(grids.TB, P)[np.argmin(np.abs(grids.nB))])).max()
    return ogw.to_iw(grids.TB, P)                                                  # (nw_b, naux, naux)


@pytest.mark.parametrize("naux,ntau,beta", [(250, 100, 100.0), (300, 120, 200.0)])
def test_screened_W_at_workload_sizes(naux, ntau, beta):
    from paper_2206_07660_amd import gw
    g = og.Grids(beta, ntau)
    P0w = physical_p0_iw(g, naux, rank=40, seed=naux, scale=3.0)[None]     # one q
    ref = ogw.screened_W(P0w)
    ctx = gw.Context((1, 1, 1), 2, naux, ntau, beta, ns=2)
    try:
        assert np.array_equal(ctx.grids["nB"], g.nB)
        Pt = torch.empty(P0w.shape, dtype=torch.complex128, device="cuda")
        gw.gw_screened_W(ctx, torch.from_numpy(P0w).to("cuda"), Pt)
        out = Pt.cpu().numpy()
        err = np.abs(out - ref).max()
        print(f"naux {naux}: max|P~ - oracle| {err:.2e} (|P~| {np.abs(ref).max():.3f}, "
              f"{P0w.shape[1]} matrices)")
        assert err < 1e-11 * max(1.0, np.abs(ref).max())
        # static screening: I - P0(i Omega_0) is positive definite, P~(i Omega_0) <= 0
        m0 = int(np.argmin(np.abs(g.nB)))
        assert np.linalg.eigvalsh(0.5 * (out[0, m0] + out[0, m0].conj().T)).max() < 1e-12
    finally:
        ctx.close()
