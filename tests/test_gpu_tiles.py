"""Every launch configuration of the two large contractions and of the
producers against the oracle on a ragged shape (naux 70: partial 64-row
tiles, K = naux not a multiple of 32).  The measurement switches read at
context creation pick them: GW_TILE_CFG 0..9 (fp64: four-product complex MFMA
form on 64x64, 64x128, 128x64, 128x64 on eight waves and 64x64 split K; the
three-product (Gauss) form on 64x64, 64x128, 64x96, 128x64 on eight waves and
128x64), GW_PROD_TILES (fp32 producers on the tiled GEMM instead of the
streaming kernel) and GW_SPLIT_CFG (bf16x3 self-energy tiles 128x128, 64x64,
128x64; bf16x6 two LDS stages instead of one).  Each must give the oracle's
Sigma[G] to the fp64 tolerance, or to the mixed-precision bound, and agree
with the default configuration of its precision."""
import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-10
SIGMA_BOUND = 1e-6
SQUARE = {0, 4, 5}      # tile shapes the Hermitian polarization takes


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


@pytest.fixture(scope="module")
def case():
    wl = inp.small_workload(name="tiles", mesh=(2, 1, 2), nao=10, naux=70, ntau=12, beta=15.0,
                            seed=29, n_target=6.0)
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    G = ogw.g0_tau(H0, S, 0.02, wl.beta, g.tau)
    r_inf, r_tau, _ = ogw.sigma_evaluation(V, G, g, wl.mesh, wl.ns)
    return wl, H0, S, V, G, r_inf, r_tau


def sigma(case, precision, hermitian, env, monkeypatch):
    from paper_2206_07660_amd import gw
    from paper_2206_07660_amd.scgw import GWPath
    wl, H0, S, V, G, _, _ = case
    for k in ("GW_TILE_CFG", "GW_PROD_TILES", "GW_SPLIT_CFG"):
        monkeypatch.delenv(k, raising=False)
    for k, v in env.items():
        monkeypatch.setenv(k, str(v))
    c = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=wl.ns, precision=precision,
                   tau_chunk=5)
    try:
        Vd = dev(V if precision == "fp64" else V.astype(np.complex64))
        path = GWPath(c, Vd, dev(H0), dev(S), wl.n_target, hermitian=hermitian)
        sinf, stau = path.sigma(dev(G))
        return sinf.cpu().numpy(), stau.cpu().numpy()
    finally:
        c.close()


@pytest.mark.parametrize("cfg", list(range(10)))
def test_fp64_tile_configs(case, cfg, monkeypatch):
    _, _, _, _, _, r_inf, r_tau = case
    scale = np.abs(r_tau).max()
    for herm in ((False, True) if cfg in SQUARE else (False,)):
        base = sigma(case, "fp64", herm, {}, monkeypatch)
        si, st = sigma(case, "fp64", herm, {"GW_TILE_CFG": cfg}, monkeypatch)
        e_or = max(np.abs(si - r_inf).max(), np.abs(st - r_tau).max())
        e_def = np.abs(st - base[1]).max() / scale
        print(f"GW_TILE_CFG={cfg} hermitian={herm}: vs oracle {e_or:.2e}, vs default {e_def:.2e} "
              f"relative (scale {scale:.2e})")
        assert e_or < TOL and scale > 1e-8
        assert e_def < 1e-12


@pytest.mark.parametrize("precision,env", [
    ("fp32", {"GW_PROD_TILES": 1}),
    ("bf16x3", {"GW_PROD_TILES": 1}),
    ("bf16x3", {"GW_SPLIT_CFG": 0}),
    ("bf16x3", {"GW_SPLIT_CFG": 1}),
    ("bf16x3", {"GW_SPLIT_CFG": 2}),
    ("bf16x6", {"GW_SPLIT_CFG": 1}),
])
def test_mixed_launch_configs(case, precision, env, monkeypatch):
    _, _, _, _, _, r_inf, r_tau = case
    scale = np.abs(r_tau).max()
    base = sigma(case, precision, True, {}, monkeypatch)
    si, st = sigma(case, precision, True, env, monkeypatch)
    e_or = max(np.abs(si - r_inf).max(), np.abs(st - r_tau).max())
    e_def = max(np.abs(si - base[0]).max(), np.abs(st - base[1]).max())
    print(f"{precision} {env}: vs oracle {e_or:.2e} Ha, vs default {e_def:.2e} Ha")
    assert e_or < SIGMA_BOUND
    # the same products summed in the same order: only the tile shape or the
    # producer kernel differs
    assert e_def < 1e-3 * SIGMA_BOUND
