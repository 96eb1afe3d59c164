"""Host-side checks of libgw.so: it loads, exports every symbol the header
declares, rejects bad arguments before touching a GPU, and its host-built
grids agree with the oracle's independent construction."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2206_07660_amd import gw
from oracle import grids as og

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = gw.load()
    hdr = open(os.path.join(ROOT, "include", "gw.h")).read()
    names = set(re.findall(r"^(?:gw_status|size_t|const char\*)\s+(gw_\w+)\(", hdr, re.M))
    assert len(names) >= 18
    for n in sorted(names):
        assert hasattr(L, n), n
    assert set(gw.EXPORTS) <= names


def test_status_strings():
    L = gw.load()
    for s in range(8):
        assert L.gw_status_string(s)
    assert L.gw_status_string(gw.GW_ERR_NONFINITE) == b"non-finite value"
    assert L.gw_status_string(2) == b"HIP runtime error"


@pytest.mark.parametrize("field,value", [("nao", 0), ("nao", 61), ("ntau", 7), ("ns", 3),
                                         ("nw_f", 5), ("nw_b", 10), ("nw_f", 97), ("nw_b", 98),
                                         ("beta", -1.0),
                                         ("naux", 0), ("precision", 9), ("precision", 4),
                                         ("precision", -1)])
def test_create_rejects_bad_dims_without_gpu(field, value):
    L = gw.load()
    d = gw.Dims((ctypes.c_int * 3)(2, 2, 2), 6, 24, 24, 24, 25, 2, 0, 50.0)
    setattr(d, field, value)
    h = ctypes.c_void_p()
    assert L.gw_create(ctypes.byref(d), None, ctypes.byref(h)) == gw.GW_ERR_ARG
    assert not h.value


def test_create_rejects_null():
    L = gw.load()
    h = ctypes.c_void_p()
    assert L.gw_create(None, None, ctypes.byref(h)) == gw.GW_ERR_ARG
    assert L.gw_destroy(None) == gw.GW_ERR_ARG


@pytest.mark.parametrize("beta,ntau", [(50.0, 24), (20.0, 20), (100.0, 60), (100.0, 100),
                                       (200.0, 120)])
def test_host_grids_match_oracle(beta, ntau):
    """(100, 100) and (200, 120) are the grids of the si-4x4x4 and si-5x5x5
    workloads."""
    p = gw.gw_grids_host(beta, ntau)
    o = og.Grids(beta, ntau)
    assert np.array_equal(p["nF"], o.nF) and np.array_equal(p["nB"], o.nB)
    assert np.abs(p["tau"] - o.tau).max() <= 1e-13 * beta
    for key in ("TF", "TB", "TFp", "TBp"):
        ref = getattr(o, key)
        assert np.abs(p[key] - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), key
    assert np.abs(p["w"] - o.w).max() < 1e-12


def test_host_grids_reject_bad_input():
    with pytest.raises(gw.GwError):
        gw.gw_grids_host(-1.0, 24)
    with pytest.raises(gw.GwError):
        gw.gw_grids_host(10.0, 7)
    bad = np.arange(24)[::-1].copy()     # not increasing
    with pytest.raises(gw.GwError):
        gw.gw_grids_host(10.0, 24, nF=bad)


def test_host_grids_given_sets_are_used():
    o = og.Grids(20.0, 20)
    p = gw.gw_grids_host(20.0, 20, nF=o.nF, nB=o.nB)
    assert np.array_equal(p["nF"], o.nF)
    assert np.abs(p["TF"] - o.TF).max() < 1e-11


# ------------------------------------------------------- IR grids (host) ---
@pytest.mark.parametrize("beta,lam,eps", [(100.0, 500.0, 1e-10), (100.0, 500.0, 1e-12),
                                          (200.0, 1000.0, 1e-12), (50.0, 200.0, 1e-10)])
def test_ir_host_grids(beta, lam, eps):
    """The library's IR tables: the oracle's basis size and Matsubara sets, tau
    nodes within the rounding of the small singular vectors (1e-5 beta), and
    transforms that are exact for single poles to the cutoff eps (checked
    against closed forms, not against the oracle's tables)."""
    from oracle import ir
    L = gw.gw_ir_size(lam, eps)
    g = gw.gw_ir_grids_host(beta, lam, eps)
    o = ir.IRGrids(beta, lam, eps)
    assert L == o.ntau and len(g["tau"]) == L
    assert np.array_equal(g["nF"], o.nF) and np.array_equal(g["nB"], o.nB)
    assert np.abs(g["tau"] - o.tau).max() < 1e-5 * beta
    tau = g["tau"]
    assert np.abs(tau + tau[::-1] - beta).max() < 1e-12 * beta
    wF, wB = (2 * g["nF"] + 1) * np.pi / beta, 2 * g["nB"] * np.pi / beta
    wmax = lam / beta
    ef = eff = eb = ew = 0.0
    for xi in np.linspace(-0.95 * wmax, 0.95 * wmax, 41):
        G = -np.exp(np.where(xi >= 0, -xi * tau, xi * (beta - tau))) / (1.0 + np.exp(-beta * abs(xi)))
        ex = 1.0 / (1j * wF - xi)
        ef = max(ef, np.abs(g["TF"] @ G - ex).max())
        eff = max(eff, np.abs(g["TFp"] @ ex - G).max())
        ew = max(ew, abs(g["w"] @ G + 1.0 / (1.0 + np.exp(beta * xi))))       # G(beta^-) = -f
        if abs(xi) > 1e-12:
            B = (-np.exp(-xi * tau) / -np.expm1(-beta * xi)) if xi > 0 else \
                (np.exp(xi * (beta - tau)) / -np.expm1(beta * xi))
            exb = 1.0 / (1j * wB - xi)
            eb = max(eb, np.abs(g["TB"] @ B - exb).max() / np.abs(exb).max())
    assert ef < 20 * eps and eb < 20 * eps and eff < 200 * eps and ew < 20 * eps


def test_ir_host_grids_reject_bad_input():
    for lam, eps in ((0.5, 1e-10), (1e6, 1e-10), (100.0, 0.0), (100.0, 0.5)):
        with pytest.raises(gw.GwError):
            gw.gw_ir_size(lam, eps)
    L = gw.load()
    n = gw.gw_ir_size(100.0, 1e-10)
    z = np.zeros(4 * n * n, np.complex128)
    p = z.ctypes.data_as(ctypes.c_void_p)
    assert L.gw_ir_grids_host(10.0, 100.0, 1e-10, n + 2, None, None, None, p, None, None, None, None) \
        == gw.GW_ERR_ARG
