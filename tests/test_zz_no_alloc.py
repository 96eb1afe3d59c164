"""gw_polarization_noalloc (the polarization on the library's fixed scratch,
for callers that cannot allocate) against gw_polarization, through the C ABI:
two calls in a row on one GPU, the second on a smaller input (fewer q and a
smaller context), each equal to the workspace form; and the clear error for
a shape whose tau slice does not fit the scratch."""
import ctypes

import numpy as np
import pytest

from paper_2206_07660_amd import inputs as inp
from oracle import grids as og
from oracle import gw as ogw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _pair(wl, q0, nq, precision, herm):
    from paper_2206_07660_amd import gw
    g = og.Grids(wl.beta, wl.ntau)
    H0, S, V = inp.make_H0(wl), inp.make_S(wl), inp.make_V(wl)
    G = ogw.g0_tau(H0, S, 0.05, wl.beta, g.tau)
    ctx = gw.Context(wl.mesh, wl.nao, wl.naux, wl.ntau, wl.beta, ns=2, precision=precision,
                     tau_chunk=3)
    try:
        gw.gw_set_hermitian(ctx, herm)
        Vd = dev(V) if precision == "fp64" else dev(V.astype(np.complex64))
        z = dict(dtype=torch.complex128, device="cuda")
        a = torch.full((nq, ctx.ntau, ctx.naux, ctx.naux), complex(np.nan, np.nan), **z)
        b = torch.full((nq, ctx.ntau, ctx.naux, ctx.naux), complex(np.nan, np.nan), **z)
        gw.gw_polarization(ctx, Vd, dev(G), q0, nq, a)
        gw.gw_polarization_noalloc(ctx, Vd, dev(G), q0, nq, b)
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        ref = ogw.polarization(V, G, wl.mesh, 2, qs=range(q0, q0 + nq))
    finally:
        ctx.close()
    return a, b, ref


@pytest.mark.parametrize("precision,herm", [("fp64", False), ("fp64", True), ("fp32", False),
                                            ("bf16x3", True)])
def test_noalloc_matches_workspace_form_twice(precision, herm):
    big = inp.small_workload(mesh=(2, 2, 2), nao=10, naux=70, ntau=20, beta=20.0, seed=81)
    small = inp.small_workload(mesh=(2, 1, 1), nao=6, naux=30, ntau=12, beta=10.0, seed=82)
    # vs the oracle, relative to the largest entry: rounding of fp64; of
    # complex64 operands; of bf16x3 products (near 2^-17 each, 4x margin)
    tol = {"fp64": 1e-13, "fp32": 1e-6, "bf16x3": 1e-4}[precision]
    for wl, q0, nq in ((big, 1, 5), (small, 1, 1)):          # the second call is smaller
        a, b, ref = _pair(wl, q0, nq, precision, herm)
        assert np.isfinite(b).all()
        scale = np.abs(a).max()
        print(f"{precision} herm={herm} {wl.mesh} nq={nq}: |noalloc - workspace| "
              f"{np.abs(a - b).max():.2e}, vs oracle {np.abs(b - ref).max():.2e} (scale {scale:.3f})")
        assert np.abs(a - b).max() <= 1e-14 * scale
        assert np.abs(b - ref).max() <= tol * scale


def test_noalloc_rejects_a_shape_beyond_the_scratch():
    """One tau slice of fp64 intermediates for Nk 64, naux 250, nao 26 is
    2 x 169 MB, above the 128 MiB scratch: GW_ERR_WORKSPACE, nothing launched
    (the arrays here are dummies; the size check comes first)."""
    from paper_2206_07660_amd import gw
    L = gw.load()
    d = gw.Dims((ctypes.c_int * 3)(4, 4, 4), 26, 250, 100, 100, 101, 2, 0, 100.0)
    h = ctypes.c_void_p()
    assert L.gw_create(ctypes.byref(d), None, ctypes.byref(h)) == gw.GW_OK
    try:
        assert L.gw_build_grids(h, None, None) == gw.GW_OK
        dummy = torch.zeros(16, dtype=torch.complex128, device="cuda")
        p = ctypes.c_void_p(dummy.data_ptr())
        assert L.gw_polarization_noalloc(h, p, p, 0, 1, p) == gw.GW_ERR_WORKSPACE
        assert b"fixed scratch" in L.gw_last_error(h)
        torch.cuda.synchronize()
        assert torch.count_nonzero(dummy).item() == 0
    finally:
        L.gw_destroy(h)
