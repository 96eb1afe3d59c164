"""Python binding of libgw.so (the C ABI declared in include/gw.h).

Argument marshalling only: every step of the GW path runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream.  The functions
keep the C names; array arguments are torch complex128 tensors on the GPU in
the layouts of include/gw.h.  If the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgw.so")

(GW_OK, GW_ERR_ARG, GW_ERR_DEVICE, GW_ERR_SINGULAR, GW_ERR_NOCONV, GW_ERR_WORKSPACE, GW_ERR_STATE,
 GW_ERR_NONFINITE) = range(8)
GW_FERMION, GW_BOSON = 0, 1
GW_PREC_FP64, GW_PREC_FP32, GW_PREC_BF16X3, GW_PREC_BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp64": GW_PREC_FP64, "fp32": GW_PREC_FP32, "bf16x3": GW_PREC_BF16X3, "bf16x6": GW_PREC_BF16X6}
(GW_OP_POLARIZATION, GW_OP_SELF_ENERGY, GW_OP_SCREENED_W, GW_OP_HF, GW_OP_DYSON_JVP, GW_OP_SIGMA,
 GW_OP_THERMO) = range(7)
KCLASS = dict(other=0, pol_contract=1, pol_producer=2, se_contract=3, se_producer=4,
              se_final=5, transform=6, hf=7, wdyson=8, dyson=9)

EXPORTS = ["gw_create", "gw_destroy", "gw_build_grids", "gw_get_grids", "gw_workspace_bytes",
           "gw_set_workspace", "gw_polarization", "gw_tau_to_iw", "gw_iw_to_tau",
           "gw_screened_W", "gw_self_energy", "gw_density", "gw_hf", "gw_dyson_G",
           "gw_find_mu", "gw_mix", "gw_grids_host", "gw_profile_enable", "gw_profile_read",
           "gw_polarization2", "gw_screened_W_lin", "gw_transform_adjoint", "gw_self_energy_vjp",
           "gw_polarization_vjp", "gw_hf_vjp", "gw_dyson_jvp", "gw_axpby", "gw_dot",
           "gw_synchronize", "gw_status_string", "gw_last_error", "gw_set_hermitian",
           "gw_hermitize", "gw_set_mu_window", "gw_finite_size", "gw_screened_W_phi",
           "gw_set_grids", "gw_sigma", "gw_sigma_jvp", "gw_sigma_vjp", "gw_polarization_noalloc",
           "gw_ir_size", "gw_ir_grids_host", "gw_build_ir_grids", "gw_thermodynamics"]


class GwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("mesh", ctypes.c_int * 3), ("nao", ctypes.c_int), ("naux", ctypes.c_int),
                ("ntau", ctypes.c_int), ("nw_f", ctypes.c_int), ("nw_b", ctypes.c_int),
                ("ns", ctypes.c_int), ("precision", ctypes.c_int), ("beta", ctypes.c_double)]


_lib = None


def load():
    """Load libgw.so from the package directory (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2206_07660_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, LL, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong, ctypes.c_size_t
    sig = {
        "gw_create": ([ctypes.POINTER(Dims), P, ctypes.POINTER(P)], I),
        "gw_destroy": ([P], I),
        "gw_build_grids": ([P, P, P], I),
        "gw_get_grids": ([P, P, P, P, P, P, P, P, P], I),
        "gw_set_grids": ([P, P, P, P, P, P, P, P, P], I),
        "gw_sigma": ([P, P, P, P, P, P, P, P, P, P], I),
        "gw_sigma_jvp": ([P, P, P, P, P, P, P, P], I),
        "gw_sigma_vjp": ([P, P, P, P, P, P, P, P], I),
        "gw_workspace_bytes": ([P, I, I], SZ),
        "gw_set_workspace": ([P, P, SZ, I], I),
        "gw_polarization": ([P, P, P, I, I, P], I),
        "gw_polarization_noalloc": ([P, P, P, I, I, P], I),
        "gw_set_hermitian": ([P, I], I),
        "gw_set_mu_window": ([P, D], I),
        "gw_finite_size": ([P, P, D, P, P, P, P, P], I),
        "gw_screened_W_phi": ([P, P, I, P, P], I),
        "gw_hermitize": ([P, P, I, LL], I),
        "gw_tau_to_iw": ([P, I, P, LL, LL, P], I),
        "gw_iw_to_tau": ([P, I, P, LL, LL, P], I),
        "gw_screened_W": ([P, P, I, P], I),
        "gw_self_energy": ([P, P, P, P, I, I, P], I),
        "gw_density": ([P, P, P, P, P], I),
        "gw_hf": ([P, P, P, P, P], I),
        "gw_dyson_G": ([P, P, P, P, P, D, P], I),
        "gw_find_mu": ([P, P, P, P, P, D, D, P, P, P, P], I),
        "gw_synchronize": ([P], I),
        "gw_mix": ([P, LL, D, P, P, P], I),
        "gw_profile_enable": ([P, I], I),
        "gw_polarization2": ([P, P, P, P, I, I, I, P], I),
        "gw_screened_W_lin": ([P, P, P, I, I, P], I),
        "gw_transform_adjoint": ([P, I, I, P, LL, LL, P], I),
        "gw_self_energy_vjp": ([P, P, P, P, P, I, I, P, P], I),
        "gw_polarization_vjp": ([P, P, P, P, I, I, P], I),
        "gw_hf_vjp": ([P, P, P, P], I),
        "gw_dyson_jvp": ([P, P, P, P, P, I, P, P], I),
        "gw_axpby": ([P, LL, D, D, P, D, D, P], I),
        "gw_dot": ([P, LL, P, P, P], I),
        "gw_profile_read": ([P, I, P, P, P], I),
        "gw_grids_host": ([D, I, P, P, P, P, P, P, P, P, P, P], I),
        "gw_ir_size": ([D, D, P], I),
        "gw_ir_grids_host": ([D, D, D, I, P, P, P, P, P, P, P, P], I),
        "gw_build_ir_grids": ([P, D, D], I),
        "gw_thermodynamics": ([P, P, P, P, P, D, D, P], I),
        "gw_status_string": ([I], ctypes.c_char_p),
        "gw_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _ptr(t, name, shape=None, dtype=None):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    want = torch.complex128 if dtype is None else dtype
    if t.dtype != want:
        raise TypeError(f"{name} must be {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def gw_grids_host(beta, ntau, nF=None, nB=None):
    """Host-only grid tables (no GPU needed); same content as Context.get_grids()."""
    L = load()
    nt, nf, nb = int(ntau), int(ntau), int(ntau) + 1
    out = dict(tau=np.zeros(nt), nF=np.zeros(nf, np.int64), nB=np.zeros(nb, np.int64),
               TF=np.zeros((nf, nt), np.complex128), TFp=np.zeros((nt, nf), np.complex128),
               TB=np.zeros((nb, nt), np.complex128), TBp=np.zeros((nt, nb), np.complex128),
               w=np.zeros(nt))
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    nfa = None if nF is None else np.ascontiguousarray(nF, np.int64)
    nba = None if nB is None else np.ascontiguousarray(nB, np.int64)
    st = L.gw_grids_host(float(beta), nt, p(nfa) if nfa is not None else None,
                         p(nba) if nba is not None else None, p(out["tau"]), p(out["nF"]),
                         p(out["nB"]), p(out["TF"]), p(out["TFp"]), p(out["TB"]), p(out["TBp"]),
                         p(out["w"]))
    if st != GW_OK:
        raise GwError(st, "gw_grids_host: " + L.gw_status_string(st).decode())
    return out


def gw_ir_size(lam, eps):
    """Basis size L of the IR grids for (lambda, eps) (host only)."""
    L = load()
    n = ctypes.c_int()
    st = L.gw_ir_size(float(lam), float(eps), ctypes.byref(n))
    if st != GW_OK:
        raise GwError(st, "gw_ir_size: " + L.gw_status_string(st).decode())
    return n.value


def gw_ir_grids_host(beta, lam, eps):
    """IR grid tables (host only): dict with tau, nF, nB, TF, TFp, TB, TBp, w."""
    L = load()
    nt = gw_ir_size(lam, eps)
    nf, nb = nt, nt + 1
    out = dict(tau=np.zeros(nt), nF=np.zeros(nf, np.int64), nB=np.zeros(nb, np.int64),
               TF=np.zeros((nf, nt), np.complex128), TFp=np.zeros((nt, nf), np.complex128),
               TB=np.zeros((nb, nt), np.complex128), TBp=np.zeros((nt, nb), np.complex128),
               w=np.zeros(nt))
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    st = L.gw_ir_grids_host(float(beta), float(lam), float(eps), nt, p(out["tau"]), p(out["nF"]),
                            p(out["nB"]), p(out["TF"]), p(out["TFp"]), p(out["TB"]), p(out["TBp"]),
                            p(out["w"]))
    if st != GW_OK:
        raise GwError(st, "gw_ir_grids_host: " + L.gw_status_string(st).decode())
    return out


class Context:
    """One library context: dimensions, grids, stream and workspace."""

    def __init__(self, mesh, nao, naux, ntau, beta, ns=2, nF=None, nB=None, tau_chunk=None,
                 max_nq=None, stream=None, workspace_gb=None, precision="fp64", grids=None, ir=None):
        """grids: None builds the Chebyshev tables in the library
        (gw_build_grids with the Matsubara sets nF, nB or its own greedy
        choice); or a dict with tau, nF, nB, TF, TFp, TB, TBp, w (numpy host
        arrays, e.g. an intermediate-representation basis) installed with
        gw_set_grids, whose shapes fix nw_f and nw_b.
        ir: None, or (lambda, eps): intermediate-representation grids built by
        the library (gw_build_ir_grids); ntau is then the basis size
        (pass None) with nw_f = ntau and nw_b = ntau + 1."""
        import torch
        L = load()
        if precision not in PRECISIONS:
            raise ValueError("precision is one of " + ", ".join(repr(k) for k in PRECISIONS))
        self.precision = precision
        self.v_dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.mesh = tuple(int(m) for m in mesh)
        self.nk = int(np.prod(self.mesh))
        self.nao, self.naux, self.beta, self.ns = int(nao), int(naux), float(beta), int(ns)
        self.ntau = None if ntau is None else int(ntau)
        if ir is not None:
            n_ir = gw_ir_size(*ir)
            if ntau is not None and int(ntau) != n_ir:
                raise ValueError(f"ntau {ntau} differs from the IR basis size {n_ir}")
            self.ntau = n_ir
        if grids is None:
            self.nw_f, self.nw_b = self.ntau, self.ntau + 1
        else:
            self.nw_f, self.nw_b = len(grids["nF"]), len(grids["nB"])
        d = Dims((ctypes.c_int * 3)(*self.mesh), self.nao, self.naux, self.ntau, self.nw_f,
                 self.nw_b, self.ns, PRECISIONS[precision],
                 self.beta)
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        st = L.gw_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != GW_OK:
            raise GwError(st, "gw_create failed: " + L.gw_status_string(st).decode())
        self.h = h
        if ir is not None:
            self._check(L.gw_build_ir_grids(self.h, float(ir[0]), float(ir[1])), "gw_build_ir_grids")
        elif grids is None:
            nf = None if nF is None else (ctypes.c_longlong * self.nw_f)(*[int(x) for x in nF])
            nb = None if nB is None else (ctypes.c_longlong * self.nw_b)(*[int(x) for x in nB])
            self._check(L.gw_build_grids(self.h, nf, nb), "gw_build_grids")
        else:
            self.set_grids(grids)
        # workspace: largest tau chunk that fits the budget (default 40% of free memory)
        free, _ = torch.cuda.mem_get_info()
        budget = int((workspace_gb * 2 ** 30) if workspace_gb else 0.4 * free)
        self.max_nq = self.nk if max_nq is None else int(max_nq)
        if tau_chunk is None:
            tau_chunk = self.ntau
            while tau_chunk > 1 and L.gw_workspace_bytes(self.h, GW_OP_POLARIZATION, tau_chunk) > budget:
                tau_chunk = (tau_chunk + 1) // 2
        self.tau_chunk = int(tau_chunk)
        need = max(L.gw_workspace_bytes(self.h, GW_OP_POLARIZATION, self.tau_chunk),
                   L.gw_workspace_bytes(self.h, GW_OP_SIGMA, self.tau_chunk),
                   L.gw_workspace_bytes(self.h, GW_OP_SCREENED_W, self.max_nq),
                   L.gw_workspace_bytes(self.h, GW_OP_HF, 1),
                   L.gw_workspace_bytes(self.h, GW_OP_DYSON_JVP, 1),
                   L.gw_workspace_bytes(self.h, GW_OP_THERMO, 1))
        self.workspace = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self._check(L.gw_set_workspace(self.h, ctypes.c_void_p(aligned), need, self.tau_chunk),
                    "gw_set_workspace")
        self.grids = self.get_grids()

    def _check(self, st, what):
        if st != GW_OK:
            L = load()
            raise GwError(st, f"{what}: {L.gw_status_string(st).decode()}: "
                              f"{L.gw_last_error(self.h).decode()}")

    def set_grids(self, grids):
        """Install host tables with gw_set_grids (see include/gw.h)."""
        L = load()
        nt, nf, nb = self.ntau, self.nw_f, self.nw_b
        shapes = dict(tau=(nt,), nF=(nf,), nB=(nb,), TF=(nf, nt), TFp=(nt, nf), TB=(nb, nt),
                      TBp=(nt, nb), w=(nt,))
        types = dict(tau=np.float64, nF=np.int64, nB=np.int64, TF=np.complex128, TFp=np.complex128,
                     TB=np.complex128, TBp=np.complex128, w=np.float64)
        arr = {}
        for k, shp in shapes.items():
            a = np.ascontiguousarray(np.asarray(grids[k]), dtype=types[k])
            if a.shape != shp:
                raise ValueError(f"grids[{k!r}] has shape {a.shape}, expected {shp}")
            arr[k] = a
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(L.gw_set_grids(self.h, p(arr["tau"]), p(arr["nF"]), p(arr["nB"]), p(arr["TF"]),
                                   p(arr["TFp"]), p(arr["TB"]), p(arr["TBp"]), p(arr["w"])),
                    "gw_set_grids")

    def get_grids(self):
        L = load()
        nt, nf, nb = self.ntau, self.nw_f, self.nw_b
        out = dict(tau=np.zeros(nt), nF=np.zeros(nf, np.int64), nB=np.zeros(nb, np.int64),
                   TF=np.zeros((nf, nt), np.complex128), TFp=np.zeros((nt, nf), np.complex128),
                   TB=np.zeros((nb, nt), np.complex128), TBp=np.zeros((nt, nb), np.complex128),
                   w=np.zeros(nt))
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(L.gw_get_grids(self.h, p(out["tau"]), p(out["nF"]), p(out["nB"]), p(out["TF"]),
                                   p(out["TFp"]), p(out["TB"]), p(out["TBp"]), p(out["w"])),
                    "gw_get_grids")
        return out

    def close(self):
        if getattr(self, "h", None) is not None:
            load().gw_destroy(self.h)
            self.h = None
            self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes
    def g_shape(self):
        return (self.ntau, self.nk, self.nao, self.nao)

    def giw_shape(self):
        return (self.nw_f, self.nk, self.nao, self.nao)

    def v_shape(self):
        return (self.nk, self.nk, self.naux, self.nao, self.nao)

    def k_shape(self):
        return (self.nk, self.nao, self.nao)


# --------------------------------------------------------------- the calls ---
GW_HERM_FORWARD, GW_HERM_TWO_SLOT = 1, 2


def gw_set_hermitian(ctx, on, two_slot=False):
    """on: gw_polarization's G is Hermitian; two_slot: so are both G of
    gw_polarization2 (see gw.h)."""
    mode = (GW_HERM_FORWARD if on else 0) | (GW_HERM_TWO_SLOT if two_slot else 0)
    ctx._check(load().gw_set_hermitian(ctx.h, mode), "gw_set_hermitian")


def gw_set_mu_window(ctx, ne_tol):
    """gw_find_mu returns the midpoint of the mu interval where
    |N_e - n_target| <= ne_tol (0: the root; see gw.h)."""
    ctx._check(load().gw_set_mu_window(ctx.h, float(ne_tol)), "gw_set_mu_window")


def gw_finite_size(ctx, S, chi, gamma=None, Sig_inf=None, G_tau=None, head=None, Sig_tau=None):
    """Sig_inf += -chi S gamma S and Sig_tau(tau_i) += -chi head[i] S G(tau_i) S
    (head: ntau values of eps^{-1}_00(-tau_i) - 1, host); see gw.h."""
    hp = None
    if head is not None:
        h = np.ascontiguousarray(np.asarray(head, dtype=np.float64))
        if h.shape != (ctx.ntau,):
            raise ValueError("head must hold ntau values")
        hp = h.ctypes.data_as(ctypes.c_void_p)
    ks, gs = ctx.k_shape(), ctx.g_shape()
    ctx._check(load().gw_finite_size(ctx.h, _ptr(S, "S", ks), float(chi), _ptr(gamma, "gamma", ks),
                                     _ptr(Sig_inf, "Sig_inf", ks), _ptr(G_tau, "G_tau", gs), hp,
                                     _ptr(Sig_tau, "Sig_tau", gs)),
               "gw_finite_size")


def gw_hermitize(ctx, X, n):
    """X viewed as [..., n, n] complex128 <- its Hermitian part, in place."""
    _ptr(X, "X")
    if X.numel() % (n * n):
        raise ValueError("gw_hermitize: X must hold whole n x n blocks")
    nmat = X.numel() // (n * n)
    for b0 in range(0, nmat, 65535):
        nb = min(65535, nmat - b0)
        ctx._check(load().gw_hermitize(ctx.h, ctypes.c_void_p(X.data_ptr() + b0 * n * n * 16),
                                       int(n), nb), "gw_hermitize")


def gw_polarization(ctx, V, G_tau, q0, nq, P0_tau):
    ctx._check(load().gw_polarization(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        int(q0), int(nq),
        _ptr(P0_tau, "P0_tau", (nq, ctx.ntau, ctx.naux, ctx.naux))), "gw_polarization")


def gw_polarization_noalloc(ctx, V, G_tau, q0, nq, P0_tau):
    """gw_polarization on the library's fixed scratch (no allocation; see gw.h)."""
    ctx._check(load().gw_polarization_noalloc(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        int(q0), int(nq),
        _ptr(P0_tau, "P0_tau", (nq, ctx.ntau, ctx.naux, ctx.naux))), "gw_polarization_noalloc")


def _transform(fn, ctx, stat, Xin, Xout, batch, fwd):
    nw = ctx.nw_f if stat == GW_FERMION else ctx.nw_b
    nin, nout = (ctx.ntau, nw) if fwd else (nw, ctx.ntau)
    if Xin.numel() % (batch * nin):
        raise ValueError("input size is not a multiple of batch * rows")
    R = Xin.numel() // (batch * nin)
    if Xout.numel() != batch * nout * R:
        raise ValueError("output size does not match")
    ctx._check(fn(ctx.h, int(stat), _ptr(Xin, "X_in"), int(batch), int(R), _ptr(Xout, "X_out")),
               fn.__name__)


def gw_tau_to_iw(ctx, stat, X_tau, X_iw, batch=1):
    """X_iw[b][n][r] = sum_i T[n][i] X_tau[b][i][r]  (tensors [batch][ntau][...])."""
    _transform(load().gw_tau_to_iw, ctx, stat, X_tau, X_iw, batch, True)


def gw_iw_to_tau(ctx, stat, X_iw, X_tau, batch=1):
    """X_tau[b][i][r] = sum_n Tp[i][n] X_iw[b][n][r]."""
    _transform(load().gw_iw_to_tau, ctx, stat, X_iw, X_tau, batch, False)


def gw_mix(ctx, alpha, X_new, Y, want_diff=False):
    """Y <- (1 - alpha) Y + alpha X_new; returns max |X_new - Y_old| when asked."""
    if X_new is not None and X_new.numel() != Y.numel():
        raise ValueError("gw_mix sizes differ")
    d = ctypes.c_double()
    ctx._check(load().gw_mix(ctx.h, int(Y.numel()), float(alpha),
                             _ptr(X_new, "X_new") if X_new is not None else None, _ptr(Y, "Y"),
                             ctypes.byref(d) if want_diff else None), "gw_mix")
    return d.value if want_diff else None


def gw_screened_W(ctx, P0_iw, Pt_iw):
    nq = int(P0_iw.shape[0])
    shp = (nq, ctx.nw_b, ctx.naux, ctx.naux)
    ctx._check(load().gw_screened_W(ctx.h, _ptr(P0_iw, "P0_iw", shp), nq, _ptr(Pt_iw, "Pt_iw", shp)),
               "gw_screened_W")


def gw_screened_W_phi(ctx, P0_iw, Pt_iw):
    """gw_screened_W plus Eq. tilde_Phi_GW over the nq q-points given; returns Phi~."""
    nq = int(P0_iw.shape[0])
    shp = (nq, ctx.nw_b, ctx.naux, ctx.naux)
    out = ctypes.c_double(0.0)
    ctx._check(load().gw_screened_W_phi(ctx.h, _ptr(P0_iw, "P0_iw", shp), nq, _ptr(Pt_iw, "Pt_iw", shp),
                                        ctypes.byref(out)), "gw_screened_W_phi")
    return out.value


def gw_self_energy(ctx, V, G_tau, Pt_tau, q0, nq, Sig_tau):
    ctx._check(load().gw_self_energy(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        _ptr(Pt_tau, "Pt_tau", (nq, ctx.ntau, ctx.naux, ctx.naux)), int(q0), int(nq),
        _ptr(Sig_tau, "Sig_tau", ctx.g_shape())), "gw_self_energy")


def gw_sigma(ctx, V, G_tau, Sig_inf, Sig_tau, gamma=None, P_tau=None, P0_iw=None, Pt_iw=None,
             want_phi=False):
    """One Sigma[G] + Pi evaluation (gw_sigma): Sig_inf, Sig_tau overwritten;
    with P_tau, P0_iw, Pt_iw ([Nk][ntau|nw_b][naux][naux]) P~ is kept there,
    else the chain runs q by q.  Returns Phi~ when want_phi, else None."""
    pt, pw = (ctx.nk, ctx.ntau, ctx.naux, ctx.naux), (ctx.nk, ctx.nw_b, ctx.naux, ctx.naux)
    phi = ctypes.c_double(0.0)
    ctx._check(load().gw_sigma(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        _ptr(gamma, "gamma", ctx.k_shape()), _ptr(Sig_inf, "Sig_inf", ctx.k_shape()),
        _ptr(Sig_tau, "Sig_tau", ctx.g_shape()), _ptr(P_tau, "P_tau", pt), _ptr(P0_iw, "P0_iw", pw),
        _ptr(Pt_iw, "Pt_iw", pw), ctypes.byref(phi) if want_phi else None), "gw_sigma")
    return phi.value if want_phi else None


def gw_sigma_jvp(ctx, V, G_tau, Pt_tau, Pt_iw, dG_tau, dSig_inf, dSig_tau):
    """dSig = J dG of G -> (Sigma_inf, Sigma~); Pt_tau, Pt_iw from gw_sigma, or
    None (P~ rebuilt per q)."""
    pt, pw = (ctx.nk, ctx.ntau, ctx.naux, ctx.naux), (ctx.nk, ctx.nw_b, ctx.naux, ctx.naux)
    ctx._check(load().gw_sigma_jvp(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        _ptr(Pt_tau, "Pt_tau", pt), _ptr(Pt_iw, "Pt_iw", pw), _ptr(dG_tau, "dG_tau", ctx.g_shape()),
        _ptr(dSig_inf, "dSig_inf", ctx.k_shape()), _ptr(dSig_tau, "dSig_tau", ctx.g_shape())),
        "gw_sigma_jvp")


def gw_sigma_vjp(ctx, V, G_tau, Pt_tau, Pt_iw, Sinf_bar, Stau_bar, G_bar):
    """G_bar = J^H (Sinf_bar, Stau_bar) (torch's complex-gradient convention)."""
    pt, pw = (ctx.nk, ctx.ntau, ctx.naux, ctx.naux), (ctx.nk, ctx.nw_b, ctx.naux, ctx.naux)
    ctx._check(load().gw_sigma_vjp(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        _ptr(Pt_tau, "Pt_tau", pt), _ptr(Pt_iw, "Pt_iw", pw),
        _ptr(Sinf_bar, "Sinf_bar", ctx.k_shape()), _ptr(Stau_bar, "Stau_bar", ctx.g_shape()),
        _ptr(G_bar, "G_bar", ctx.g_shape())), "gw_sigma_vjp")


def gw_density(ctx, G_tau, S, gamma, want_count=True):
    n = ctypes.c_double()
    ctx._check(load().gw_density(ctx.h, _ptr(G_tau, "G_tau", ctx.g_shape()),
                                 _ptr(S, "S", ctx.k_shape()), _ptr(gamma, "gamma", ctx.k_shape()),
                                 ctypes.byref(n) if want_count else None), "gw_density")
    return n.value if want_count else None


def gw_hf(ctx, V, G_tau, gamma, Sig_inf):
    ctx._check(load().gw_hf(ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype),
                            _ptr(G_tau, "G_tau", ctx.g_shape()),
                            _ptr(gamma, "gamma", ctx.k_shape()) if gamma is not None else None,
                            _ptr(Sig_inf, "Sig_inf", ctx.k_shape())), "gw_hf")


def gw_dyson_G(ctx, H0, S, Sig_inf, Sig_iw, mu, G_iw):
    ctx._check(load().gw_dyson_G(
        ctx.h, _ptr(H0, "H0", ctx.k_shape()), _ptr(S, "S", ctx.k_shape()),
        _ptr(Sig_inf, "Sig_inf", ctx.k_shape()) if Sig_inf is not None else None,
        _ptr(Sig_iw, "Sig_iw", ctx.giw_shape()) if Sig_iw is not None else None,
        float(mu), _ptr(G_iw, "G_iw", ctx.giw_shape())), "gw_dyson_G")


def gw_find_mu(ctx, H0, S, Sig_inf, Sig_iw, n_target, mu0=0.0, tol=1e-13, G_iw=None, G_tau=None):
    mu = ctypes.c_double(mu0)
    n = ctypes.c_double()
    ctx._check(load().gw_find_mu(
        ctx.h, _ptr(H0, "H0", ctx.k_shape()), _ptr(S, "S", ctx.k_shape()),
        _ptr(Sig_inf, "Sig_inf", ctx.k_shape()) if Sig_inf is not None else None,
        _ptr(Sig_iw, "Sig_iw", ctx.giw_shape()) if Sig_iw is not None else None,
        float(n_target), float(tol), ctypes.byref(mu),
        _ptr(G_iw, "G_iw", ctx.giw_shape()) if G_iw is not None else None,
        _ptr(G_tau, "G_tau", ctx.g_shape()) if G_tau is not None else None,
        ctypes.byref(n)), "gw_find_mu")
    return mu.value, n.value


class Thermo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("omega", "phi_inf", "phi_tilde", "tr_ln", "tr_sigma_g",
                                                "e_one_body", "e_gm", "n_e")]


def gw_thermodynamics(ctx, H0, S, Sig_inf, Sig_iw, mu, phi_tilde):
    """Grand potential (Eq. GP), its parts and the Galitskii-Migdal energy, as a dict."""
    t = Thermo()
    ctx._check(load().gw_thermodynamics(
        ctx.h, _ptr(H0, "H0", ctx.k_shape()), _ptr(S, "S", ctx.k_shape()),
        _ptr(Sig_inf, "Sig_inf", ctx.k_shape()), _ptr(Sig_iw, "Sig_iw", ctx.giw_shape()),
        float(mu), float(phi_tilde), ctypes.byref(t)), "gw_thermodynamics")
    return {n: getattr(t, n) for n, _ in Thermo._fields_}


def gw_synchronize(ctx):
    ctx._check(load().gw_synchronize(ctx.h), "gw_synchronize")


def gw_profile_enable(ctx, on=True):
    ctx._check(load().gw_profile_enable(ctx.h, 1 if on else 0), "gw_profile_enable")


def gw_profile_read(ctx, kclass):
    """(launches, milliseconds, algorithmic flops) of one kernel class."""
    n, ms, fl = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
    ctx._check(load().gw_profile_read(ctx.h, int(kclass), ctypes.byref(n), ctypes.byref(ms),
                                      ctypes.byref(fl)), "gw_profile_read")
    return n.value, ms.value, fl.value


# ----------------------------------------------------------- derivatives ---
def gw_polarization2(ctx, V, G_a, G_b, q0, nq, P0_tau, accumulate=False):
    ctx._check(load().gw_polarization2(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_a, "G_a", ctx.g_shape()),
        _ptr(G_b, "G_b", ctx.g_shape()), int(q0), int(nq), 1 if accumulate else 0,
        _ptr(P0_tau, "P0_tau", (nq, ctx.ntau, ctx.naux, ctx.naux))), "gw_polarization2")


def gw_screened_W_lin(ctx, Pt_iw, X_iw, Y_iw, adjoint=False):
    nq = int(Pt_iw.shape[0])
    shp = (nq, ctx.nw_b, ctx.naux, ctx.naux)
    ctx._check(load().gw_screened_W_lin(ctx.h, _ptr(Pt_iw, "Pt_iw", shp), _ptr(X_iw, "X_iw", shp), nq,
                                        1 if adjoint else 0, _ptr(Y_iw, "Y_iw", shp)),
               "gw_screened_W_lin")


def gw_transform_adjoint(ctx, stat, inverse, X_in, X_out, batch=1):
    """inverse=False: cotangent of gw_tau_to_iw's output [b][nw][..] -> its input [b][ntau][..];
    inverse=True: cotangent of gw_iw_to_tau's output [b][ntau][..] -> input [b][nw][..]."""
    nw = ctx.nw_f if stat == GW_FERMION else ctx.nw_b
    nin, nout = (nw, ctx.ntau) if not inverse else (ctx.ntau, nw)
    R = X_in.numel() // (batch * nin)
    if X_in.numel() != batch * nin * R or X_out.numel() != batch * nout * R:
        raise ValueError("adjoint transform shapes do not match")
    ctx._check(load().gw_transform_adjoint(ctx.h, int(stat), 1 if inverse else 0, _ptr(X_in, "X_in"),
                                           int(batch), int(R), _ptr(X_out, "X_out")),
               "gw_transform_adjoint")


def gw_self_energy_vjp(ctx, V, G_tau, Pt_tau, Sig_bar, q0, nq, G_bar, Pt_bar):
    shp = (nq, ctx.ntau, ctx.naux, ctx.naux)
    ctx._check(load().gw_self_energy_vjp(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        _ptr(Pt_tau, "Pt_tau", shp), _ptr(Sig_bar, "Sig_bar", ctx.g_shape()), int(q0), int(nq),
        _ptr(G_bar, "G_bar", ctx.g_shape()), _ptr(Pt_bar, "Pt_bar", shp)), "gw_self_energy_vjp")


def gw_polarization_vjp(ctx, V, G_tau, P0_bar, q0, nq, G_bar):
    ctx._check(load().gw_polarization_vjp(
        ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype), _ptr(G_tau, "G_tau", ctx.g_shape()),
        _ptr(P0_bar, "P0_bar", (nq, ctx.ntau, ctx.naux, ctx.naux)), int(q0), int(nq),
        _ptr(G_bar, "G_bar", ctx.g_shape())), "gw_polarization_vjp")


def gw_hf_vjp(ctx, V, Sinf_bar, G_bar):
    ctx._check(load().gw_hf_vjp(ctx.h, _ptr(V, "V", ctx.v_shape(), ctx.v_dtype),
                                _ptr(Sinf_bar, "Sinf_bar", ctx.k_shape()),
                                _ptr(G_bar, "G_bar", ctx.g_shape())), "gw_hf_vjp")


def gw_dyson_jvp(ctx, S, G_iw, dSinf, dSig_iw, dG_iw, fixed_mu=False):
    dmu = ctypes.c_double()
    ctx._check(load().gw_dyson_jvp(
        ctx.h, _ptr(S, "S", ctx.k_shape()), _ptr(G_iw, "G_iw", ctx.giw_shape()),
        _ptr(dSinf, "dSinf", ctx.k_shape()) if dSinf is not None else None,
        _ptr(dSig_iw, "dSig_iw", ctx.giw_shape()) if dSig_iw is not None else None,
        1 if fixed_mu else 0, _ptr(dG_iw, "dG_iw", ctx.giw_shape()), ctypes.byref(dmu)),
        "gw_dyson_jvp")
    return dmu.value


def gw_axpby(ctx, a, X, b, Y):
    """Y = a X + b Y (complex scalars a, b)."""
    a, b = complex(a), complex(b)
    if X is not None and X.numel() != Y.numel():
        raise ValueError("gw_axpby sizes differ")
    ctx._check(load().gw_axpby(ctx.h, int(Y.numel()), a.real, a.imag,
                               _ptr(X, "X") if X is not None else None, b.real, b.imag,
                               _ptr(Y, "Y")), "gw_axpby")


def gw_dot(ctx, X, Y):
    """sum conj(X) Y as a Python complex."""
    if X.numel() != Y.numel():
        raise ValueError("gw_dot sizes differ")
    out = (ctypes.c_double * 2)()
    ctx._check(load().gw_dot(ctx.h, int(X.numel()), _ptr(X, "X"), _ptr(Y, "Y"), out), "gw_dot")
    return complex(out[0], out[1])
