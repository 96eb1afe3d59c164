"""Seeded synthetic inputs for the density-fitted GW hot path.

This module draws random numbers and lays them out; it holds none of the
method's arithmetic.  Both the HIP path and the CPU oracle are fed from here.

Recipe (paper Sec. II-III; the paper's PySCF integrals are replaced by draws):
  * H0(k) = U_k diag(eps_k) U_k^dagger with U_k Haar-random (QR of a complex
    Gaussian matrix, phases fixed) and eps_k drawn per band group.
  * S(k) = I by default, or a random Hermitian positive-definite matrix.
  * V^{k1,k2}_{ij}(Q): circular complex Gaussian entries, E|z|^2 = sigma^2,
    with V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger for every Q (the Hermiticity of the
    Gaussian density-fitting tensor, Eqs. VijQ-DF_J).  Stored as
    V[q][k][Q][i][j] = V^{k, k+q}_{ij}(Q).  Every (k1,k2) pair is drawn from
    its own counter-seeded stream, so any q-slab can be produced alone.
"""
from __future__ import annotations

import dataclasses
import numpy as np


# ----------------------------------------------------------------- k-mesh ---
def mesh_points(mesh):
    """Integer coordinates (Nk, 3) of a Gamma-centred mesh, k = (i1*n2+i2)*n3+i3."""
    n1, n2, n3 = mesh
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    return g.reshape(-1, 3)


def _mesh_index(pts, mesh):
    n1, n2, n3 = mesh
    return (pts[..., 0] % n1 * n2 + pts[..., 1] % n2) * n3 + pts[..., 2] % n3


def _shift(mesh):
    """plus[q, k] = index of k+q; minus[q] = index of -q (layout helpers only)."""
    p = mesh_points(mesh)
    plus = _mesh_index(p[:, None, :] + p[None, :, :], mesh)
    neg = _mesh_index(-p, mesh)
    return plus, neg


# ------------------------------------------------------------ random parts ---
def haar_unitary(rng, n):
    z = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))[None, :]


def circular_gaussian(rng, shape, sigma):
    s = sigma / np.sqrt(2.0)
    return rng.standard_normal(shape) * s + 1j * (rng.standard_normal(shape) * s)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload.  `bands` lists (count, lo, hi) groups of H0
    eigenvalues in Hartree; the remaining bands (if any) use the last group."""
    name: str
    mesh: tuple
    nao: int
    naux: int
    ntau: int
    beta: float
    seed: int
    bands: tuple = ((None, -1.0, 1.0),)
    sigma: float = 0.1
    ns: int = 2
    n_target: float | None = None
    s_kind: str = "identity"
    mu0: float = 0.0

    @property
    def nk(self):
        return int(np.prod(self.mesh))

    @property
    def nw_f(self):
        return self.ntau

    @property
    def nw_b(self):
        return self.ntau + 1


WORKLOADS = {
    # oracle-size FP64 case: 2x2x2, nao 6, naux 24, ntau 24, beta 50
    "tiny-2x2x2": Workload("tiny-2x2x2", (2, 2, 2), 6, 24, 24, 50.0, 1,
                           ((None, -1.0, 1.0),), 0.1, 2, 6.0),
    # Si-like FP64 scGW: 4x4x4, nao 26, naux 250, ntau 100, beta 100, 8 e/cell
    "si-4x4x4": Workload("si-4x4x4", (4, 4, 4), 26, 250, 100, 100.0, 2,
                         ((4, -1.0, -0.2), (None, 0.1, 3.0)),
                         0.1 * np.sqrt(24.0 / 250.0), 2, 8.0),
    # differentiation case: 3x3x3, nao 16, naux 150, ntau 60, beta 100
    "ad-3x3x3": Workload("ad-3x3x3", (3, 3, 3), 16, 150, 60, 100.0, 4,
                         ((4, -1.0, -0.2), (None, 0.1, 3.0)),
                         0.1 * np.sqrt(24.0 / 150.0), 2, 8.0),
    # large mixed case: 5x5x5, nao 26, naux 300, ntau 120, beta 200
    "si-5x5x5": Workload("si-5x5x5", (5, 5, 5), 26, 300, 120, 200.0, 5,
                         ((4, -1.0, -0.2), (None, 0.1, 3.0)),
                         0.1 * np.sqrt(24.0 / 300.0), 2, 8.0),
}


def band_energies(rng, nao, bands):
    out = []
    left = nao
    for cnt, lo, hi in bands:
        c = left if cnt is None else min(cnt, left)
        out.append(rng.uniform(lo, hi, size=c))
        left -= c
        if left == 0:
            break
    return np.sort(np.concatenate(out))


def make_H0(wl: Workload, rng=None):
    rng = np.random.default_rng([wl.seed, 11]) if rng is None else rng
    H = np.empty((wl.nk, wl.nao, wl.nao), np.complex128)
    for k in range(wl.nk):
        U = haar_unitary(rng, wl.nao)
        e = band_energies(rng, wl.nao, wl.bands)
        h = (U * e[None, :]) @ U.conj().T
        H[k] = 0.5 * (h + h.conj().T)
    return H


def make_S(wl: Workload, rng=None, kind=None):
    kind = wl.s_kind if kind is None else kind
    S = np.empty((wl.nk, wl.nao, wl.nao), np.complex128)
    if kind == "identity":
        S[:] = np.eye(wl.nao)
        return S
    rng = np.random.default_rng([wl.seed, 12]) if rng is None else rng
    for k in range(wl.nk):
        A = circular_gaussian(rng, (wl.nao, wl.nao), 0.15)
        S[k] = np.eye(wl.nao) + 0.5 * (A @ A.conj().T) / wl.nao
        S[k] = 0.5 * (S[k] + S[k].conj().T)
    return S


def _pair_block(seed, canon, naux, nao, sigma, hermitian):
    rng = np.random.default_rng([seed, 13, int(canon)])
    R = circular_gaussian(rng, (naux, nao, nao), sigma)
    if hermitian:
        R = (R + np.conj(np.swapaxes(R, 1, 2))) / np.sqrt(2.0)
    return R


def make_V_slab(wl: Workload, q, dtype=np.complex128):
    """V[q] with shape (Nk, naux, nao, nao): V[q][k][Q] = V^{k,k+q}(Q)."""
    plus, neg = _shift(wl.mesh)
    nk = wl.nk
    out = np.empty((nk, wl.naux, wl.nao, wl.nao), dtype)
    for k in range(nk):
        k2 = plus[q, k]
        me = q * nk + k                 # (q, k) holds V^{k,k2}
        partner = neg[q] * nk + k2      # (-q, k2) holds V^{k2,k}
        if me == partner:               # q = 0: V^{kk}(Q) is Hermitian
            out[k] = _pair_block(wl.seed, me, wl.naux, wl.nao, wl.sigma, True)
        elif me < partner:
            out[k] = _pair_block(wl.seed, me, wl.naux, wl.nao, wl.sigma, False)
        else:
            out[k] = np.conj(np.swapaxes(
                _pair_block(wl.seed, partner, wl.naux, wl.nao, wl.sigma, False), 1, 2))
    return out


def make_V(wl: Workload, dtype=np.complex128):
    """Full V[q][k][Q][i][j] (Nk, Nk, naux, nao, nao)."""
    return np.stack([make_V_slab(wl, q, dtype) for q in range(wl.nk)])


def random_hermitian_tau(rng, ntau, nk, n, scale=0.1):
    """Random data X[t][k] that is Hermitian at every (t, k) (test inputs)."""
    A = circular_gaussian(rng, (ntau, nk, n, n), scale)
    return np.ascontiguousarray(0.5 * (A + np.conj(np.swapaxes(A, -1, -2))))


def small_workload(name="small", mesh=(2, 2, 2), nao=10, naux=70, ntau=20, beta=20.0,
                   seed=7, sigma=0.1, ns=2, n_target=None, s_kind="identity", bands=None):
    bands = ((None, -1.0, 1.0),) if bands is None else bands
    nt = float(nao) if n_target is None else n_target
    return Workload(name, tuple(mesh), nao, naux, ntau, float(beta), seed, bands, sigma,
                    ns, nt, s_kind)
