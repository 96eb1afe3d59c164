/*
 * gw.h -- C ABI of the MI355X density-fitted GW hot path (libgw.so).
 *
 * The library evaluates the dynamical GW self-energy of a periodic solid in a
 * Gaussian Bloch-orbital basis with density-fitted Coulomb integrals, after
 * Yeh, Iskakov, Zgid and Gull, "Fully self-consistent finite-temperature GW
 * in Gaussian Bloch orbitals for solids" (Sec. III and Algorithm 1), together
 * with the imaginary-time / Matsubara transforms, the Hartree-Fock part, the
 * Dyson equation and the chemical-potential search of the scGW loop (Sec. IV.A).
 *
 * Conventions shared by every call
 * --------------------------------
 * Pointers.  Unless a parameter says "host", an array pointer is a DEVICE
 *   pointer owned by the caller; the library never frees it.  Complex numbers
 *   are interleaved (re, im) doubles (gw_z).  Arrays are row-major:
 *     G, Sigma~, X_tau      [tau][k][i][j]           (ntau, Nk, nao, nao)
 *     G(iw), Sigma~(iw)     [n][k][i][j]             (nw_f, Nk, nao, nao)
 *     V                     [q][k][Q][i][j] = V^{k,k+q}_{ij}(Q)  (Nk, Nk, naux, nao, nao)
 *     P0, P~ (tau)          [q][tau][Q][Q']          (nq, ntau, naux, naux)
 *     P0, P~ (i Omega)      [q][m][Q][Q']            (nq, nw_b, naux, naux)
 *     H0, S, Sigma_inf      [k][i][j]                (Nk, nao, nao)
 *   k = (i1 * n2 + i2) * n3 + i3 on a Gamma-centred n1 x n2 x n3 mesh; k+q and
 *   k-q are taken component-wise modulo the mesh.  V must satisfy
 *   V^{k2,k1}(Q) = V^{k1,k2}(Q)^dagger (Hermiticity of the Gaussian density
 *   fitting, Eqs. VijQ-DF_J); the library reads V^{k+q,k} as the conjugate
 *   transpose of the stored V^{k,k+q}.
 * Streams.  Every call enqueues its kernels on the hipStream_t given to
 *   gw_create and returns without waiting, except where a call says that it
 *   synchronises (gw_screened_W, gw_dyson_G, gw_find_mu and gw_get_grids
 *   synchronise to report pivots and scalars).
 * Errors.  Every call returns gw_status.  Argument errors are found on the
 *   host before anything is launched, and nothing is written.  The text of the
 *   last error of a context is returned by gw_last_error.  No C++ exception
 *   crosses this interface.  An empty range (nq = 0, batch = 0 or R = 0) is
 *   a no-op that accepts NULL arrays.
 * Memory.  The library owns the context: the dimensions, the grid tables and
 *   the k+q tables (device copies made by gw_create / gw_build_grids).  All
 *   other scratch memory is the caller's, handed over by gw_set_workspace and
 *   sized by gw_workspace_bytes.
 * Spin.  Spin-restricted: ns (1 or 2) multiplies the polarization, the
 *   Hartree term and the electron count; exchange and Sigma~ carry no spin sum.
 * Environment (read by gw_create).  GW_DEBUG_BOUNDS=1 makes every call check
 *   on the host, before launching, that each GEMM descriptor it builds stays
 *   inside the extents of its operands (a failed check returns GW_ERR_ARG);
 *   GW_TILE_CFG=0..9 forces the tile shape of the two large fp64
 *   contractions (measurement only): 0..4 the four-product complex MFMA form,
 *   5..9 the three-product (Gauss) form (defaults: 0 for the polarization,
 *   7 for the self-energy); the Hermitian polarization needs a square shape:
 *   0, 4 or 5.  GW_PROD_TILES=1 runs the fp32 producers on the tiled GEMM
 *   instead of the streaming kernel.  GW_SPLIT_CFG selects split-bf16 tiles:
 *   bf16x3 self-energy 0 = 128x128 (default), 1 = 64x64, 2 = 128x64; bf16x6
 *   1 = two LDS stages instead of one.  GW_SPLIT_GROUP=g > 0 walks the
 *   split-bf16 tiles in groups of g over the tau batch.  All of these are
 *   for measurement only.
 */
#ifndef GW_H
#define GW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } gw_z;

typedef enum {
  GW_OK = 0,
  GW_ERR_ARG = 1,        /* bad dimension, null pointer, out-of-range index  */
  GW_ERR_DEVICE = 2,     /* a HIP runtime call failed                        */
  GW_ERR_SINGULAR = 3,   /* a zero pivot in a Dyson solve                    */
  GW_ERR_NOCONV = 4,     /* mu search did not bracket or converge            */
  GW_ERR_WORKSPACE = 5,  /* workspace missing or too small                   */
  GW_ERR_STATE = 6,      /* call made before gw_build_grids / gw_set_grids   */
  GW_ERR_NONFINITE = 7   /* a NaN or Inf met where a finite value is needed  */
} gw_status;

enum { GW_FERMION = 0, GW_BOSON = 1 };

/* Contraction precision of the polarization and self-energy chains.
 * GW_PREC_FP64: everything in fp64, V complex128.
 * GW_PREC_FP32: mixed precision.  V is stored complex64 (gw_c); in
 *   gw_polarization and gw_self_energy G is rounded to complex64, the
 *   products run as complex fp32 MFMA GEMMs with their intermediates in
 *   complex64, and the long contraction sums add each 512-term chunk
 *   accumulated in fp32 into fp64; their outputs (P0, Sigma~) are
 *   complex128.  gw_hf reads the complex64 V in fp64 arithmetic; the
 *   transforms, both Dyson solves and the mu search are fp64 as in
 *   GW_PREC_FP64.
 * GW_PREC_BF16X3: as GW_PREC_FP32, except that the two large contractions
 *   (sum over (k, d, b) of Eq. tilde_P0_tau, and P~ V of Eq. tilde_sigma2)
 *   run on bf16 MFMA with split operands: each real operand x is held as
 *   hi + lo, hi = bf16(x), lo = bf16(x - hi), and each real product as
 *   a_hi b_hi + a_hi b_lo + a_lo b_hi (relative error near 2^-16 per
 *   product), with fp32 accumulation; the polarization's long K is summed
 *   as 512-term fp32 chunks added in fp32 (rounding near 1e-7 relative).
 * GW_PREC_BF16X6: as GW_PREC_BF16X3 with three levels, x = hi + mid + lo,
 *   and the six level products up to second order (relative error near
 *   2^-24, that of fp32), fp32 chunks added in fp64.                      */
enum { GW_PREC_FP64 = 0, GW_PREC_FP32 = 1, GW_PREC_BF16X3 = 2, GW_PREC_BF16X6 = 3 };
typedef struct { float re, im; } gw_c;

typedef struct {
  int mesh[3];     /* n1, n2, n3 >= 1; Nk = n1 n2 n3                          */
  int nao;         /* orbitals per cell, 1..60                                */
  int naux;        /* auxiliary functions Q, >= 1                             */
  int ntau;        /* imaginary-time nodes, even, 2..512                      */
  int nw_f;        /* fermionic sparse frequencies, ntau..4 ntau (gw_build_grids:
                      exactly ntau)                                           */
  int nw_b;        /* bosonic sparse frequencies, ntau..4 ntau + 1 (gw_build_grids:
                      exactly ntau + 1)                                       */
  int ns;          /* spin factor, 1 or 2                                     */
  int precision;   /* GW_PREC_*                                               */
  double beta;     /* inverse temperature (1/Ha), > 0                         */
} gw_dims;

typedef struct gw_ctx gw_ctx;

/* Create a context bound to the current HIP device and to hip_stream (a
 * hipStream_t; NULL means the default stream).  Validates d (GW_ERR_ARG).  */
gw_status gw_create(const gw_dims* d, void* hip_stream, gw_ctx** out);
gw_status gw_destroy(gw_ctx* ctx);

/* Build the discretisation on the host and copy it to the device.
 *   tau nodes: roots of the Chebyshev polynomial T_ntau mapped to [0, beta],
 *     mirrored so that tau_{ntau-1-i} = beta - tau_i (G(beta - tau_i) is node
 *     ntau-1-i).
 *   transforms: T[n][i] = int_0^beta L_i(tau) exp(i nu_n tau) d tau, L_i the
 *     Lagrange polynomials of the nodes (Eqs. tau_to_iw and P0t_to_P0w of the
 *     paper applied to the interpolant); the inverse transforms (Eqs.
 *     iw_to_tau and Piw_to_Pt) are the least-squares inverses of T.
 *   frequencies: fermionic omega_n = (2n+1) pi / beta, bosonic Omega_m =
 *     2 m pi / beta.  nF (nw_f entries) and nB (nw_b entries), host arrays of
 *     Matsubara indices, may be given; NULL selects them greedily: symmetric
 *     pairs {n, -n-1} (fermionic) or {0} then {m, -m} (bosonic) among
 *     0 <= n < 4 ntau, each time the pair whose transform rows keep the
 *     largest residual after the rows already chosen are projected out
 *     (ties within a relative 1e-9 go to the smallest n).  Sets are returned
 *     sorted ascending.
 *   density row: w_i = L_i(beta), so gamma = -G(beta^-) = -sum_i w_i G(tau_i).
 * Host-only arithmetic; synchronises once for the uploads.                  */
gw_status gw_build_grids(gw_ctx* ctx, const long long* nF, const long long* nB);

/* Install caller-built grid tables in place of gw_build_grids (Sec. IV.C:
 * any sparse representation on the imaginary axes whose tables have these
 * meanings, e.g. an intermediate-representation basis with its sampling
 * points).  All arrays are HOST arrays, row-major, copied by the call:
 *   tau[ntau]        nodes in (0, beta), strictly increasing and mirrored,
 *                    |tau_{ntau-1-i} - (beta - tau_i)| <= 1e-12 beta (the
 *                    polarization reads G(beta - tau_i) as node ntau-1-i)
 *   nF[nw_f], nB[nw_b]  Matsubara indices (omega_n = (2n+1) pi / beta,
 *                    Omega_m = 2 m pi / beta), strictly increasing
 *   TF[nw_f*ntau], TB[nw_b*ntau]     tau -> i w transforms (Eqs. tau_to_iw,
 *                    P0t_to_P0w): X(i w_n) = sum_i T[n][i] X(tau_i)
 *   TFp[ntau*nw_f], TBp[ntau*nw_b]   i w -> tau fits (Eqs. iw_to_tau,
 *                    Piw_to_Pt): X(tau_i) = sum_n Tp[i][n] X(i w_n)
 *   w[ntau]          density row: gamma = -G(beta^-) = -sum_i w_i G(tau_i)
 * Non-finite entries or violated orderings are GW_ERR_ARG (nothing is
 * changed).  The electron-count row r = w TFp and the frequency values are
 * derived here.  Synchronises once for the uploads.                         */
gw_status gw_set_grids(gw_ctx* ctx, const double* tau, const long long* nF, const long long* nB,
                       const gw_z* TF, const gw_z* TFp, const gw_z* TB, const gw_z* TBp,
                       const double* w);

/* Intermediate-representation (IR) grids with sparse sampling on both axes
 * (Sec. IV.C: dynamical quantities expanded in the IR basis, its cutoff
 * lambda chosen above beta times the bandwidth, sampled sparsely in tau and
 * in Matsubara frequency).  Host-only arithmetic:
 *   basis: the singular-value expansion of the logistic kernel
 *     K(x, y) = exp(-lambda y (x + 1) / 2) / (1 + exp(-lambda y)) on
 *     x = 2 tau / beta - 1, y = omega / omega_max, lambda = beta omega_max
 *     (one basis for fermionic and bosonic functions), by an SVD on composite
 *     Gauss-Legendre rules; L = the number of singular values above eps times
 *     the largest, rounded up to even; basis functions by the Nystrom
 *     extension, whose Matsubara transforms are closed forms;
 *   tau nodes: the L roots of the first basis function left out (mirrored:
 *     tau_{L-1-i} = beta - tau_i);
 *   Matsubara sets: symmetric pairs chosen greedily by the largest residual
 *     of their (column-scaled) transform rows among |n| < 4 lambda / pi + 4 L:
 *     L fermionic, L + 1 bosonic;
 *   tables: T = Uhat U(tau)^{-1}, Tp = U(tau) Uhat^+, density row
 *     w = u(beta) U(tau)^{-1}.
 * gw_ir_size returns L for (lambda, eps) (lambda in 1..1e5, eps in
 * 1e-14..1e-2; otherwise GW_ERR_ARG); a context for IR grids is created with
 * ntau = L, nw_f = L, nw_b = L + 1.  gw_ir_grids_host fills HOST arrays of
 * the sizes of gw_get_grids (each may be NULL) without a context;
 * gw_build_ir_grids installs the tables in a context whose dims match
 * (GW_ERR_ARG otherwise) and synchronises once for the uploads.  The
 * expansion is cached per (lambda, eps) for the life of the process.        */
gw_status gw_ir_size(double lambda, double eps, int* ntau);
gw_status gw_ir_grids_host(double beta, double lambda, double eps, int ntau, double* tau, long long* nF,
                           long long* nB, gw_z* TF, gw_z* TFp, gw_z* TB, gw_z* TBp, double* w);
gw_status gw_build_ir_grids(gw_ctx* ctx, double lambda, double eps);

/* Copy the host tables out (each pointer is a HOST array and may be NULL):
 * tau[ntau], nF[nw_f], nB[nw_b], TF[nw_f*ntau], TFp[ntau*nw_f],
 * TB[nw_b*ntau], TBp[ntau*nw_b] (row-major), w[ntau].                       */
gw_status gw_get_grids(const gw_ctx* ctx, double* tau, long long* nF, long long* nB,
                       gw_z* TF, gw_z* TFp, gw_z* TB, gw_z* TBp, double* w);

/* Host-only form of gw_build_grids for inspection and testing: builds the
 * same tables for (beta, ntau) without a context or a GPU.  nF / nB as in
 * gw_build_grids (NULL selects them); every output is a HOST array of the
 * size given for gw_get_grids and may be NULL.                              */
gw_status gw_grids_host(double beta, int ntau, const long long* nF, const long long* nB,
                        double* tau, long long* nF_out, long long* nB_out, gw_z* TF, gw_z* TFp,
                        gw_z* TB, gw_z* TBp, double* w);

/* Workspace.  gw_workspace_bytes returns the bytes a call needs: op is one of
 * GW_OP_*; for the chains, tau_chunk (1..ntau) is how many tau nodes are
 * processed per pass (memory grows linearly with it); for GW_OP_SCREENED_W,
 * tau_chunk is read as nq; GW_OP_SIGMA (gw_sigma, gw_sigma_jvp,
 * gw_sigma_vjp) is the largest of the chain, Hartree-Fock and one-q
 * screened-interaction needs plus six per-q polarization buffers.  gw_set_workspace hands over a device buffer
 * (caller-owned, >= 256-byte aligned) and the tau chunk to use; calls that
 * need more than that buffer return GW_ERR_WORKSPACE.                       */
enum { GW_OP_POLARIZATION = 0, GW_OP_SELF_ENERGY = 1, GW_OP_SCREENED_W = 2, GW_OP_HF = 3,
       GW_OP_DYSON_JVP = 4, GW_OP_SIGMA = 5, GW_OP_THERMO = 6 };
size_t gw_workspace_bytes(const gw_ctx* ctx, int op, int tau_chunk);
gw_status gw_set_workspace(gw_ctx* ctx, void* dev, size_t bytes, int tau_chunk);

/* Eq. tilde_P0_tau (reading: G(-tau) of the bubble is the stored G(beta -
 * tau), sign chosen so that the static bubble is negative semidefinite):
 *   P0^q_{QQ'}(tau_i) = -(ns/Nk) sum_k sum_{abcd} V^{k,k+q}_{da}(Q) G^{k+q}_{ab}(tau_i)
 *                       V^{k+q,k}_{bc}(Q') G^k_{cd}(tau_{ntau-1-i})
 * for q = q0 .. q0+nq-1, written to P0_tau[q-q0][i] (overwritten).          */
gw_status gw_polarization(gw_ctx* ctx, const void* V, const gw_z* G_tau, int q0, int nq,
                          gw_z* P0_tau);   /* V: gw_z (GW_PREC_FP64) or gw_c (the other modes) */

/* gw_polarization for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result, with the chain's intermediates in a fixed scratch array of
 * 128 MiB that the library holds on each GPU until the process ends, instead
 * of the caller's workspace.  The call allocates nothing: no hipMalloc,
 * hipFree or allocating library routine, and no profiling events (launches
 * made through it are not counted by gw_profile_read).  The tau chunk is the
 * largest that fits the scratch; if one tau slice of the intermediates does
 * not fit (fp64: 32 Nk naux nao^2 bytes > 128 MiB; fp32: 16 Nk naux nao^2 +
 * 16 ntau Nk nao^2 bytes; bf16x3 about the fp32 figure plus 8 Nk nao^2
 * naux' + 8 naux naux', naux' = naux rounded up to 32) the call returns GW_ERR_WORKSPACE and launches
 * nothing.  Every call on one GPU shares that GPU's scratch, whatever the
 * context: calls that overlap in time on one GPU (different streams or host
 * threads) race and give undefined results.  Other arguments and errors as
 * gw_polarization.                                                          */
gw_status gw_polarization_noalloc(gw_ctx* ctx, const void* V, const gw_z* G_tau, int q0, int nq,
                                  gw_z* P0_tau);

/* Hermitian mode of the polarization (off after gw_create).  mode is a bit
 * set: GW_HERM_FORWARD states that every G_tau passed to gw_polarization is
 * Hermitian in its orbital indices at each tau and k (true of the Green's
 * function of a Hermitian H0, S and Sigma); GW_HERM_TWO_SLOT states the same
 * of both G_a and G_b of every gw_polarization2 call (true of G and of the
 * Dyson response dG to a Hermitian dSigma).  With V^{k+q,k}(Q) =
 * V^{k,k+q}(Q)^H (Eq. tilde_P0_tau's pair relation), the conjugate of the
 * bubble trace for (Q, Q') is then the trace for (Q', Q), so P0^q(tau) (and
 * each two-slot term) is Hermitian: only the output tiles on and above the
 * diagonal are contracted and the rest is filled by conjugation (also when
 * accumulating, where the previous contents must be Hermitian as well).
 * Results for inputs that break these properties are undefined.          */
enum { GW_HERM_FORWARD = 1, GW_HERM_TWO_SLOT = 2 };
gw_status gw_set_hermitian(gw_ctx* ctx, int mode);

/* Eqs. tau_to_iw / P0t_to_P0w: X_iw[b][n][r] = sum_i T[n][i] X_tau[b][i][r]
 * for b < batch, r < R, with T the fermionic (stat = GW_FERMION, nw = nw_f)
 * or bosonic (GW_BOSON, nw = nw_b) transform.  X_iw is overwritten.          */
gw_status gw_tau_to_iw(gw_ctx* ctx, int stat, const gw_z* X_tau, long long batch, long long R,
                       gw_z* X_iw);

/* Eqs. iw_to_tau / Piw_to_Pt as least-squares fits:
 * X_tau[b][i][r] = sum_n Tp[i][n] X_iw[b][n][r].                            */
gw_status gw_iw_to_tau(gw_ctx* ctx, int stat, const gw_z* X_iw, long long batch, long long R,
                       gw_z* X_tau);

/* Eq. tilde_P_omega with I the identity: for each of the nq * nw_b matrices,
 * Pt_iw = [I - P0_iw]^{-1} P0_iw, by LU with partial pivoting (never by the
 * geometric series).  Pt_iw may not alias P0_iw.  Synchronises; a zero pivot
 * returns GW_ERR_SINGULAR (the outputs are then undefined).                  */
gw_status gw_screened_W(gw_ctx* ctx, const gw_z* P0_iw, int nq, gw_z* Pt_iw);

/* gw_screened_W plus the dynamical Luttinger-Ward term of the same
 * factorisation, Eq. tilde_Phi_GW:
 *   *phi = (1/(2 Nk)) sum_{q < nq} (1/beta) sum_n tr{ln[I - P0^q(i W_n)] + P0^q(i W_n)}
 * (host double; the q given are the first nq of the P0_iw array, so q ranges
 * add up).  Phi is real and F(-iW) = conj F(iW) on the symmetric sparse sets,
 * so only Re F = ln|det(I - P0)| + Re tr P0 enters, with ln|det| from the
 * diagonal of U.  The sum over all bosonic frequencies is the value at tau = 0
 * of the bosonic function whose transform is F: the least-squares fit on the
 * tau nodes evaluated at tau = 0 (weights: the beta^- row reversed, by the
 * mirrored nodes, times the inverse bosonic transform, real part).
 * Synchronises; errors as gw_screened_W (then *phi = 0).                  */
gw_status gw_screened_W_phi(gw_ctx* ctx, const gw_z* P0_iw, int nq, gw_z* Pt_iw, double* phi);

/* Eq. tilde_sigma2, ACCUMULATED over q = q0 .. q0+nq-1 (Pt_tau[q-q0] holds
 * P~^q(tau)):
 *   Sig_tau^k_{ij}(tau) += -(1/Nk) sum_q sum_{ab} sum_{QQ'} G^{k-q}_{ab}(tau)
 *                          V^{k,k-q}_{ia}(Q) P~^q_{QQ'}(tau) V^{k-q,k}_{bj}(Q')
 * Callers zero Sig_tau before the first q-batch.                            */
gw_status gw_self_energy(gw_ctx* ctx, const void* V, const gw_z* G_tau, const gw_z* Pt_tau,
                         int q0, int nq, gw_z* Sig_tau);   /* V as in gw_polarization */

/* Density matrix and electron count (Sec. III): gamma^k = -G^k(beta^-) =
 * -sum_i w_i G^k(tau_i); N_e = (ns/Nk) sum_k Re tr[gamma^k S^k].  gamma is a
 * device array [k][i][j]; n_out (host, may be NULL) synchronises.            */
gw_status gw_density(gw_ctx* ctx, const gw_z* G_tau, const gw_z* S, gw_z* gamma, double* n_out);

/* Eqs. HF_J and HF_K with gamma^k = -G^k(beta^-):
 *   J^k = sum_Q v_Q V^{kk}(Q),  v_Q = (ns/Nk) sum_k' tr[gamma^k' V^{k'k'}(Q)]
 *   K^k = -(1/Nk) sum_q sum_Q V^{k,k+q}(Q) gamma^{k+q} V^{k+q,k}(Q)
 * Sig_inf = J + K is overwritten; gamma (may be NULL) receives gamma.        */
gw_status gw_hf(gw_ctx* ctx, const void* V, const gw_z* G_tau, gw_z* gamma, gw_z* Sig_inf);

/* Eq. Dyson: G^k(i w_n) = [(i w_n + mu) S^k - H0^k - Sig_inf^k - Sig_iw^k(i w_n)]^{-1}
 * for every sparse fermionic n and every k, by Gauss-Jordan elimination with
 * partial pivoting.  Sig_inf and Sig_iw may be NULL (zero).  Synchronises; a
 * zero pivot returns GW_ERR_SINGULAR.                                       */
gw_status gw_dyson_G(gw_ctx* ctx, const gw_z* H0, const gw_z* S, const gw_z* Sig_inf,
                     const gw_z* Sig_iw, double mu, gw_z* G_iw);

/* Chemical potential for a fixed electron count (Sec. IV.A): bisection on
 * N_e(mu) = n_target, N_e from gw_dyson_G and gamma = -G(beta^-).  The bracket
 * starts at *mu_inout +/- 1 Ha and doubles outward until it holds the root;
 * bisection stops when it is narrower than tol (Ha; tol <= 0 means 1e-13).
 * On return *mu_inout is the midpoint, G_iw (may be NULL) holds G at that mu,
 * G_tau (may be NULL) its transform to the tau nodes, *n_out (may be NULL)
 * the electron count there.  n_target outside (0, ns*nao) is GW_ERR_ARG; a
 * bracket that cannot be found, or a bisection that cannot narrow the
 * bracket to tol within 400 halvings (tol below the spacing of doubles near
 * mu), is GW_ERR_NOCONV; a non-finite electron count is GW_ERR_NONFINITE.
 * With a window set by gw_set_mu_window the result is instead *mu_inout
 * itself if its count is within the window of n_target, else the midpoint of
 * the two roots of N_e(mu) = n_target -/+ window (each found the same way).
 * Synchronises.                                                             */
gw_status gw_find_mu(gw_ctx* ctx, const gw_z* H0, const gw_z* S, const gw_z* Sig_inf,
                     const gw_z* Sig_iw, double n_target, double tol, double* mu_inout,
                     gw_z* G_iw, gw_z* G_tau, double* n_out);

/* Electron-count window of the mu search (Sec. IV.A adjusts mu until the
 * count is within a threshold, 1e-9 there).  ne_tol > 0: gw_find_mu keeps
 * the mu it is given when |N_e(mu) - n_target| <= ne_tol there, and
 * otherwise returns the midpoint of the interval of mu where that holds
 * (ne_tol clamped to half the distance of n_target from 0 and from ns*nao);
 * for a metal that interval is narrow and its midpoint is the root, for a
 * gapped system it lies mid-gap.  ne_tol = 0 (the default): the root.
 * Why: in a gapped system at low temperature the count is flat across the
 * gap up to the representation error of the sparse grids, so the root lies
 * where a Fermi tail cancels that error, near a band edge, and moves far
 * with small changes of Sigma; and every mu in the gap gives nearly a
 * solution (G(tau) moves with mu roughly as exp(dmu tau)), a direction in
 * which a self-consistency iteration hardly contracts unless mu is held.
 * A negative or non-finite ne_tol is GW_ERR_ARG.                            */
gw_status gw_set_mu_window(gw_ctx* ctx, double ne_tol);

/* Finite-size corrections of Eqs. K_corr and GW_head_corr (Sec. III.D),
 * added in place:
 *   Sig_inf^k           += -chi S^k gamma^k S^k
 *   Sig_tau^k(tau_i)    += -chi head[i] S^k G^k(tau_i) S^k
 * chi is the supercell Madelung constant and head[i] (host, ntau doubles) is
 * eps^{-1}_{00}(-tau_i) - 1, the head of the inverse dielectric function at
 * q = 0 minus one; both are inputs (the paper fits eps from q-points near
 * Gamma of a real crystal).  S, gamma, Sig_inf are [k][i][j]; G_tau, Sig_tau
 * [tau][k][i][j].  gamma with Sig_inf and G_tau with head and Sig_tau may
 * each be NULL to skip that term.  Needs nao <= 64; either precision.       */
gw_status gw_finite_size(gw_ctx* ctx, const gw_z* S, double chi, const gw_z* gamma, gw_z* Sig_inf,
                         const gw_z* G_tau, const double* head, gw_z* Sig_tau);

/* One whole Sigma[G] + Pi evaluation (Sec. III, Algorithm 1): gamma and
 * Sigma_inf = J + K (as gw_hf), then for every q P0^q(tau) (Eq.
 * tilde_P0_tau; Hermitian mode as set by gw_set_hermitian), P0^q(i Omega),
 * P~^q(i Omega) = (I - P0)^{-1} P0 (Eq. tilde_P_omega), P~^q(tau), and
 * Sig_tau = Sigma~(tau) (Eq. tilde_sigma2, overwritten).
 * Polarization storage, either all three or none:
 *   P_tau [Nk][ntau][naux][naux]: receives P~(tau) (P0(tau) on the way);
 *   P0_iw, Pt_iw [Nk][nw_b][naux][naux]: P0(i Omega) and P~(i Omega).
 *   These are what gw_sigma_jvp / gw_sigma_vjp take.  With all three NULL the
 *   evaluation runs q by q in per-q buffers of the workspace (GW_OP_SIGMA)
 *   and keeps nothing.  The screened-interaction solves of the stored form
 *   run in q-batches as large as the workspace holds.
 * gamma (may be NULL) receives gamma = -G(beta^-).  phi (host, may be NULL)
 * receives Phi~ (Eq. tilde_Phi_GW, as gw_screened_W_phi over all q) and makes
 * the call synchronise.  Errors as the calls it is made of.                 */
gw_status gw_sigma(gw_ctx* ctx, const void* V, const gw_z* G_tau, gw_z* gamma, gw_z* Sig_inf,
                   gw_z* Sig_tau, gw_z* P_tau, gw_z* P0_iw, gw_z* Pt_iw, double* phi);

/* Grand potential and energies of Sec. III.C (per unit cell, Ha), from the
 * self-energy (Sig_inf [k][i][j], Sig_iw [n][k][i][j] on the fermionic
 * sparse set; either may be NULL for zero) at chemical potential mu, with G
 * from the Dyson equation and Phi~ given (gw_screened_W_phi or gw_sigma):
 *   Omega = Phi_inf + Phi~ - Tr ln(-G^{-1}) - Tr{Sigma G}          (Eq. GP)
 *   Phi_inf = (1/2) Tr{Sigma_inf gamma}                             (Eq. Phi_GW)
 *   Tr ln(-G^{-1}) = (ns/Nk) sum_k [ (1/beta) sum_a ln(1 + e^{-beta xi_a})
 *                    + (1/beta) sum_n ln|det(I - G_ref Sigma~(i w_n))| ]
 *     with xi_a the eigenvalues of (H0 + Sig_inf - mu S, S) and G_ref the
 *     Green's function of the static part;
 *   Tr{Sigma G} = (ns/Nk) sum_k [ tr(Sig_inf gamma) + (1/beta) sum_n tr(Sig~ G) ];
 *   E_GM = Tr{H0 gamma} + (1/2) Tr{Sigma G} (Galitskii-Migdal).
 * Every equal-time trace takes G(0^-) = gamma = -G(beta^-).  The Matsubara
 * sums of the decaying terms are read off the sparse grid as the symmetric
 * average of the fitted tau function at 0+ and 0-: (1/beta) sum_n F(i w_n)
 * = -sum_n Re(r_n) Re F(i w_n), r = w TFp, so only ln|det| enters.  n_e is
 * the electron count of G.  Uses the GW_OP_THERMO workspace; copies H0,
 * S and Sig_inf to the host for the Nk small eigenvalue problems;
 * synchronises.  GW_ERR_SINGULAR for a zero pivot in either Dyson solve,
 * GW_ERR_ARG for an S that is not positive definite.                       */
typedef struct {
  double omega, phi_inf, phi_tilde, tr_ln, tr_sigma_g, e_one_body, e_gm, n_e;
} gw_thermo;
gw_status gw_thermodynamics(gw_ctx* ctx, const gw_z* H0, const gw_z* S, const gw_z* Sig_inf,
                            const gw_z* Sig_iw, double mu, double phi_tilde, gw_thermo* out);

/* Damped update and convergence measure of the scGW loop (Sec. IV.A):
 * Y <- (1 - alpha) Y + alpha X_new over n complex elements.  X_new may be
 * NULL, in which case Y <- (1 - alpha) Y, and alpha = 1 writes zeros without
 * reading Y.  maxdiff (host, may be NULL) receives max_i |X_new[i] - Y_old[i]|
 * (max |Y_old[i]| when X_new is NULL) and makes the call synchronise; if that
 * maximum is not finite (a NaN or Inf element, or Inf - Inf) the update is
 * still made, *maxdiff holds the non-finite value and the call returns
 * GW_ERR_NONFINITE, so that no convergence test passes on such a state.    */
gw_status gw_mix(gw_ctx* ctx, long long n, double alpha, const gw_z* X_new, gw_z* Y,
                 double* maxdiff);

/* ---- Derivatives of G -> (Sigma_inf, Sigma~) ----
 * All run in every precision.  The JVP calls (gw_polarization2,
 * gw_screened_W_lin, gw_transform_adjoint, gw_dyson_jvp, with gw_hf and
 * gw_self_energy, which are linear in G and in P~) follow the forward
 * precision; in the complex64 modes the VJP calls that read V
 * (gw_self_energy_vjp, gw_polarization_vjp; V is gw_c there) run their
 * products as complex fp32 MFMA GEMMs with complex64 intermediates and fp64
 * sums of 512-term chunks, and gw_hf_vjp reads the complex64 V in fp64
 * arithmetic; the cotangents and results are complex128.
 * The map is holomorphic in G, so a vector-Jacobian product (VJP) applies the
 * conjugate-transposed Jacobian to the cotangent; for a real loss L of the
 * outputs this is the gradient dL/dRe + i dL/dIm (torch autograd convention).
 * The forward quantities Pt (P~) are those of the same G.                   */

/* Two-slot polarization: Eq. tilde_P0_tau with G_a in the tau slot
 * (G^{k+q}(tau_i)) and G_b in the mirrored slot (G^k(tau_{ntau-1-i})).  The
 * derivative of P0 along dG is P0[dG, G] + P0[G, dG].  accumulate = 1 adds to
 * P0_tau instead of overwriting it.                                         */
gw_status gw_polarization2(gw_ctx* ctx, const void* V, const gw_z* G_a, const gw_z* G_b, int q0,
                           int nq, int accumulate, gw_z* P0_tau);

/* Derivative of Eq. tilde_P_omega: since (I - P0)^{-1} = I + P~,
 * d P~ = (I + P~) dP0 (I + P~).  adjoint = 0: Y = (I + Pt) X (I + Pt) (JVP);
 * adjoint = 1: Y = (I + Pt)^H X (I + Pt)^H (VJP).  Arrays [q][m][Q][Q'] for
 * nq * nw_b matrices; Y may not alias Pt or X.  Uses the GW_OP_SCREENED_W
 * workspace.                                                                */
gw_status gw_screened_W_lin(gw_ctx* ctx, const gw_z* Pt_iw, const gw_z* X_iw, int nq, int adjoint,
                            gw_z* Y_iw);

/* Adjoints of the transforms.  inverse = 0: X_tau[b][i][r] = sum_n
 * conj(T[n][i]) X_iw[b][n][r] (VJP of gw_tau_to_iw); inverse = 1:
 * X_iw[b][n][r] = sum_i conj(Tp[i][n]) X_tau[b][i][r] (VJP of gw_iw_to_tau).
 * Xin / Xout are laid out as the cotangents of the output / input.          */
gw_status gw_transform_adjoint(gw_ctx* ctx, int stat, int inverse, const gw_z* Xin,
                               long long batch, long long R, gw_z* Xout);

/* VJP of Eq. tilde_sigma2 for q = q0 .. q0+nq-1 with cotangent Sig_bar
 * [tau][k][i][j]: G_bar += the G part (accumulated), Pt_bar[q-q0][tau]
 * receives the P~ part (overwritten).                                        */
gw_status gw_self_energy_vjp(gw_ctx* ctx, const void* V, const gw_z* G_tau, const gw_z* Pt_tau,
                             const gw_z* Sig_bar, int q0, int nq, gw_z* G_bar, gw_z* Pt_bar);

/* VJP of Eq. tilde_P0_tau (both G slots) with cotangent P0_bar[q-q0][tau]:
 * G_bar += (accumulated).                                                    */
gw_status gw_polarization_vjp(gw_ctx* ctx, const void* V, const gw_z* G_tau, const gw_z* P0_bar,
                              int q0, int nq, gw_z* G_bar);

/* VJP of G -> gamma = -G(beta^-) -> Sigma_inf = J + K (Eqs. HF_J, HF_K) with
 * cotangent Sinf_bar [k][i][j]: G_bar += (accumulated).  The JVP is gw_hf
 * itself, which is linear in G.                                             */
gw_status gw_hf_vjp(gw_ctx* ctx, const void* V, const gw_z* Sinf_bar, gw_z* G_bar);

/* JVP of the Dyson step with the electron count held fixed (Eq. Dyson,
 * Sec. IV.A): for G(i w) at the current mu and a change of the self-energy
 * (dSinf [k][i][j] and dSig_iw [n][k][i][j], either may be NULL),
 *   dG = G (dSinf + dSig(i w_n) - dmu S) G,
 * where dmu makes the change of N_e = -(ns/Nk) sum Re(r_n tr[G S]) vanish
 * (r = w Tp, the beta^- row of the fermionic fit); fixed_mu = 1 uses
 * dmu = 0.  *dmu (host, may be NULL) receives it.  Synchronises.  Uses the
 * GW_OP_DYSON_JVP workspace.                                                */
gw_status gw_dyson_jvp(gw_ctx* ctx, const gw_z* S, const gw_z* G_iw, const gw_z* dSinf,
                       const gw_z* dSig_iw, int fixed_mu, gw_z* dG_iw, double* dmu);

/* Whole-chain derivatives of G -> (Sigma_inf[G], Sigma~[G]), the composition
 * of the calls above (derivative of the chain of Eqs. HF_J, HF_K,
 * tilde_P0_tau, P0t_to_P0w, tilde_P_omega, Piw_to_Pt, tilde_sigma2):
 *   JVP  dSig_inf = HF[gamma(dG)],  dP0 = P0[dG, G] + P0[G, dG],
 *        dP~(i Omega) = (I + P~) dP0(i Omega) (I + P~),
 *        dSig_tau = Sigma~[dP~, G] + Sigma~[P~, dG];
 *   VJP  G_bar = the conjugate-transposed steps applied to (Sinf_bar,
 *        Stau_bar) in reverse order (torch's convention for complex inputs).
 * Pt_tau [Nk][ntau][naux][naux] and Pt_iw [Nk][nw_b][naux][naux] are P~ of G
 * for all q as gw_sigma leaves them; with both NULL, P~^q is rebuilt q by q
 * inside the call from G (one polarization, transform and solve per q, with
 * the Hermitian mode of gw_set_hermitian), so nothing of size Nk naux^2 is
 * held.  The JVP uses GW_HERM_TWO_SLOT when set (dG Hermitian like G).
 * Outputs are overwritten: dSig_inf [k][i][j], dSig_tau and G_bar
 * [tau][k][i][j].  Workspace GW_OP_SIGMA.  Both run in every precision
 * (V complex128 or, in the complex64 modes, gw_c).                         */
gw_status gw_sigma_jvp(gw_ctx* ctx, const void* V, const gw_z* G_tau, const gw_z* Pt_tau,
                       const gw_z* Pt_iw, const gw_z* dG_tau, gw_z* dSig_inf, gw_z* dSig_tau);
gw_status gw_sigma_vjp(gw_ctx* ctx, const void* V, const gw_z* G_tau, const gw_z* Pt_tau,
                       const gw_z* Pt_iw, const gw_z* Sinf_bar, const gw_z* Stau_bar, gw_z* G_bar);

/* Vector operations of the Newton-Krylov solver: Y = a X + b Y for complex
 * a, b over n elements (X may be NULL; b = 0 does not read Y), and
 * out[0] + i out[1] = sum_i conj(X_i) Y_i (fixed reduction order; out is a
 * host array; synchronises).                                                */
gw_status gw_axpby(gw_ctx* ctx, long long n, double a_re, double a_im, const gw_z* X, double b_re,
                   double b_im, gw_z* Y);
gw_status gw_dot(gw_ctx* ctx, long long n, const gw_z* X, const gw_z* Y, double* out);

/* X[b] <- (X[b] + X[b]^H) / 2 for the nmat row-major n x n matrices of X
 * (1 <= n <= 8192, nmat <= 65535 per call): the projection onto Hermitian
 * matrices.  The self-energy of a Hermitian H0, S is Hermitian at every k
 * and tau, and the chemical-potential constraint makes G(Sigma) only real-
 * differentiable, so the Newton-Krylov iterates are kept on that subspace. */
gw_status gw_hermitize(gw_ctx* ctx, gw_z* X, int n, long long nmat);

/* Measurement.  While enabled, every launch of a kernel class is bracketed
 * by HIP events recorded on the context's stream; gw_profile_read
 * (synchronises) returns the launch count, the summed event time in ms and
 * the flops those launches execute on the matrix cores: 8 real flops per
 * complex multiply-add, 6 where a contraction uses the three-product
 * (Gauss) form (by default the self-energy contraction P~ V in fp64 and in
 * GW_PREC_FP32);
 * (32/3) n^3 per screened-interaction solve.  Enabling clears the counters. */
enum { GW_KCLASS_OTHER = 0, GW_KCLASS_POL_CONTRACT = 1, GW_KCLASS_POL_PRODUCER = 2,
       GW_KCLASS_SE_CONTRACT = 3, GW_KCLASS_SE_PRODUCER = 4, GW_KCLASS_SE_FINAL = 5,
       GW_KCLASS_TRANSFORM = 6, GW_KCLASS_HF = 7, GW_KCLASS_WDYSON = 8, GW_KCLASS_DYSON = 9 };
gw_status gw_profile_enable(gw_ctx* ctx, int on);
gw_status gw_profile_read(gw_ctx* ctx, int kclass, long long* launches, double* ms, double* flops);

/* Block until every call enqueued on the context's stream has finished. */
gw_status gw_synchronize(gw_ctx* ctx);

const char* gw_status_string(gw_status s);
const char* gw_last_error(const gw_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GW_H */
