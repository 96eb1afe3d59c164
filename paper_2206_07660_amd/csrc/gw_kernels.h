// Kernel descriptors shared by the HIP kernels and the host API (internal).
#pragma once
#include <hip/hip_runtime.h>

// Unsigned division by an invariant divisor d >= 1 as a multiply-high, an
// add and two shifts (Granlund and Montgomery, PLDI 1994, Fig. 4.1):
// l = ceil(log2 d), mul = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0); then n / d = (t + ((n - t) >> s1)) >> s2 with
// t = mulhi(n, mul), exact for every 32-bit n.
struct Udiv {
  unsigned d, mul, s1, s2;
};

static inline Udiv udiv_make(unsigned d) {
  unsigned l = 0;
  while (l < 32 && (1ull << l) < d) ++l;
  const unsigned long long mul = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return Udiv{d, (unsigned)mul, l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}

__host__ __device__ __forceinline__ unsigned udiv(unsigned n, const Udiv& u) {
#if defined(__HIP_DEVICE_COMPILE__)
  const unsigned t = __umulhi(n, u.mul);
#else
  const unsigned t = (unsigned)(((unsigned long long)n * u.mul) >> 32);
#endif
  return (t + ((n - t) >> u.s1)) >> u.s2;
}

// Index map i -> (i / (din*dmid)) * sout + ((i / din) % dmid) * smid + (i % din) * sin.
// An affine map has din = 0x7fffffff, dmid = 1 (aff() below).  qin and qmid
// divide by din and dmid.
struct Map3 {
  long long sout, smid, sin;
  unsigned din, dmid;
  Udiv qin, qmid;
};

static inline Map3 three(unsigned din, long long sin, unsigned dmid, long long smid, long long sout) {
  return Map3{sout, smid, sin, din, dmid, udiv_make(din), udiv_make(dmid)};
}
static inline Map3 aff(long long s) { return three(0x7fffffffu, s, 1u, 0, 0); }
static inline Map3 two(unsigned din, long long sin, long long sout) {
  return three(din, sin, 1u, 0, sout);
}

// C[b](m, n) = alpha * sum_k op(A)[b](m, k) * op(B)[b](k, n) + beta * C[b](m, n)
// with A[b](m, k) = A[ba(b) + tab[b % tmod] * tsA + am(m) + ak(k)] (conjugated if conjA),
// and likewise for B and C.  Offsets count complex elements of the operand's type.
// Kernel classes (profiling roles); values match GW_KCLASS_* of gw.h.
enum { KC_OTHER = 0, KC_POL_CONTRACT = 1, KC_POL_PRODUCER = 2, KC_SE_CONTRACT = 3,
       KC_SE_PRODUCER = 4, KC_SE_FINAL = 5, KC_TRANSFORM = 6, KC_HF = 7, KC_WDYSON = 8,
       KC_DYSON = 9, KC_COUNT = 10 };

struct GemmDesc {
  const void* A;   // element type by ta: 0 complex128 (double2), 1 complex64 (float2)
  const void* B;   // tb
  void* C;         // tc
  int M, N, K, batch;
  Map3 am, ak, bk, bn, cm, cn;
  Map3 ba, bb, bc;
  const int* tab;
  int tmod;
  long long tsA, tsB, tsC;
  int conjA, conjB;
  double alpha_r, alpha_i, beta_r, beta_i;
  int beta_zero;
  int tag;   // KC_*
  int cfg;   // tile configuration of the large contractions
  int ta, tb, tc;   // storage types of A, B, C (0 complex128, 1 complex64)
  int f32;          // 1: fp32 MFMA with fp64 promotion every kchunk K-elements
  int kchunk;
  int batch_fastest;  // workgroup order: 0 tile-fastest, 1 batch-fastest,
                      // 2 batch-fastest over groups of `group` tiles
  int group;
  int tri;            // 1: M == N and only the output tiles on or above the
                      // diagonal are computed (Hermitian products)
  // filled by the launcher: dividers of the workgroup-id decomposition
  Udiv q_tiles_m, q_tiles, q_batch, q_tmod;
};

static inline GemmDesc gemm_desc() {
  GemmDesc d{};
  d.ba = d.bb = d.bc = aff(0);
  d.am = d.ak = d.bk = d.bn = d.cm = d.cn = aff(0);
  d.tmod = 1;
  d.alpha_r = 1.0;
  d.beta_zero = 1;
  d.batch = 1;
  return d;
}

// Split-bf16 complex GEMM (bsgemm_k, bf16x3 or bf16x6 with operands split in LDS):
// C[b](m, n) = alpha * sum_k A[b](m, k) B[b](n, k) + beta * C[b](m, n) with
// A(m, k) = A[ba(b) + am(m) + k aks] and B(n, k) = B[bb(b) + bn(n) + k bks].
// Offsets count complex elements of the operand's storage type.
struct SplitDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K, batch;
  int ta, tb, tc;     // storage types: 0 complex128, 1 complex64
  Map3 am, bn, cm, cn;
  long long aks, bks;
  Map3 ba, bb, bc;
  double alpha_r;
  double beta_r;
  int beta_zero;
  int tri;            // as GemmDesc::tri
  int batch_fastest;  // as GemmDesc::batch_fastest
  int group;          // as GemmDesc::group
  int kchunk;         // fp32 accumulation length before the fp64 sum (multiple of 32)
  int tag;            // KC_POL_CONTRACT or KC_SE_CONTRACT
  int cfg;            // tile configuration (see bsgemm_launch)
  int nsplit;         // bf16 levels per real operand: 2 (bf16x3) or 3 (bf16x6)
  Udiv q_tiles_m, q_tiles, q_batch;
};

static inline SplitDesc split_desc() {
  SplitDesc d{};
  d.am = d.bn = d.cm = d.cn = aff(0);
  d.ba = d.bb = d.bc = aff(0);
  d.alpha_r = 1.0;
  d.beta_zero = 1;
  d.batch = 1;
  d.kchunk = 512;
  d.cfg = -1;
  d.nsplit = 2;
  return d;
}

struct DysonArgs {
  const double2* H0;
  const double2* S;
  const double2* Sinf;   // may be null
  const double2* Siw;    // may be null
  const double* wF;
  const double2* rrow;   // electron-count row r = w Tp (nw)
  double mu;
  int nk, nao;
  double2* G;            // may be null
  double* part;          // may be null
  int* flag;
  double* logdet;        // may be null: logdet[n*nk+k] = ln|det M| of the Dyson matrix
};

hipError_t zgemm_launch(const GemmDesc& d, hipStream_t st);
// true when zgemm_launch runs d on the three-product (Gauss) form: 6 real
// MFMA flops per complex multiply-add instead of 8
bool zgemm_three_product(const GemmDesc& d);
hipError_t bsgemm_launch(const SplitDesc& d, hipStream_t st);
hipError_t dyson_launch(const DysonArgs& a, int nw, hipStream_t st);
hipError_t sum_launch(const double* x, long long n, double scale, double* out, hipStream_t st);
hipError_t trace_launch(const double2* g, const double2* S, int n, int nk, double* part,
                        hipStream_t st);
hipError_t mix_launch(long long n, double alpha, const double2* X, double2* Y, double* part,
                      int nblk, hipStream_t st);
hipError_t zero_flag_launch(int* p, hipStream_t st);
hipError_t to_c64_launch(const double2* x, float2* y, long long n, hipStream_t st);
hipError_t axpby_launch(long long n, double ar, double ai, const double2* X, double br, double bi,
                        double2* Y, hipStream_t st);
hipError_t dot_launch(long long n, const double2* X, const double2* Y, double* part, int nblk,
                      double* out, hipStream_t st);
// part[n*nk+k] = Re(r_n tr[P[n][k] S[k]]) (S per k: s_per_w = 0) or with S[n][k] (s_per_w = 1).
hipError_t wtrace_launch(const double2* P, const double2* S, const double2* r, int nao, int nk, int nw,
                         double* part, hipStream_t st, int s_per_w = 0);
// P[b] for b < nmat (n x n, row-major): entries below the diagonal become the
// conjugates of their mirror images above it.
hipError_t herm_fill_launch(double2* P, int n, long long nmat, hipStream_t st);
// P[b] <- (P[b] + P[b]^H) / 2 for b < nmat (n x n, row-major).
hipError_t herm_avg_launch(double2* P, int n, long long nmat, hipStream_t st);
// Eq. tilde_Phi_GW: for each of nmat matrices m of an LU-factorised I - P0
// (packed in LU, U on and above the diagonal) writes
// part[m] = wts[m % nw] (sum_i ln|U_ii| + Re tr P0_m), then out[0] = sum_m part[m]
// in a fixed order.
hipError_t phi_terms_launch(const double2* LU, const double2* P0, int n, long long nmat,
                            const double* wts, int nw, double* part, double* out, hipStream_t st);
// Finite-size corrections: Out[b] += alpha S[b % nk] X[b] S[b % nk] for
// b < nmat (nk S matrices, nmat X and Out matrices, all n x n, n <= 64).
hipError_t sxs_add_launch(const double2* S, const double2* X, double2* Out, int n, int nk,
                          long long nmat, double alpha, hipStream_t st);
hipError_t wlu_launch(int which, const double2* P0, double2* A, double2* B, int n, int j0, int nb,
                      long long nmat, int* flag, hipStream_t st);
