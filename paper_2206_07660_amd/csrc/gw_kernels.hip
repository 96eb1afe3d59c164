// Device kernels of the density-fitted GW hot path for CDNA4 (gfx950).
//
//  * zgemm_k     batched complex fp64 GEMM on v_mfma_f64_16x16x4_f64 with
//                per-operand index maps, used for every contraction of the
//                polarization and self-energy chains, the tau <-> i omega
//                transforms and the Hartree-Fock terms.
//                fp32 MFMA variant for the mixed-precision path.
//  * wlu_*_k     panel and triangular kernels of the blocked LU of I - P0
//                (Eq. tilde_P_omega); its trailing updates are zgemm_k calls.
//  * dyson_k     G = [(i w + mu) S - H0 - Sigma]^{-1} by Gauss-Jordan (Eq. Dyson),
//                with the electron-count partials of gamma = -G(beta^-).
//  * herm_fill_k, herm_avg_k   Hermitian fill / Hermitian part of matrices.
//  * small reductions and vector kernels (sums, traces, mixing, axpby, dot).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "gw_kernels.h"

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ long long map3(const Map3& m, unsigned i) {
  const unsigned r = udiv(i, m.qin);
  const unsigned a = i - r * m.din;
  const unsigned c = udiv(r, m.qmid);
  const unsigned b = r - c * m.dmid;
  return (long long)c * m.sout + (long long)b * m.smid + (long long)a * m.sin;
}

// Running offset of a mapped index that advances by a fixed step.
struct Ctr {
  long long off;
  unsigned a, b;
};

__device__ __forceinline__ Ctr ctr_init(const Map3& m, unsigned i) {
  Ctr c;
  const unsigned r = udiv(i, m.qin);
  c.a = i - r * m.din;
  const unsigned o = udiv(r, m.qmid);
  c.b = r - o * m.dmid;
  c.off = (long long)o * m.sout + (long long)c.b * m.smid + (long long)c.a * m.sin;
  return c;
}

__device__ __forceinline__ void ctr_step(const Map3& m, Ctr& c, unsigned st) {
  c.a += st;
  c.off += (long long)st * m.sin;
  while (c.a >= m.din) {
    c.a -= m.din;
    c.off -= (long long)m.din * m.sin;
    c.off += m.smid;
    if (++c.b >= m.dmid) {
      c.b = 0;
      c.off -= (long long)m.dmid * m.smid;
      c.off += m.sout;
    }
  }
}

// Same as ctr_step for st <= din and st <= din * dmid (at most one carry per
// digit), written with selects so that the K loop has no divergent branches.
__device__ __forceinline__ void ctr_step1(const Map3& m, Ctr& c, unsigned st) {
  c.a += st;
  c.off += (long long)st * m.sin;
  const bool w1 = c.a >= m.din;
  c.a = w1 ? c.a - m.din : c.a;
  c.off += w1 ? (m.smid - (long long)m.din * m.sin) : 0;
  c.b += w1 ? 1u : 0u;
  const bool w2 = c.b >= m.dmid;
  c.b = w2 ? 0u : c.b;
  c.off += w2 ? (m.sout - (long long)m.dmid * m.smid) : 0;
}

__device__ __forceinline__ long long batch_off(const Map3& m, const int* tab, const Udiv& tmod, long long ts,
                                               unsigned b) {
  long long o = map3(m, b);
  if (ts != 0) o += (long long)tab[b - udiv(b, tmod) * tmod.d] * ts;
  return o;
}

// Output tile (tm, tn) and batch entry bt of this workgroup.  XCD-aware
// order: the dispatcher deals workgroup ids round-robin over the 8 XCDs, so
// id w runs on XCD w % 8.  Each XCD gets a contiguous range of logical ids,
// so that the tiles of one batch entry (which share operand rows and
// columns) meet in the same L2.  With d.tri only the tiles on or above the
// diagonal are enumerated, row by row.  With d.batch_fastest = 1 the batch
// shares an operand (e.g. one V slab for every tau): consecutive ids walk the
// batch and keep that operand's tile in L2; = 2 does the same for groups of
// d.group tiles.
struct TilePos {
  int tm, tn;
  unsigned bt;
};

template <class D>
__device__ __forceinline__ TilePos tile_pos(const D& d, int TM, int TN) {
  const int tiles_m = (d.M + TM - 1) / TM;
  const unsigned tiles = d.tri ? (unsigned)tiles_m * (unsigned)(tiles_m + 1) / 2u
                               : (unsigned)tiles_m * (unsigned)((d.N + TN - 1) / TN);
  const unsigned total = gridDim.x;
  const unsigned w = blockIdx.x;
  const unsigned xcd = w % 8u, slot = w / 8u, per = total / 8u, rem = total % 8u;
  const unsigned logical = xcd < rem ? xcd * (per + 1u) + slot : rem * (per + 1u) + (xcd - rem) * per + slot;
  const unsigned nbatch = (unsigned)d.batch;
  unsigned tile, bt;
  if (d.batch_fastest == 2) {
    // groups of d.group consecutive tiles (the last one may be shorter): a
    // group walks the batch, each batch entry its tiles, so the operand the
    // batch shares stays in L2 for the group while each entry's own operand
    // is fetched once per group
    const unsigned G = (unsigned)d.group, span = G * nbatch, full = tiles / G;
    const unsigned g = logical / span;
    const unsigned gl = g < full ? G : tiles - full * G;
    const unsigned rem = logical - g * span;
    bt = rem / gl;
    tile = g * G + (rem - bt * gl);
  } else {
    const unsigned lq = udiv(logical, d.batch_fastest ? d.q_batch : d.q_tiles);
    const unsigned lr = logical - lq * (d.batch_fastest ? nbatch : tiles);
    tile = d.batch_fastest ? lq : lr;
    bt = d.batch_fastest ? lr : lq;
  }
  TilePos p;
  if (d.tri) {
    unsigned t = tile, r = 0, len = (unsigned)tiles_m;
    while (t >= len) {
      t -= len;
      ++r;
      --len;
    }
    p.tm = (int)r;
    p.tn = (int)(r + t);
  } else {
    const unsigned tn_ = udiv(tile, d.q_tiles_m);
    p.tm = (int)(tile - tn_ * (unsigned)tiles_m);
    p.tn = (int)tn_;
  }
  p.bt = bt;
  return p;
}

// ---------------------------------------------------------------------------
// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b], complex.
// Waves: WM x WN tile the output, WK split the K loop (reduced through LDS).
// Each wave owns BM x BN blocks of 16 x 16 complex outputs.  The fragments of
// A and B are loaded straight from global memory (one complex per lane per
// block per K-step of 4) into a two-stage register ping-pong.
// TA, TB, TC are the storage types (double2 = complex128, float2 = complex64).
// F32 = false: v_mfma_f64_16x16x4_f64, fp64 accumulation.
// F32 = true:  v_mfma_f32_16x16x4_f32 on operands rounded to fp32, fp32
//              accumulation inside chunks of d.kchunk K-elements, each chunk
//              added into fp64 accumulators.
// TAG only separates the roles of the kernel in profiles (KC_*).

__device__ __forceinline__ double2 to_d2(double2 v) { return v; }
__device__ __forceinline__ double2 to_d2(float2 v) { return double2{(double)v.x, (double)v.y}; }
__device__ __forceinline__ float2 to_f2(double2 v) { return float2{(float)v.x, (float)v.y}; }
__device__ __forceinline__ float2 to_f2(float2 v) { return v; }
template <class T> __device__ __forceinline__ T from_d2(double2 v);
template <> __device__ __forceinline__ double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ __forceinline__ float2 from_d2<float2>(double2 v) {
  return float2{(float)v.x, (float)v.y};
}

// bf16 pairs (round to nearest even) for the split-bf16 contractions:
// element 0 in the low half, as in memory.
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
  const bf2v v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ float bf16_low(unsigned p) { return __builtin_bit_cast(float, p << 16); }
__device__ __forceinline__ float bf16_high(unsigned p) { return __builtin_bit_cast(float, p & 0xffff0000u); }

template <bool F32> struct Mfma;
template <> struct Mfma<false> {
  typedef double S;
  typedef double2 S2;
  typedef d4 Acc;
  static __device__ __forceinline__ Acc run(S a, S b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // c - a b: the f64 MFMA reads its last control field as negate flags
  static __device__ __forceinline__ Acc run_neg(S a, S b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 1);
  }
  template <class T> static __device__ __forceinline__ S2 cvt(T v) { return to_d2(v); }
  // output row of accumulator element r held by lane group g = lane / 16
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <> struct Mfma<true> {
  typedef float S;
  typedef float2 S2;
  typedef f4 Acc;
  static __device__ __forceinline__ Acc run(S a, S b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ Acc run_neg(S a, S b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(-a, b, c, 0, 0, 0);
  }
  template <class T> static __device__ __forceinline__ S2 cvt(T v) { return to_f2(v); }
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

// Raw buffer loads (gfx9 descriptor format).  A lane whose byte offset is not
// below the record count reads zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, 0x7fffffff, 0x00020000);
}
// (The loaded vector is reinterpreted as a whole: element-wise access of the
// builtins' vector results is not reliable with this compiler.)
struct Dd { double x, y; };
struct Ff { float x, y; };
template <class T> __device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so);
template <> __device__ __forceinline__ double2 buf_load<double2>(__amdgpu_buffer_rsrc_t r, unsigned vo,
                                                                 unsigned so) {
  const Dd v = __builtin_bit_cast(Dd, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0));
  double2 x;
  x.x = v.x;
  x.y = v.y;
  return x;
}
template <> __device__ __forceinline__ float2 buf_load<float2>(__amdgpu_buffer_rsrc_t r, unsigned vo,
                                                               unsigned so) {
  const Ff v = __builtin_bit_cast(Ff, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0));
  float2 x;
  x.x = v.x;
  x.y = v.y;
  return x;
}
// x or -x by a uniform sign mask (0 or the sign bit of the high word)
__device__ __forceinline__ double flip(double x, unsigned m) {
  return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, x) ^ ((unsigned long long)m << 32));
}
__device__ __forceinline__ float flip(float x, unsigned m) {
  return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, x) ^ m);
}

// KM: K-loop form.  0 general index maps (any number of carries per step);
// 1 at most one carry per digit and step; 2 "uniform" (see launch_cfg): the
// K offset is a wave-uniform scalar and each lane keeps a constant offset.
// G3 (uniform-K loop): the complex product on three real MFMAs (Gauss):
// P1 = sum ar br, P2 = sum ai bi, P3 = sum (ar + ai)(br + bi), then
// re = P1 - P2 and im = P3 - P1 - P2 (with F32 at every fp64 promotion).  A
// quarter fewer MFMAs for a third accumulator set; the rounding error stays
// a few ulps of sum |a| |b|.
template <int WM, int WN, int WK, int BM, int BN, int TAG, int KM, class TA, class TB, class TC,
          bool F32, bool G3 = false>
__global__ void __launch_bounds__(64 * WM * WN * WK) zgemm_k(GemmDesc d) {
  constexpr bool M3 = G3 && KM == 2;
  typedef Mfma<F32> MM;
  typedef typename MM::S S;
  typedef typename MM::S2 S2;
  typedef typename MM::Acc Acc;
  constexpr int TM = WM * BM * 16, TN = WN * BN * 16;
  const int lane = threadIdx.x & 63;
  // the wave index is uniform within a wave; saying so keeps the K loop scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wn = (wave / WM) % WN, wk = wave / (WM * WN);
  const TilePos tp = tile_pos(d, TM, TN);
  const int tm = tp.tm, tn = tp.tn;
  const unsigned bt = tp.bt;

  const TA* A = (const TA*)d.A + batch_off(d.ba, d.tab, d.q_tmod, d.tsA, bt);
  const TB* B = (const TB*)d.B + batch_off(d.bb, d.tab, d.q_tmod, d.tsB, bt);
  TC* C = (TC*)d.C + batch_off(d.bc, d.tab, d.q_tmod, d.tsC, bt);

  const int m0 = tm * TM + wm * BM * 16;
  const int n0 = tn * TN + wn * BN * 16;
  const int r16 = lane & 15;
  const int kl = lane >> 4;

  long long aoff[BM], boff[BN];
  bool av[BM], bv[BN];
#pragma unroll
  for (int i = 0; i < BM; ++i) {
    const int m = m0 + i * 16 + r16;
    av[i] = m < d.M;
    aoff[i] = av[i] ? map3(d.am, m) : 0;
  }
#pragma unroll
  for (int j = 0; j < BN; ++j) {
    const int n = n0 + j * 16 + r16;
    bv[j] = n < d.N;
    boff[j] = bv[j] ? map3(d.bn, n) : 0;
  }

  Acc accR[BM][BN], accI[BM][BN], accN[M3 ? BM : 1][M3 ? BN : 1];
  double sumR[F32 ? BM : 1][F32 ? BN : 1][4], sumI[F32 ? BM : 1][F32 ? BN : 1][4];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      accR[i][j] = Acc{0, 0, 0, 0};
      accI[i][j] = Acc{0, 0, 0, 0};
      if constexpr (M3) accN[i][j] = Acc{0, 0, 0, 0};
    }
  if constexpr (F32) {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) sumR[i][j][r] = sumI[i][j][r] = 0.0;
  }
  auto promote = [&]() {
    if constexpr (F32) {
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (M3) {
              const double p1 = accR[i][j][r], p2 = accN[i][j][r], p3 = accI[i][j][r];
              sumR[i][j][r] += p1 - p2;
              sumI[i][j][r] += p3 - p1 - p2;
            } else {
              sumR[i][j][r] += (double)accR[i][j][r];
              sumI[i][j][r] += (double)accI[i][j][r];
            }
          }
          accR[i][j] = Acc{0, 0, 0, 0};
          accI[i][j] = Acc{0, 0, 0, 0};
          if constexpr (M3) accN[i][j] = Acc{0, 0, 0, 0};
        }
    }
  };

  const unsigned K = (unsigned)d.K;
  const unsigned kstep = 4u * WK;
  const S sa = d.conjA ? S(-1) : S(1);
  const S sb = d.conjB ? S(-1) : S(1);
  const S2 zero2 = S2{0, 0};

  // Branch-free fragment loads: an out-of-range lane reads the operand's first
  // element (always valid) and keeps zero.
  auto load = [&](S2 (&a)[BM], S2 (&b)[BN], const Ctr& ca, const Ctr& cb, bool kv) {
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      const bool ok = av[i] && kv;
      const S2 v = MM::cvt(A[ok ? aoff[i] + ca.off : 0]);
      a[i] = ok ? v : zero2;
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const bool ok = bv[j] && kv;
      const S2 v = MM::cvt(B[ok ? boff[j] + cb.off : 0]);
      b[j] = ok ? v : zero2;
    }
  };
  // complex 4M update: re += ar br - ai bi, im += ar bi + ai br
  auto mma = [&](const S2 (&a)[BM], const S2 (&b)[BN]) {
    S ar[BM], ai[BM], nai[BM], br[BN], bi[BN];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      ar[i] = a[i].x;
      ai[i] = sa * a[i].y;
      nai[i] = -ai[i];
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      br[j] = b[j].x;
      bi[j] = sb * b[j].y;
    }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        accR[i][j] = MM::run(ar[i], br[j], accR[i][j]);
        accI[i][j] = MM::run(ar[i], bi[j], accI[i][j]);
      }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        accR[i][j] = MM::run(nai[i], bi[j], accR[i][j]);
        accI[i][j] = MM::run(ai[i], br[j], accI[i][j]);
      }
  };
  auto step = [&](Ctr& ca, Ctr& cb) {
    if constexpr (KM == 1) {
      ctr_step1(d.ak, ca, kstep);
      ctr_step1(d.bk, cb, kstep);
    } else {
      ctr_step(d.ak, ca, kstep);
      ctr_step(d.bk, cb, kstep);
    }
  };

  // Ping-pong register buffers: the loads of one K-step are in flight while
  // the MFMAs of the previous one run.  nsteps and the promotion period are
  // uniform across the wave.
  const unsigned kfirst = 4u * wk;
  const unsigned nsteps = kfirst < K ? (K - kfirst + kstep - 1) / kstep : 0u;
  const unsigned cper = F32 && d.kchunk > 0 ? (unsigned)d.kchunk / kstep : 0u;
  S2 a0[BM], b0[BN], a1[BM], b1[BN];
  if constexpr (KM == 2) {
    // Operand loads: buffer loads, except for the polarization contraction,
    // whose two streamed operands come back from HBM less often with global
    // loads (measured: 100 vs 139 GB fetched per launch, 25.5 vs 27.1 ms).
    constexpr bool LOADG = TAG == KC_POL_CONTRACT;
    // The fp32 polarization and self-energy contractions (split-K tiles) run
    // faster with a conditional prefetch that the scheduler interleaves with
    // the MFMAs (measured at si-4x4x4, ms per q: 18.8 vs 19.7 / 22.1 and 23.0
    // vs 25.1 / 25.3); every other kernel gains from the branch-free, pinned
    // one (fp64 polarization 23.8 -> 22.6, fp32 final contraction 6.6 -> 5.4)
    constexpr bool PIN = !(F32 && (TAG == KC_POL_CONTRACT || TAG == KC_SE_CONTRACT));
    // The four k of a step lie in one aligned group of every K map, so the
    // K offset is one scalar per operand (the buffer soffset) and a lane's
    // byte offset (voffset) is fixed for the whole loop.  Rows past M or N,
    // and k past K on the last step, get an offset past the record count and
    // read zeros.  The complex product needs no VALU: the -ai bi term uses
    // the MFMA's negate flag, conjugation is a sign-bit flip.
    constexpr unsigned kOut = 0x80000000u;
    const __amdgpu_buffer_rsrc_t ra = buf_rsrc(A), rb = buf_rsrc(B);
    unsigned voa[BM], vob[BN];
#pragma unroll
    for (int i = 0; i < BM; ++i) {
      const int m = m0 + i * 16 + r16;
      if constexpr (LOADG) {
        // global loads: rows past M read row M - 1 (their outputs are dropped)
        voa[i] = (unsigned)((map3(d.am, min(m, d.M - 1)) + (long long)kl * d.ak.sin) * (long long)sizeof(TA));
      } else {
        voa[i] = m < d.M ? (unsigned)((map3(d.am, m) + (long long)kl * d.ak.sin) * (long long)sizeof(TA)) : kOut;
      }
    }
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int n = n0 + j * 16 + r16;
      if constexpr (LOADG) {
        vob[j] = (unsigned)((map3(d.bn, min(n, d.N - 1)) + (long long)kl * d.bk.sin) * (long long)sizeof(TB));
      } else {
        vob[j] = n < d.N ? (unsigned)((map3(d.bn, n) + (long long)kl * d.bk.sin) * (long long)sizeof(TB)) : kOut;
      }
    }
    bool kvl = true;   // LOADG: this lane's k is below K (only false on the last step)
    Ctr ua = ctr_init(d.ak, kfirst), ub = ctr_init(d.bk, kfirst);
    const unsigned ma = d.conjA ? 0x80000000u : 0u, mb = d.conjB ? 0x80000000u : 0u;
    // adv = false: a prefetch past the last full step re-reads the step
    // loaded last (valid addresses) and leaves the counters where they are.
    // Selects, not a branch: a load under a branch makes the first use of
    // any fragment loaded before it wait for all outstanding loads.
    long long la = ua.off, lb = ub.off;   // K offsets of the step loaded last
    auto ldf = [&](S2 (&a)[BM], S2 (&b)[BN], bool adv) {
      const long long oa = adv ? ua.off : la, ob = adv ? ub.off : lb;
      la = oa;
      lb = ob;
      const unsigned soa = (unsigned)(oa * (long long)sizeof(TA));
      const unsigned sob = (unsigned)(ob * (long long)sizeof(TB));
      if constexpr (LOADG) {
        const char* pa = (const char*)A + soa;
        const char* pb = (const char*)B + sob;
#pragma unroll
        for (int i = 0; i < BM; ++i) {
          const S2 v = MM::cvt(*(const TA*)(pa + voa[i]));
          a[i] = kvl ? v : zero2;
        }
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          const S2 v = MM::cvt(*(const TB*)(pb + vob[j]));
          b[j] = kvl ? v : zero2;
        }
      } else {
#pragma unroll
        for (int i = 0; i < BM; ++i) a[i] = MM::cvt(buf_load<TA>(ra, voa[i], soa));
#pragma unroll
        for (int j = 0; j < BN; ++j) b[j] = MM::cvt(buf_load<TB>(rb, vob[j], sob));
      }
      Ctr na = ua, nb = ub;
      ctr_step1(d.ak, na, kstep);
      ctr_step1(d.bk, nb, kstep);
      ua.off = adv ? na.off : ua.off;
      ua.a = adv ? na.a : ua.a;
      ua.b = adv ? na.b : ua.b;
      ub.off = adv ? nb.off : ub.off;
      ub.a = adv ? nb.a : ub.a;
      ub.b = adv ? nb.b : ub.b;
    };
    auto mmf = [&](const S2 (&a)[BM], const S2 (&b)[BN]) {
      S ar[BM], ai[BM], br[BN], bi[BN];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        ar[i] = a[i].x;
        ai[i] = flip(a[i].y, ma);
      }
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        br[j] = b[j].x;
        bi[j] = flip(b[j].y, mb);
      }
      if constexpr (M3) {
        S as[BM], bs[BN];
#pragma unroll
        for (int i = 0; i < BM; ++i) as[i] = ar[i] + ai[i];
#pragma unroll
        for (int j = 0; j < BN; ++j) bs[j] = br[j] + bi[j];
#pragma unroll
        for (int i = 0; i < BM; ++i)
#pragma unroll
          for (int j = 0; j < BN; ++j) {
            accR[i][j] = MM::run(ar[i], br[j], accR[i][j]);
            accN[i][j] = MM::run(ai[i], bi[j], accN[i][j]);
            accI[i][j] = MM::run(as[i], bs[j], accI[i][j]);
          }
        return;
      }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          accR[i][j] = MM::run(ar[i], br[j], accR[i][j]);
          accI[i][j] = MM::run(ar[i], bi[j], accI[i][j]);
        }
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
          accR[i][j] = MM::run_neg(ai[i], bi[j], accR[i][j]);
          accI[i][j] = MM::run(ai[i], br[j], accI[i][j]);
        }
    };
    auto pc = [&](unsigned st) {
      if constexpr (F32) {
        if (cper && (st + 1) % cper == 0) promote();
      }
    };
    // steps whose four k are all below K
    const unsigned nfull = kfirst + 4u <= K ? (K - kfirst - 4u) / kstep + 1u : 0u;
    unsigned s = 0;
    if (nfull) ldf(a0, b0, true);
    for (; s + 2 <= nfull; s += 2) {
      ldf(a1, b1, true);
      // keep each prefetch ahead of the MFMAs it is meant to overlap
      if constexpr (PIN) __builtin_amdgcn_sched_barrier(0);
      mmf(a0, b0);
      pc(s);
      if constexpr (PIN) {
        ldf(a0, b0, s + 2 < nfull);
        __builtin_amdgcn_sched_barrier(0);
      } else if (s + 2 < nfull) {
        ldf(a0, b0, true);
      }
      mmf(a1, b1);
      pc(s + 1);
    }
    if (s < nfull) {
      mmf(a0, b0);
      pc(s);
      ++s;
    }
    if (s < nsteps) {
      // last, partial step: lanes with k >= K read zeros
      const unsigned k0 = kfirst + s * kstep;
      const bool kv = k0 + (unsigned)kl < K;
      if constexpr (LOADG) {
        // lanes past K read the step's first k (valid) and keep zeros
#pragma unroll
        for (int i = 0; i < BM; ++i) voa[i] -= kv ? 0u : (unsigned)(kl * d.ak.sin * (long long)sizeof(TA));
#pragma unroll
        for (int j = 0; j < BN; ++j) vob[j] -= kv ? 0u : (unsigned)(kl * d.bk.sin * (long long)sizeof(TB));
        kvl = kv;
      } else {
#pragma unroll
        for (int i = 0; i < BM; ++i) voa[i] = kv ? voa[i] : kOut;
#pragma unroll
        for (int j = 0; j < BN; ++j) vob[j] = kv ? vob[j] : kOut;
      }
      ldf(a0, b0, true);
      mmf(a0, b0);
      pc(s);
    }
  } else {
    unsigned k = kfirst + kl;                  // this lane's k for the step in buffer 0
    Ctr ca = ctr_init(d.ak, k), cb = ctr_init(d.bk, k);
    load(a0, b0, ca, cb, k < K);
    unsigned s = 0;
    for (; s + 1 < nsteps; s += 2) {
      step(ca, cb);
      load(a1, b1, ca, cb, k + kstep < K);
      mma(a0, b0);
      if (cper && (s + 1) % cper == 0) promote();
      step(ca, cb);
      load(a0, b0, ca, cb, k + 2u * kstep < K);
      mma(a1, b1);
      if (cper && (s + 2) % cper == 0) promote();
      k += 2u * kstep;
    }
    if (s < nsteps) mma(a0, b0);
  }
  promote();

  // lane-local result, fp64
  auto res = [&](int i, int j, int r, bool im) -> double {
    if constexpr (F32) return im ? sumI[i][j][r] : sumR[i][j][r];   // M3 combined in promote
    else if constexpr (M3)
      return im ? accI[i][j][r] - accR[i][j][r] - accN[i][j][r] : accR[i][j][r] - accN[i][j][r];
    else return im ? accI[i][j][r] : accR[i][j][r];
  };

  double outR[BM][BN][4], outI[BM][BN][4];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        outR[i][j][r] = res(i, j, r, false);
        outI[i][j][r] = res(i, j, r, true);
      }

  if constexpr (WK > 1) {
    // deterministic split-K reduction: waves wk > 0 park their sums in LDS,
    // wave wk = 0 adds them in wk order.
    __shared__ double red[(WK > 1 ? WK - 1 : 1) * WM * WN * BM * BN * 8 * 64];
    const int slot = (wm + WM * wn) * BM * BN * 8;
    if (wk > 0) {
      double* p = red + ((size_t)(wk - 1) * WM * WN * BM * BN * 8) * 64;
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            p[(slot + ((i * BN + j) * 8 + r)) * 64 + lane] = outR[i][j][r];
            p[(slot + ((i * BN + j) * 8 + 4 + r)) * 64 + lane] = outI[i][j][r];
          }
    }
    __syncthreads();
    if (wk > 0) return;
    for (int w2 = 1; w2 < WK; ++w2) {
      const double* p = red + ((size_t)(w2 - 1) * WM * WN * BM * BN * 8) * 64;
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            outR[i][j][r] += p[(slot + ((i * BN + j) * 8 + r)) * 64 + lane];
            outI[i][j][r] += p[(slot + ((i * BN + j) * 8 + 4 + r)) * 64 + lane];
          }
    }
  }

  // epilogue: lane holds column lane%16 of each 16 x 16 block and the rows
  // given by MM::row (f64 MFMA: lane/16 + 4r; f32 MFMA: 4 (lane/16) + r)
  long long roff[BM][4];
  bool rok[BM][4];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + i * 16 + MM::row(kl, r);
      rok[i][r] = m < d.M;
      roff[i][r] = rok[i][r] ? map3(d.cm, m) : 0;
    }
  // PLAIN: alpha = 1 and beta = 0, the common case, without the scaling
  auto store = [&](auto plain) {
#pragma unroll
    for (int j = 0; j < BN; ++j) {
      const int n = n0 + j * 16 + r16;
      if (n >= d.N) continue;
      const long long con = map3(d.cn, n);
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!rok[i][r]) continue;
          const long long o = roff[i][r] + con;
          const double xr = outR[i][j][r], xi = outI[i][j][r];
          double2 v;
          if constexpr (decltype(plain)::value) {
            v.x = xr;
            v.y = xi;
          } else {
            v.x = d.alpha_r * xr - d.alpha_i * xi;
            v.y = d.alpha_r * xi + d.alpha_i * xr;
            if (!d.beta_zero) {
              const double2 c = to_d2(C[o]);
              v.x += d.beta_r * c.x - d.beta_i * c.y;
              v.y += d.beta_r * c.y + d.beta_i * c.x;
            }
          }
          C[o] = from_d2<TC>(v);
        }
    }
  };
  if (d.beta_zero && d.alpha_r == 1.0 && d.alpha_i == 0.0)
    store(std::true_type{});
  else
    store(std::false_type{});
}

// ---------------------------------------------------------------------------
// Producers with short K (K <= 32, e.g. X = V G with K = nao): the GemmDesc
// product of zgemm_k (index maps, batch tables, conjugation, alpha, beta),
// organised for an output-bound product.  Each wave keeps the A fragments of
// its 32 rows for all K-steps in registers and walks a run of 16-column
// blocks: the B fragments of the next block load while the MFMAs of the
// current block run and its results are stored, so operand loads, MFMAs and
// stores of consecutive blocks overlap.  Used for the fp32-MFMA producers;
// with fp64 MFMA the tiled kernel stays ahead (see launch_typed).
// KS (the K-steps of 4) is a compile-time count, so that no load or MFMA
// sits under a branch: a branch there makes every use of a prefetched
// fragment wait for all outstanding memory operations, stores included.
// Rows past M and k past K contribute zeros; loads of clamped rows, columns
// and k stay inside the operands.
constexpr int kProdRows = 128;    // rows per workgroup: 4 waves x 32
constexpr int kProdBlocks = 16;   // 16-column blocks per workgroup

template <int TAG, int KS, class TA, class TB, class TC, bool F32>
__global__ void __launch_bounds__(256) prod_k(GemmDesc d) {
  typedef Mfma<F32> MM;
  typedef typename MM::S S;
  typedef typename MM::S2 S2;
  typedef typename MM::Acc Acc;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r16 = lane & 15, kl = lane >> 4;
  // XCD-contiguous logical id (as tile_pos), decomposed as (run fastest,
  // row tile, batch entry): consecutive workgroups share the A rows of a row
  // tile, and a batch entry's B stays in its XCD's L2
  const unsigned w = blockIdx.x, total = gridDim.x;
  const unsigned xcd = w % 8u, slot = w / 8u, per = total / 8u, rem = total % 8u;
  const unsigned logical = xcd < rem ? xcd * (per + 1u) + slot : rem * (per + 1u) + (xcd - rem) * per + slot;
  const unsigned bt = udiv(logical, d.q_tiles);
  const unsigned rest = logical - bt * d.q_tiles.d;
  const unsigned tm = udiv(rest, d.q_tiles_m);
  const unsigned run = rest - tm * d.q_tiles_m.d;

  const TA* A = (const TA*)d.A + batch_off(d.ba, d.tab, d.q_tmod, d.tsA, bt);
  const TB* B = (const TB*)d.B + batch_off(d.bb, d.tab, d.q_tmod, d.tsB, bt);
  TC* C = (TC*)d.C + batch_off(d.bc, d.tab, d.q_tmod, d.tsC, bt);
  const int K = d.K;
  const unsigned ma = d.conjA ? 0x80000000u : 0u, mb = d.conjB ? 0x80000000u : 0u;
  const int m0 = (int)tm * kProdRows + wave * 32;

  S ar[2][KS], ai[2][KS];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int m = m0 + i * 16 + r16;
    const bool mv = m < d.M;
    const long long ao = map3(d.am, (unsigned)(mv ? m : d.M - 1));
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + kl;
      const bool ok = mv && k < K;
      const S2 v = MM::cvt(A[ao + map3(d.ak, (unsigned)(k < K ? k : K - 1))]);
      ar[i][s] = ok ? v.x : S(0);
      ai[i][s] = ok ? flip(v.y, ma) : S(0);
    }
  }
  long long bko[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + kl;
    bko[s] = map3(d.bk, (unsigned)(k < K ? k : K - 1));
  }
  long long ro[2][4];
  bool rok[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + i * 16 + MM::row(kl, r);
      rok[i][r] = m < d.M;
      ro[i][r] = rok[i][r] ? map3(d.cm, (unsigned)m) : 0;
    }

  auto ldb = [&](S (&br)[KS], S (&bi)[KS], int jb) {
    const int n = min(jb * 16 + r16, d.N - 1);
    const long long bo = map3(d.bn, (unsigned)n);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const S2 v = MM::cvt(B[bo + bko[s]]);
      br[s] = v.x;
      bi[s] = flip(v.y, mb);
    }
  };
  // PLAIN: alpha = 1 and beta = 0, without the scaling and the read of C
  auto blk = [&](const S (&br)[KS], const S (&bi)[KS], int jb, auto plain) {
    Acc cr[2], ci[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) cr[i] = ci[i] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        cr[i] = MM::run(ar[i][s], br[s], cr[i]);
        ci[i] = MM::run(ar[i][s], bi[s], ci[i]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        cr[i] = MM::run_neg(ai[i][s], bi[s], cr[i]);
        ci[i] = MM::run(ai[i][s], br[s], ci[i]);
      }
    }
    const int n = jb * 16 + r16;
    if (n >= d.N) return;
    const long long con = map3(d.cn, (unsigned)n);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!rok[i][r]) continue;
        const long long o = ro[i][r] + con;
        const double xr = (double)cr[i][r], xi = (double)ci[i][r];
        double2 v;
        if constexpr (decltype(plain)::value) {
          v.x = xr;
          v.y = xi;
        } else {
          v.x = d.alpha_r * xr - d.alpha_i * xi;
          v.y = d.alpha_r * xi + d.alpha_i * xr;
          if (!d.beta_zero) {
            const double2 c = to_d2(C[o]);
            v.x += d.beta_r * c.x - d.beta_i * c.y;
            v.y += d.beta_r * c.y + d.beta_i * c.x;
          }
        }
        C[o] = from_d2<TC>(v);
      }
  };

  // j0 < j1: run < ceil(nblk / kProdBlocks).  The prefetches are not under
  // a branch (the block index is clamped; the last one goes unused), or the
  // compiler waits for them right after issuing them.
  const int nblk = (d.N + 15) / 16;
  const int j0 = (int)run * kProdBlocks, j1 = min(j0 + kProdBlocks, nblk);
  auto walk = [&](auto plain) {
    S br0[KS], bi0[KS], br1[KS], bi1[KS];
    int jb = j0;
    ldb(br0, bi0, jb);
    for (; jb + 2 <= j1; jb += 2) {
      ldb(br1, bi1, jb + 1);
      // keep the prefetch ahead of this block's MFMAs (the scheduler would
      // sink it into them and shorten its cover)
      __builtin_amdgcn_sched_barrier(0);
      blk(br0, bi0, jb, plain);
      ldb(br0, bi0, min(jb + 2, j1 - 1));
      __builtin_amdgcn_sched_barrier(0);
      blk(br1, bi1, jb + 1, plain);
    }
    if (jb < j1) blk(br0, bi0, jb, plain);
  };
  if (d.beta_zero && d.alpha_r == 1.0 && d.alpha_i == 0.0)
    walk(std::true_type{});
  else
    walk(std::false_type{});
}

template <int TAG, class TA, class TB, class TC, bool F32>
static hipError_t launch_prod(const GemmDesc& d0, hipStream_t st) {
  GemmDesc d = d0;
  if (d.K > 32 || d.tri || d.tmod <= 0) return hipErrorInvalidValue;
  const long long tiles_m = (d.M + kProdRows - 1) / kProdRows;
  const long long nrun = ((d.N + 15) / 16 + kProdBlocks - 1) / kProdBlocks;
  const long long total = tiles_m * nrun * d.batch;
  if (tiles_m * nrun > 0x7fffffffLL || total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  d.q_tiles_m = udiv_make((unsigned)nrun);
  d.q_tiles = udiv_make((unsigned)(tiles_m * nrun));
  d.q_batch = udiv_make((unsigned)d.batch);
  d.q_tmod = udiv_make((unsigned)d.tmod);
  const dim3 grid((unsigned)total, 1, 1);
  if (d.K <= 8)
    prod_k<TAG, 2, TA, TB, TC, F32><<<grid, 256, 0, st>>>(d);
  else if (d.K <= 16)
    prod_k<TAG, 4, TA, TB, TC, F32><<<grid, 256, 0, st>>>(d);
  else if (d.K <= 28)
    prod_k<TAG, 7, TA, TB, TC, F32><<<grid, 256, 0, st>>>(d);
  else
    prod_k<TAG, 8, TA, TB, TC, F32><<<grid, 256, 0, st>>>(d);
  return hipGetLastError();
}

static bool one_carry(const Map3& m, unsigned st) {
  return m.din >= st && (unsigned long long)m.din * m.dmid >= st;
}

// Upper bound of map3(m, i) over 0 <= i < n for non-negative strides.
static long long map_max(const Map3& m, long long n) {
  if (n <= 0) return 0;
  const unsigned long long last = (unsigned long long)(n - 1), da = m.din, dm = m.dmid;
  const unsigned long long a = std::min(da - 1ull, last), b = std::min(dm - 1ull, last / da);
  const unsigned long long c = last / (da * dm);
  return (long long)c * m.sout + (long long)b * m.smid + (long long)a * m.sin;
}

static bool nonneg(const Map3& m) { return m.sout >= 0 && m.smid >= 0 && m.sin >= 0; }

// The uniform K loop (KM = 2) needs: every K map either never wraps inside
// [0, K) or wraps at multiples of 4 (then the four k of a step, which start
// at a multiple of 4, share all digits but the last); non-negative row,
// column and K strides; and lane offset + K offset below 2^31 bytes.
static bool uniform_k(const GemmDesc& d, unsigned kstep, long long ea, long long eb) {
  auto aligned = [&](const Map3& m) {
    return (m.din >= (unsigned)d.K || m.din % 4u == 0u) && one_carry(m, kstep);
  };
  if (!aligned(d.ak) || !aligned(d.bk)) return false;
  if (!nonneg(d.am) || !nonneg(d.ak) || !nonneg(d.bk) || !nonneg(d.bn)) return false;
  const long long lim = 0x7fffffffLL;
  const long long va = (map_max(d.am, d.M) + 3 * d.ak.sin) * ea, ka = map_max(d.ak, d.K) * ea;
  const long long vb = (map_max(d.bn, d.N) + 3 * d.bk.sin) * eb, kb = map_max(d.bk, d.K) * eb;
  return va + ka + ea <= lim && vb + kb + eb <= lim;
}

// The fp64 polarization contraction (uniform-K loop) reserves LDS it does
// not use, so that at most two workgroups share a CU: the tiles of one tau
// then drift less apart in K and meet more often in L2 (measured at
// si-4x4x4: 24.0 ms per launch against 25.5 ms with four workgroups per CU
// and 32.0 ms with one).
template <int TAG, bool F32>
static constexpr size_t residency_lds() {
  return (TAG == KC_POL_CONTRACT && !F32) ? size_t(60000) : size_t(0);
}

template <int WM, int WN, int WK, int BM, int BN, int TAG, class TA, class TB, class TC, bool F32,
          bool G3 = false>
static hipError_t launch_cfg(const GemmDesc& d0, hipStream_t st) {
  constexpr int TM = WM * BM * 16, TN = WN * BN * 16;
  const long long tm_ = (d0.M + TM - 1) / TM;
  if (d0.tri && (d0.M != d0.N || TM != TN)) return hipErrorInvalidValue;
  const long long tiles = d0.tri ? tm_ * (tm_ + 1) / 2 : tm_ * ((d0.N + TN - 1) / TN);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (tiles * (long long)d0.batch > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  if (d0.tmod <= 0) return hipErrorInvalidValue;
  GemmDesc d = d0;
  d.q_tiles_m = udiv_make((unsigned)((d.M + TM - 1) / TM));
  d.q_tiles = udiv_make((unsigned)tiles);
  d.q_batch = udiv_make((unsigned)d.batch);
  d.q_tmod = udiv_make((unsigned)d.tmod);
  dim3 grid((unsigned)(tiles * d.batch), 1, 1);
  const unsigned kstep = 4u * WK;
  if (F32 && d.kchunk > 0 && d.kchunk % kstep) return hipErrorInvalidValue;
  constexpr int nt = 64 * WM * WN * WK;
  if (uniform_k(d, kstep, sizeof(TA), sizeof(TB)))
    zgemm_k<WM, WN, WK, BM, BN, TAG, 2, TA, TB, TC, F32, G3><<<grid, nt, residency_lds<TAG, F32>(), st>>>(d);
  else if (one_carry(d.ak, kstep) && one_carry(d.bk, kstep))
    zgemm_k<WM, WN, WK, BM, BN, TAG, 1, TA, TB, TC, F32><<<grid, nt, 0, st>>>(d);
  else
    zgemm_k<WM, WN, WK, BM, BN, TAG, 0, TA, TB, TC, F32><<<grid, nt, 0, st>>>(d);
  return hipGetLastError();
}

// Tile shape: 32 x 32 with four-way split K for small outputs; 64 x 128 for
// the producers; otherwise 64 x 64, or for the two large fp64 contractions
// the configuration in d.cfg
// (0: 64x64, 1: 64x128, 2: 128x64, 3: 128x64 on eight waves, 4: 64x64 with
// two-way split K; 5..9 the three-product form on 64x64, 64x128, 64x96,
// 128x64 on eight waves, 128x64).  Measured at si-4x4x4 (ms per q, fp64):
// polarization 22.6 (0) vs 23.3 (5), 28.0 (4); self-energy 31.7 (1) vs 25.7
// (7), 27.2 (5), 28.6 (8), 34.5 (6), 35.2 (9) -- 6 and 9 need more than 256
// VGPRs and run one wave per SIMD; loads two K-steps ahead (a third register
// stage) gained nothing on either.  The producers (K = nao) gain nothing
// from the three-product form (11.7 vs 12.0 ms), their stores bound them.
template <int TAG, class TA, class TB, class TC, bool F32>
static hipError_t launch_typed(const GemmDesc& d, hipStream_t st) {
  if (d.M <= 32 && d.N <= 32) return launch_cfg<1, 1, 4, 2, 2, TAG, TA, TB, TC, F32>(d, st);
  if constexpr ((TAG == KC_POL_CONTRACT || TAG == KC_SE_CONTRACT) && !F32) {
    switch (d.cfg) {
      case 1: return launch_cfg<2, 2, 1, 2, 4, TAG, TA, TB, TC, F32>(d, st);
      case 2: return launch_cfg<2, 2, 1, 4, 2, TAG, TA, TB, TC, F32>(d, st);
      case 3: return launch_cfg<4, 2, 1, 2, 2, TAG, TA, TB, TC, F32>(d, st);
      case 4: return launch_cfg<2, 2, 2, 2, 2, TAG, TA, TB, TC, F32>(d, st);
      case 5: return launch_cfg<2, 2, 1, 2, 2, TAG, TA, TB, TC, F32, true>(d, st);
      case 6: return launch_cfg<2, 2, 1, 2, 4, TAG, TA, TB, TC, F32, true>(d, st);
      case 7: return launch_cfg<2, 2, 1, 2, 3, TAG, TA, TB, TC, F32, true>(d, st);
      case 8: return launch_cfg<4, 2, 1, 2, 2, TAG, TA, TB, TC, F32, true>(d, st);
      case 9: return launch_cfg<2, 2, 1, 4, 2, TAG, TA, TB, TC, F32, true>(d, st);
      default: break;
    }
  }
  // fp32 MFMA steps are half as long, so the two large contractions split K
  // over two waves per output block (64 x 64, 8 waves): measured 19.2 vs
  // 20.5 ms (polarization) and 22.6 vs 26.0 ms (self-energy) per q
  // The product form follows d.cfg (5..9: three products), the tile does
  // not: the fp32 self-energy contraction (default 7) runs three products,
  // 19.9-20.3 vs 23.1 ms per q, the polarization one (default 0) four, 19.1
  // vs 19.9 ms.
  if constexpr ((TAG == KC_POL_CONTRACT || TAG == KC_SE_CONTRACT) && F32) {
    if (d.cfg >= 5 && d.cfg <= 9) return launch_cfg<2, 2, 2, 2, 2, TAG, TA, TB, TC, F32, true>(d, st);
    return launch_cfg<2, 2, 2, 2, 2, TAG, TA, TB, TC, F32>(d, st);
  }
  // the producers (K = nao): fp32 MFMA (complex64 intermediates) on the
  // streaming kernel (measured 7.7 vs 8.2 ms per polarization call and 3.8
  // vs 4.0 ms per self-energy producer at si-4x4x4); fp64 on 64 x 128 tiles,
  // which give each wave twice the MFMA work per load latency of 64 x 64
  // ones (12.6 vs 14.0 ms) and beat the streaming kernel (11.7 vs 12.9 ms)
  if constexpr (TAG == KC_POL_PRODUCER || TAG == KC_SE_PRODUCER) {
    if constexpr (F32) {
      if (d.K <= 32 && !d.tri && d.cfg != 1) return launch_prod<TAG, TA, TB, TC, F32>(d, st);
    }
    return launch_cfg<2, 2, 1, 2, 4, TAG, TA, TB, TC, F32>(d, st);
  }
  return launch_cfg<2, 2, 1, 2, 2, TAG, TA, TB, TC, F32>(d, st);
}

// Storage / precision combinations, only those each kernel class uses:
// fp64 everywhere; in the mixed-precision path complex64 V and
// intermediates with fp32 MFMA, and complex64 V read by the fp64 HF terms.
template <int TAG>
static hipError_t launch_tag(const GemmDesc& d, hipStream_t st) {
  const int code = d.ta | (d.tb << 1) | (d.tc << 2) | (d.f32 << 3);
  if (code == 0) return launch_typed<TAG, double2, double2, double2, false>(d, st);
  if constexpr (TAG == KC_HF) {
    if (code == 1) return launch_typed<TAG, float2, double2, double2, false>(d, st);
    if (code == 2) return launch_typed<TAG, double2, float2, double2, false>(d, st);
  }
  if constexpr (TAG == KC_POL_PRODUCER || TAG == KC_SE_PRODUCER) {
    if (code == (8 | 1 | 2 | 4)) return launch_typed<TAG, float2, float2, float2, true>(d, st);
    // mixed-precision VJP: complex64 V times a complex128 G or cotangent
    if (code == (8 | 1 | 4)) return launch_typed<TAG, float2, double2, float2, true>(d, st);
    if (code == (8 | 2 | 4)) return launch_typed<TAG, double2, float2, float2, true>(d, st);
  }
  if constexpr (TAG == KC_POL_CONTRACT || TAG == KC_SE_FINAL) {
    if (code == (8 | 1 | 2)) return launch_typed<TAG, float2, float2, double2, true>(d, st);
  }
  if constexpr (TAG == KC_SE_CONTRACT) {
    if (code == (8 | 2 | 4)) return launch_typed<TAG, double2, float2, float2, true>(d, st);
  }
  return hipErrorInvalidValue;
}

bool zgemm_three_product(const GemmDesc& d) {
  if (d.tag != KC_POL_CONTRACT && d.tag != KC_SE_CONTRACT) return false;
  if (d.cfg < 5 || d.cfg > 9 || (d.M <= 32 && d.N <= 32)) return false;
  // the fp32 tile splits K over two waves: K-steps of 8
  return uniform_k(d, d.f32 ? 8u : 4u, d.ta ? 8 : 16, d.tb ? 8 : 16);
}

hipError_t zgemm_launch(const GemmDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.K <= 0) return hipErrorInvalidValue;
  switch (d.tag) {
    case KC_POL_CONTRACT: return launch_tag<KC_POL_CONTRACT>(d, st);
    case KC_POL_PRODUCER: return launch_tag<KC_POL_PRODUCER>(d, st);
    case KC_SE_CONTRACT: return launch_tag<KC_SE_CONTRACT>(d, st);
    case KC_SE_PRODUCER: return launch_tag<KC_SE_PRODUCER>(d, st);
    case KC_SE_FINAL: return launch_tag<KC_SE_FINAL>(d, st);
    case KC_TRANSFORM: return launch_tag<KC_TRANSFORM>(d, st);
    case KC_HF: return launch_tag<KC_HF>(d, st);
    default: return launch_tag<0>(d, st);
  }
}

// ---------------------------------------------------------------------------
// Split-bf16 complex GEMM (bf16x3), the mixed-precision form of the two large
// contractions:  C[b](m, n) = alpha * sum_k A[b](m, k) B[b](n, k) + beta C[b](m, n)
// with A(m, k) = A[ba(b) + am(m) + k aks] and B(n, k) = B[bb(b) + bn(n) + k bks],
// complex128 or complex64 in memory.  Each K-step of 32 brings the A and B
// tiles into LDS, splitting every real part x on the way into NS bf16 levels
// (round to nearest even): NS = 2, x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi) (16 significant bits); NS = 3, x = hi + mid + lo (24).
// A real product is the sum of the level products a_u b_v with u + v < NS on
// v_mfma_f32_16x16x32_bf16: a_hi b_hi + a_hi b_lo + a_lo b_hi (bf16x3; the
// dropped terms and residuals are near 2^-17 |a b|), or the six products up
// to u + v = 2 (bf16x6, near 2^-24, the fp32 rounding).  The Im(a) Im(b)
// part of Re(a b) accumulates on its own and is subtracted at the end of each
// chunk, so the loop has no sign flips.
// LDS row of a tile: 32 k as 2 NS planes [level 0 re][level 0 im][level 1
// re]... of 8 x 4 bf16 (64 bytes each), rows row_bytes(NS) apart (16 bytes of
// padding spread the rows of one fragment read over the banks); two stages,
// so the global loads and splits of step s + 1 overlap the MFMAs of step s.
// Loader: each thread owns chunks of 8 consecutive k of one row; with aks = 1
// four threads read a row's 32 k (k-contiguous operands), otherwise
// consecutive threads take consecutive rows (operands contiguous along the
// rows, e.g. V with k = Q').  k >= K reads zeros.
// MFMA operand layout: lane l holds row l % 16 and k = 8 (l / 16) .. +7 of A
// (column l % 16, same k, of B); the result holds column l % 16 and rows
// 4 (l / 16) .. +3.  Waves: WM x WN tile the output, each BM x BN blocks.
// SUMS: fp32 accumulation inside chunks of d.kchunk k, each chunk added into
// a SUMT (fp64 or fp32) sum; without them (K <= kchunk) one fp32 chunk.
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
template <int NS> static constexpr int row_bytes() { return 128 * NS + 16; }

template <class T> struct Chunk;
template <> struct Chunk<float2> { float2 v[8]; };
template <> struct Chunk<double2> { double2 v[8]; };

// loads 8 consecutive k (stride ks elements, 1 if CONTIG) from p; k >= K
// gives zeros
// A chunk whose eight k all lie below K: no branch, so that the loads of the
// next K-step stay in flight while the MFMAs of the current one run (a
// branch around them makes the compiler wait for them at once).
template <bool CONTIG, class T>
__device__ __forceinline__ void load_chunk_full(Chunk<T>& c, const T* p, long long ks, int k0) {
  if constexpr (CONTIG) {
#pragma unroll
    for (int e = 0; e < 8; ++e) c.v[e] = p[k0 + e];
  } else {
    // byte stride as a wave-uniform 32-bit value: the eight addresses are
    // scalar offsets from one per-lane pointer
    const unsigned sb = __builtin_amdgcn_readfirstlane((unsigned)(ks * (long long)sizeof(T)));
    const char* q = (const char*)(p + (long long)k0 * ks);
#pragma unroll
    for (int e = 0; e < 8; ++e) c.v[e] = *(const T*)(q + (unsigned)e * sb);
  }
}

// Any chunk (the last, partial K-step): k past K reads zeros.
template <bool CONTIG, class T>
__device__ __forceinline__ void load_chunk(Chunk<T>& c, const T* p, long long ks, int k0, int K) {
  if (k0 + 8 <= K) {
    load_chunk_full<CONTIG>(c, p, ks, k0);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + e;
      const T z{0, 0};
      c.v[e] = k < K ? p[(long long)k * ks] : z;
    }
  }
}

// split 8 complex values into NS levels and write the 2 NS planes of one LDS
// chunk (16 bytes each, 64 bytes apart)
template <int NS, class T>
__device__ __forceinline__ void put_chunk(const Chunk<T>& c, unsigned char* row, int kgc) {
  float re[8], im[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    re[e] = (float)c.v[e].x;
    im[e] = (float)c.v[e].y;
  }
  uint4* q = (uint4*)(row + 16 * kgc);
#pragma unroll
  for (int l = 0; l < NS; ++l) {
    uint4 pr, pi;
    unsigned* ur = (unsigned*)&pr;
    unsigned* ui = (unsigned*)&pi;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ur[i] = pack_bf16(re[2 * i], re[2 * i + 1]);
      ui[i] = pack_bf16(im[2 * i], im[2 * i + 1]);
      if (l + 1 < NS) {                 // residuals for the next level
        re[2 * i] -= bf16_low(ur[i]);
        re[2 * i + 1] -= bf16_high(ur[i]);
        im[2 * i] -= bf16_low(ui[i]);
        im[2 * i + 1] -= bf16_high(ui[i]);
      }
    }
    q[8 * l] = pr;
    q[8 * l + 4] = pi;
  }
}

template <int WM, int WN, int BM, int BN, int TAG, class TA, class TB, class TC, bool SUMS, bool AK1, bool BK1,
          class SUMT, int NS, int NSTG = 2>
__global__ void __launch_bounds__(64 * WM * WN) bsgemm_k(SplitDesc d) {
  static_assert(NSTG == 1 || NSTG == 2, "one or two LDS stages");
  constexpr int kRowB = row_bytes<NS>();
  constexpr int NT = 64 * WM * WN, TM = WM * BM * 16, TN = WN * BN * 16;
  constexpr int CA = TM * 4 / NT, CB = TN * 4 / NT;   // loader chunks per thread
  static_assert(CA >= 1 && CB >= 1 && CA * NT == TM * 4 && CB * NT == TN * 4, "loader split");
  constexpr int STAGE = (TM + TN) * kRowB;
  __shared__ __attribute__((aligned(16))) unsigned char lds[NSTG * STAGE];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % WM, wn = wave / WM;
  const TilePos tp = tile_pos(d, TM, TN);
  const TA* A = (const TA*)d.A + map3(d.ba, tp.bt);
  const TB* B = (const TB*)d.B + map3(d.bb, tp.bt);
  const int tm0 = tp.tm * TM, tn0 = tp.tn * TN;

  // loader rows (clamped to the last row: their outputs are dropped); AK1,
  // BK1: the operand's K stride is 1
  constexpr bool acontig = AK1, bcontig = BK1;
  const TA* pa[CA];
  const TB* pb[CB];
  int ra[CA], ka[CA], rb[CB], kb[CB];
#pragma unroll
  for (int u = 0; u < CA; ++u) {
    const int c = tid + u * NT;
    ra[u] = acontig ? c >> 2 : c % TM;
    ka[u] = acontig ? c & 3 : c / TM;
    pa[u] = A + map3(d.am, (unsigned)min(tm0 + ra[u], d.M - 1));
  }
#pragma unroll
  for (int u = 0; u < CB; ++u) {
    const int c = tid + u * NT;
    rb[u] = bcontig ? c >> 2 : c % TN;
    kb[u] = bcontig ? c & 3 : c / TN;
    pb[u] = B + map3(d.bn, (unsigned)min(tn0 + rb[u], d.N - 1));
  }
  Chunk<TA> ca[CA];
  Chunk<TB> cb[CB];
  auto fetch = [&](int s) {
#pragma unroll
    for (int u = 0; u < CA; ++u) load_chunk<AK1>(ca[u], pa[u], d.aks, 32 * s + 8 * ka[u], d.K);
#pragma unroll
    for (int u = 0; u < CB; ++u) load_chunk<BK1>(cb[u], pb[u], d.bks, 32 * s + 8 * kb[u], d.K);
  };
  auto fetch_full = [&](int s) {
#pragma unroll
    for (int u = 0; u < CA; ++u) load_chunk_full<AK1>(ca[u], pa[u], d.aks, 32 * s + 8 * ka[u]);
#pragma unroll
    for (int u = 0; u < CB; ++u) load_chunk_full<BK1>(cb[u], pb[u], d.bks, 32 * s + 8 * kb[u]);
  };
  auto stash = [&](int stage) {
    unsigned char* base = lds + stage * STAGE;
#pragma unroll
    for (int u = 0; u < CA; ++u) put_chunk<NS>(ca[u], base + ra[u] * kRowB, ka[u]);
#pragma unroll
    for (int u = 0; u < CB; ++u) put_chunk<NS>(cb[u], base + (TM + rb[u]) * kRowB, kb[u]);
  };

  f4 accR[BM][BN], accN[BM][BN], accI[BM][BN];
  SUMT sumR[SUMS ? BM : 1][SUMS ? BN : 1][4], sumI[SUMS ? BM : 1][SUMS ? BN : 1][4];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int j = 0; j < BN; ++j) accR[i][j] = accN[i][j] = accI[i][j] = f4{0, 0, 0, 0};
  if constexpr (SUMS) {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) sumR[i][j][r] = sumI[i][j][r] = SUMT(0);
  }
  auto promote = [&]() {
    if constexpr (SUMS) {
#pragma unroll
      for (int i = 0; i < BM; ++i)
#pragma unroll
        for (int j = 0; j < BN; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            sumR[i][j][r] += (SUMT)accR[i][j][r] - (SUMT)accN[i][j][r];
            sumI[i][j][r] += (SUMT)accI[i][j][r];
          }
          accR[i][j] = accN[i][j] = accI[i][j] = f4{0, 0, 0, 0};
        }
    }
  };
  const int r16 = lane & 15, kg = lane >> 4;
  auto bf = [](const uint4& v) { return __builtin_bit_cast(bf8v, v); };
  // one K-step from LDS stage `stage`: planes 0 hi(re), 1 hi(im), 2 lo(re),
  // 3 lo(im).  Terms (hi, hi), (hi, lo), (lo, hi) in three phases, each
  // reading only the planes it adds.
  auto rd = [&](const unsigned char* base, int row0, int p) {
    return *(const uint4*)(base + (row0 + r16) * kRowB + 16 * kg + 64 * p);
  };
  auto terms = [&](const uint4 (&ar)[BM], const uint4 (&ai)[BM], const uint4 (&br)[BN], const uint4 (&bi)[BN]) {
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(ar[i]), bf(br[j]), accR[i][j], 0, 0, 0);
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(ar[i]), bf(bi[j]), accI[i][j], 0, 0, 0);
        accN[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(ai[i]), bf(bi[j]), accN[i][j], 0, 0, 0);
      }
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int j = 0; j < BN; ++j)
        accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf(ai[i]), bf(br[j]), accI[i][j], 0, 0, 0);
  };
  auto compute = [&](int stage) {
    const unsigned char* base = lds + stage * STAGE;
    const int ra0 = wm * BM * 16, rb0 = TM + wn * BN * 16;
    // all B levels, then A level by level with the B levels v < NS - u
    uint4 br[NS][BN], bi[NS][BN];
#pragma unroll
    for (int l = 0; l < NS; ++l)
#pragma unroll
      for (int j = 0; j < BN; ++j) {
        br[l][j] = rd(base, rb0 + 16 * j, 2 * l);
        bi[l][j] = rd(base, rb0 + 16 * j, 2 * l + 1);
      }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      uint4 ar[BM], ai[BM];
#pragma unroll
      for (int i = 0; i < BM; ++i) {
        ar[i] = rd(base, ra0 + 16 * i, 2 * u);
        ai[i] = rd(base, ra0 + 16 * i, 2 * u + 1);
      }
#pragma unroll
      for (int v = 0; v + u < NS; ++v) terms(ar, ai, br[v], bi[v]);
    }
  };

  // step t's chunks live in LDS stage t % 2; the loads of step s + 1 are
  // issued before the MFMAs of step s.  The main loop prefetches only full
  // K-steps (no branch around the loads); the partial last step, if any,
  // goes through the second loop.
  const int nsteps = (d.K + 31) / 32, nfull = d.K / 32;
  const int cper = d.kchunk / 32;
  fetch(0);
  stash(0);
  __syncthreads();
  int s = 0;
  // one LDS stage: the next step's chunks wait in registers until every wave
  // has read the stage (a second barrier per step, half the LDS)
  auto stg = [](int t) { return NSTG == 2 ? (t & 1) : 0; };
  for (; s + 1 < nfull; ++s) {
    fetch_full(s + 1);
    compute(stg(s));
    if constexpr (NSTG == 1) __syncthreads();
    stash(stg(s + 1));
    if ((s + 1) % cper == 0) promote();
    __syncthreads();
  }
  for (; s < nsteps; ++s) {
    if (s + 1 < nsteps) fetch(s + 1);
    compute(stg(s));
    if constexpr (NSTG == 1) __syncthreads();
    if (s + 1 < nsteps) stash(stg(s + 1));
    if ((s + 1) % cper == 0) promote();
    __syncthreads();
  }
  promote();

  // epilogue: fp32 MFMA result layout, rows 4 (lane / 16) + r, column lane % 16
  auto res = [&](int i, int j, int r, bool im) -> double {
    if constexpr (SUMS) return im ? (double)sumI[i][j][r] : (double)sumR[i][j][r];
    else return im ? (double)accI[i][j][r] : (double)accR[i][j][r] - (double)accN[i][j][r];
  };
  TC* C = (TC*)d.C + map3(d.bc, tp.bt);
  const int m0 = tm0 + wm * BM * 16, n0 = tn0 + wn * BN * 16;
  long long roff[BM][4];
  bool rok[BM][4];
#pragma unroll
  for (int i = 0; i < BM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + i * 16 + 4 * kg + r;
      rok[i][r] = m < d.M;
      roff[i][r] = rok[i][r] ? map3(d.cm, m) : 0;
    }
#pragma unroll
  for (int j = 0; j < BN; ++j) {
    const int n = n0 + j * 16 + r16;
    if (n >= d.N) continue;
    const long long con = map3(d.cn, n);
#pragma unroll
    for (int i = 0; i < BM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (!rok[i][r]) continue;
        const long long o = roff[i][r] + con;
        double2 v{d.alpha_r * res(i, j, r, false), d.alpha_r * res(i, j, r, true)};
        if (!d.beta_zero) {
          const double2 c = to_d2(C[o]);
          v.x += d.beta_r * c.x;
          v.y += d.beta_r * c.y;
        }
        C[o] = from_d2<TC>(v);
      }
  }
}

template <int WM, int WN, int BM, int BN, int TAG, class TA, class TB, class TC, bool SUMS, bool AK1, bool BK1,
          class SUMT, int NS, int NSTG = 2>
static hipError_t bs_cfg(const SplitDesc& d0, hipStream_t st) {
  constexpr int TM = WM * BM * 16, TN = WN * BN * 16;
  const long long tm_ = (d0.M + TM - 1) / TM;
  if (d0.tri && (d0.M != d0.N || TM != TN)) return hipErrorInvalidValue;
  if (!SUMS && d0.K > d0.kchunk) return hipErrorInvalidValue;
  if (d0.batch_fastest == 2 && d0.group <= 0) return hipErrorInvalidValue;
  const long long tiles = d0.tri ? tm_ * (tm_ + 1) / 2 : tm_ * ((d0.N + TN - 1) / TN);
  if (tiles * (long long)d0.batch > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  SplitDesc d = d0;
  d.q_tiles_m = udiv_make((unsigned)tm_);
  d.q_tiles = udiv_make((unsigned)tiles);
  d.q_batch = udiv_make((unsigned)d.batch);
  if ((d0.aks == 1) != AK1 || (d0.bks == 1) != BK1) return hipErrorInvalidValue;
  bsgemm_k<WM, WN, BM, BN, TAG, TA, TB, TC, SUMS, AK1, BK1, SUMT, NS, NSTG><<<dim3((unsigned)(tiles * d.batch)), 64 * WM * WN, 0, st>>>(d);
  return hipGetLastError();
}

// Tile configurations (d.cfg < 0: the default of the role).  Polarization
// (complex64 operands, long K, square tiles for the Hermitian mode): 64x64 on
// 4 waves, the 512-term fp32 chunks summed in fp32:
// 229 VGPRs, so two workgroups share a CU (7.2 ms per q at si-4x4x4, against
// 10.9 ms with fp64 chunk sums and loads three steps ahead, 309 VGPRs, one
// workgroup per CU; the outer fp32 sum's rounding, ~1e-7 relative, is far
// below the bf16x3 product error).  Self-energy
// P~ V (complex64 P~ and V, K = naux <= kchunk):
// 0 128x128 on 8 waves (4 x 2 blocks each), 1 64x64 on 4 waves, 2 128x64 on
// 4 waves (4 x 2).
hipError_t bsgemm_launch(const SplitDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
  if (d.K <= 0 || d.kchunk <= 0 || d.kchunk % 32) return hipErrorInvalidValue;
  // the polarization's operands have K contiguous; the self-energy's V has
  // K = Q' with stride n2
  if (d.nsplit == 3) {
    // bf16x6: fp64 chunk sums (the products are as accurate as fp32 ones);
    // 64 x 64 tiles, as 128 x 128 ones would need 205 KB of LDS with two
    // stages, and the loader needs at least one chunk of each operand per
    // thread
    // One LDS stage (51 KB) lets two workgroups share a CU where two stages
    // (102 KB) allow one: 8.7 vs 9.8 ms (polarization) and 14.3 vs 22.1 ms
    // (self-energy) per q at si-4x4x4.  d.cfg = 1 selects two stages.
    if (d.tag == KC_POL_CONTRACT && d.ta == 1 && d.tb == 1 && d.tc == 0) {
      if (d.cfg == 1)
        return bs_cfg<2, 2, 2, 2, KC_POL_CONTRACT, float2, float2, double2, true, true, true, double, 3>(d, st);
      return bs_cfg<2, 2, 2, 2, KC_POL_CONTRACT, float2, float2, double2, true, true, true, double, 3, 1>(d, st);
    }
    if (d.tag == KC_SE_CONTRACT && d.ta == 1 && d.tb == 1 && d.tc == 1) {
      if (d.K > d.kchunk)
        return bs_cfg<2, 2, 2, 2, KC_SE_CONTRACT, float2, float2, float2, true, true, false, double, 3, 1>(d, st);
      if (d.cfg == 1)
        return bs_cfg<2, 2, 2, 2, KC_SE_CONTRACT, float2, float2, float2, false, true, false, double, 3>(d, st);
      return bs_cfg<2, 2, 2, 2, KC_SE_CONTRACT, float2, float2, float2, false, true, false, double, 3, 1>(d, st);
    }
    return hipErrorInvalidValue;
  }
  if (d.nsplit != 2) return hipErrorInvalidValue;
  if (d.tag == KC_POL_CONTRACT && d.ta == 1 && d.tb == 1 && d.tc == 0)
    return bs_cfg<2, 2, 2, 2, KC_POL_CONTRACT, float2, float2, double2, true, true, true, float, 2>(d, st);
  if (d.tag == KC_SE_CONTRACT && d.ta == 1 && d.tb == 1 && d.tc == 1) {
    if (d.K > d.kchunk)
      return bs_cfg<2, 2, 2, 2, KC_SE_CONTRACT, float2, float2, float2, true, true, false, double, 2>(d, st);
    switch (d.cfg) {
      case 1: return bs_cfg<2, 2, 2, 2, KC_SE_CONTRACT, float2, float2, float2, false, true, false, double, 2>(d, st);
      case 2: return bs_cfg<2, 2, 4, 2, KC_SE_CONTRACT, float2, float2, float2, false, true, false, double, 2>(d, st);
      default: return bs_cfg<2, 4, 4, 2, KC_SE_CONTRACT, float2, float2, float2, false, true, false, double, 2>(d, st);
    }
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Lower triangle from the upper one: P[b](r, c) = conj(P[b](c, r)) for r > c.
// Grid: x over the n*n entries of a matrix, y over the matrices; threads on
// or above the diagonal do nothing.
__global__ void herm_fill_k(double2* P, int n) {
  const unsigned nn = (unsigned)n * (unsigned)n;
  const unsigned e = blockIdx.x * 256u + threadIdx.x;
  if (e >= nn) return;
  const unsigned r = e / (unsigned)n, c = e - r * (unsigned)n;
  if (r <= c) return;
  double2* M = P + (size_t)blockIdx.y * nn;
  const double2 v = M[(size_t)c * n + r];
  M[e] = double2{v.x, -v.y};
}

// Hermitian part: one thread per entry (r, c) with r <= c of each matrix; it
// reads both mirror entries and writes both.
__global__ void herm_avg_k(double2* P, int n) {
  const unsigned nn = (unsigned)n * (unsigned)n;
  const unsigned e = blockIdx.x * 256u + threadIdx.x;
  if (e >= nn) return;
  const unsigned r = e / (unsigned)n, c = e - r * (unsigned)n;
  if (r > c) return;
  double2* M = P + (size_t)blockIdx.y * nn;
  const double2 a = M[e], b = M[(size_t)c * n + r];
  const double2 v = double2{0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
  M[e] = v;
  M[(size_t)c * n + r] = double2{v.x, -v.y};
}

hipError_t herm_avg_launch(double2* P, int n, long long nmat, hipStream_t st) {
  if (n <= 0 || nmat <= 0) return hipSuccess;
  if (nmat > 65535 || (long long)n * n > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const unsigned bx = (unsigned)(((long long)n * n + 255) / 256);
  herm_avg_k<<<dim3(bx, (unsigned)nmat, 1), 256, 0, st>>>(P, n);
  return hipGetLastError();
}

// Finite-size corrections (Eqs. K_corr, GW_head_corr): one workgroup per
// matrix b.  T = X[b] S[k] is formed in LDS (one thread per entry, a row of
// X times a column of S), then every thread adds alpha (S[k] T)(i, j) for its
// entries.  n <= 64, so T fits in 64 KiB of LDS.
__global__ void __launch_bounds__(256) sxs_add_k(const double2* S, const double2* X, double2* Out,
                                                 int n, int nk, double alpha) {
  __shared__ double2 T[64 * 64];
  const unsigned nn = (unsigned)n * (unsigned)n;
  const unsigned b = blockIdx.x;
  const double2* Sk = S + (size_t)(b % (unsigned)nk) * nn;
  const double2* Xb = X + (size_t)b * nn;
  for (unsigned e = threadIdx.x; e < nn; e += 256u) {
    const unsigned r = e / (unsigned)n, c = e - r * (unsigned)n;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < n; ++a) {
      const double2 x = Xb[(size_t)r * n + a], s = Sk[(size_t)a * n + c];
      re += x.x * s.x - x.y * s.y;
      im += x.x * s.y + x.y * s.x;
    }
    T[e] = double2{re, im};
  }
  __syncthreads();
  double2* Ob = Out + (size_t)b * nn;
  for (unsigned e = threadIdx.x; e < nn; e += 256u) {
    const unsigned r = e / (unsigned)n, c = e - r * (unsigned)n;
    double re = 0.0, im = 0.0;
    for (int a = 0; a < n; ++a) {
      const double2 s = Sk[(size_t)r * n + a], x = T[(unsigned)a * (unsigned)n + c];
      re += s.x * x.x - s.y * x.y;
      im += s.x * x.y + s.y * x.x;
    }
    const double2 o = Ob[e];
    Ob[e] = double2{o.x + alpha * re, o.y + alpha * im};
  }
}

hipError_t sxs_add_launch(const double2* S, const double2* X, double2* Out, int n, int nk,
                          long long nmat, double alpha, hipStream_t st) {
  if (n <= 0 || nmat <= 0) return hipSuccess;
  if (n > 64 || nk <= 0 || nmat > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  sxs_add_k<<<dim3((unsigned)nmat, 1, 1), 256, 0, st>>>(S, X, Out, n, nk, alpha);
  return hipGetLastError();
}

// Eq. tilde_Phi_GW: one wave per matrix; lanes stride over the diagonal,
// a butterfly reduction sums the wave, lane 0 writes the weighted term of
// its matrix.  The terms are then summed by sum_k in a fixed order, so the
// result does not depend on the order in which the waves finish.
__global__ void __launch_bounds__(64) phi_terms_k(const double2* LU, const double2* P0, int n,
                                                  const double* wts, int nw, double* part) {
  const size_t m = blockIdx.x;
  const size_t nn = (size_t)n * (size_t)n;
  const double2* A = LU + m * nn;
  const double2* P = P0 + m * nn;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) {
    const double2 u = A[(size_t)i * n + i];
    s += log(hypot(u.x, u.y)) + P[(size_t)i * n + i].x;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) part[m] = wts[m % (size_t)nw] * s;
}

hipError_t phi_terms_launch(const double2* LU, const double2* P0, int n, long long nmat,
                            const double* wts, int nw, double* part, double* out, hipStream_t st) {
  if (n <= 0 || nmat <= 0) return hipSuccess;
  if (nw <= 0 || nmat > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  phi_terms_k<<<dim3((unsigned)nmat, 1, 1), 64, 0, st>>>(LU, P0, n, wts, nw, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return sum_launch(part, nmat, 1.0, out, st);
}

hipError_t herm_fill_launch(double2* P, int n, long long nmat, hipStream_t st) {
  if (n <= 0 || nmat <= 0) return hipSuccess;
  if (nmat > 65535 || (long long)n * n > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  const unsigned bx = (unsigned)(((long long)n * n + 255) / 256);
  herm_fill_k<<<dim3(bx, (unsigned)nmat, 1), 256, 0, st>>>(P, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One workgroup per (n, k): in-place Gauss-Jordan inversion with row pivoting
// of M = (i w_n + mu) S - H0 - Sig_inf - Sig_iw in LDS.  When G is non-null the
// inverse is written out; when part is non-null, part[n*nk+k] receives
// Re(r_n tr[G S]) for the electron count.
__global__ void __launch_bounds__(256) dyson_k(DysonArgs a) {
  extern __shared__ double2 sm[];
  const int n = a.nao;
  const int k = blockIdx.x % a.nk, iw = blockIdx.x / a.nk;
  double2* M = sm;                          // n x n
  double2* fcol = sm + n * n;               // n
  int* perm = (int*)(fcol + n);             // n
  __shared__ double pv[256];
  __shared__ int pi_[256];
  __shared__ double2 pinv_s;
  __shared__ int piv_s;
  double lsum = 0.0;                        // thread 0: sum of ln|pivot|
  const int tid = threadIdx.x, nt = blockDim.x;
  const size_t nn = (size_t)n * n;
  const double w = a.wF[iw];
  for (int e = tid; e < (int)nn; e += nt) {
    const int r = e / n, c = e % n;
    const double2 s = a.S[k * nn + e];
    const double2 h = a.H0[k * nn + e];
    double2 v;
    v.x = a.mu * s.x - w * s.y - h.x;
    v.y = a.mu * s.y + w * s.x - h.y;
    if (a.Sinf) { v.x -= a.Sinf[k * nn + e].x; v.y -= a.Sinf[k * nn + e].y; }
    if (a.Siw) {
      const double2 q = a.Siw[((size_t)iw * a.nk + k) * nn + e];
      v.x -= q.x;
      v.y -= q.y;
    }
    M[e] = v;
    (void)r; (void)c;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double best = -1.0;
    int bi = j;
    for (int r = j + tid; r < n; r += nt) {
      const double2 x = M[r * n + j];
      const double v = fabs(x.x) + fabs(x.y);
      if (v > best) { best = v; bi = r; }
    }
    pv[tid] = best;
    pi_[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) {
        if (pv[tid + s] > pv[tid] || (pv[tid + s] == pv[tid] && pi_[tid + s] < pi_[tid])) {
          pv[tid] = pv[tid + s];
          pi_[tid] = pi_[tid + s];
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      piv_s = pi_[0];
      perm[j] = pi_[0];
      if (!(pv[0] > 0.0)) atomicOr(a.flag, 1);
    }
    __syncthreads();
    const int p = piv_s;
    if (p != j)
      for (int c = tid; c < n; c += nt) {
        const double2 t = M[j * n + c];
        M[j * n + c] = M[p * n + c];
        M[p * n + c] = t;
      }
    __syncthreads();
    if (tid == 0) {
      const double2 x = M[j * n + j];
      const double den = x.x * x.x + x.y * x.y;
      pinv_s = den > 0.0 ? double2{x.x / den, -x.y / den} : double2{0.0, 0.0};
      lsum += 0.5 * log(den);
    }
    __syncthreads();
    const double2 q = pinv_s;
    for (int c = tid; c < n; c += nt) {
      const double2 x = (c == j) ? double2{1.0, 0.0} : M[j * n + c];
      M[j * n + c] = double2{x.x * q.x - x.y * q.y, x.x * q.y + x.y * q.x};
    }
    for (int r = tid; r < n; r += nt) fcol[r] = M[r * n + j];
    __syncthreads();
    for (int e = tid; e < (int)nn; e += nt) {
      const int r = e / n, c = e % n;
      if (r == j) continue;
      const double2 f = fcol[r];
      const double2 u = M[j * n + c];
      double2 x = (c == j) ? double2{0.0, 0.0} : M[e];
      x.x -= f.x * u.x - f.y * u.y;
      x.y -= f.x * u.y + f.y * u.x;
      M[e] = x;
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges of the inverse
  for (int j = n - 1; j >= 0; --j) {
    const int p = perm[j];
    if (p != j)
      for (int r = tid; r < n; r += nt) {
        const double2 t = M[r * n + j];
        M[r * n + j] = M[r * n + p];
        M[r * n + p] = t;
      }
    __syncthreads();
  }
  if (a.logdet && tid == 0) a.logdet[(size_t)iw * a.nk + k] = lsum;
  if (a.G) {
    double2* g = a.G + ((size_t)iw * a.nk + k) * nn;
    for (int e = tid; e < (int)nn; e += nt) g[e] = M[e];
  }
  if (a.part) {
    // tr[G S] = sum_{ij} G_ij S_ji
    double tr_r = 0.0, tr_i = 0.0;
    for (int e = tid; e < (int)nn; e += nt) {
      const int r = e / n, c = e % n;
      const double2 g = M[e];
      const double2 s = a.S[k * nn + (size_t)c * n + r];
      tr_r += g.x * s.x - g.y * s.y;
      tr_i += g.x * s.y + g.y * s.x;
    }
    pv[tid] = tr_r;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) pv[tid] += pv[tid + s];
      __syncthreads();
    }
    const double sr = pv[0];
    __syncthreads();
    pv[tid] = tr_i;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) pv[tid] += pv[tid + s];
      __syncthreads();
    }
    if (tid == 0) {
      const double2 rr = a.rrow[iw];
      a.part[(size_t)iw * a.nk + k] = rr.x * sr - rr.y * pv[0];
    }
  }
}

hipError_t dyson_launch(const DysonArgs& a, int nw, hipStream_t st) {
  if (nw <= 0 || a.nk <= 0) return hipSuccess;
  const size_t shm = (size_t)a.nao * a.nao * sizeof(double2) + (size_t)a.nao * sizeof(double2) +
                     (size_t)a.nao * sizeof(int);
  dyson_k<<<(unsigned)(nw * a.nk), 256, shm, st>>>(a);
  return hipGetLastError();
}

// Sum of x[0..n) in a fixed order (one workgroup), out[0] = scale * sum.
__global__ void __launch_bounds__(256) sum_k(const double* x, long long n, double scale,
                                              double* out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) acc += x[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = scale * s[0];
}

hipError_t sum_launch(const double* x, long long n, double scale, double* out, hipStream_t st) {
  sum_k<<<1, 256, 0, st>>>(x, n, scale, out);
  return hipGetLastError();
}

// part[k] = Re tr[gamma^k S^k]
__global__ void __launch_bounds__(64) trace_k(const double2* g, const double2* S, int n,
                                             double* part) {
  const int k = blockIdx.x;
  const size_t nn = (size_t)n * n;
  double acc = 0.0;
  for (int e = threadIdx.x; e < (int)nn; e += 64) {
    const int r = e / n, c = e % n;
    const double2 x = g[k * nn + e];
    const double2 s = S[k * nn + (size_t)c * n + r];
    acc += x.x * s.x - x.y * s.y;
  }
  __shared__ double sh[64];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[k] = sh[0];
}

hipError_t trace_launch(const double2* g, const double2* S, int n, int nk, double* part,
                        hipStream_t st) {
  trace_k<<<nk, 64, 0, st>>>(g, S, n, part);
  return hipGetLastError();
}

// max that propagates NaN: fmax drops a NaN operand, which would let a
// corrupted vector report a finite (even zero) largest difference.
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

// Y = (1 - alpha) Y + alpha X (X may be null); per-block max |X - Y_old| into part
// (NaN if any difference is NaN, e.g. a NaN element or Inf - Inf).
__global__ void __launch_bounds__(256) mix_k(long long n, double alpha, const double2* X, double2* Y,
                                              double* part) {
  __shared__ double s[256];
  double mx = 0.0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
    const double2 x = X ? X[i] : double2{0.0, 0.0};
    double2 y;
    if (alpha == 1.0 && !part) {
      y = double2{0.0, 0.0};
    } else {
      y = Y[i];
      const double dx = x.x - y.x, dy = x.y - y.y;
      mx = nan_max(mx, sqrt(dx * dx + dy * dy));
    }
    Y[i] = double2{y.x + alpha * (x.x - y.x), y.y + alpha * (x.y - y.y)};
  }
  if (!part) return;
  s[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = nan_max(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) max_k(const double* x, int n, double* out) {
  __shared__ double s[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = nan_max(m, x[i]);
  s[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = nan_max(s[threadIdx.x], s[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0];
}

hipError_t mix_launch(long long n, double alpha, const double2* X, double2* Y, double* part,
                      int nblk, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  mix_k<<<nblk, 256, 0, st>>>(n, alpha, X, Y, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !part) return e;
  max_k<<<1, 256, 0, st>>>(part, nblk, part + nblk);
  return hipGetLastError();
}

__global__ void zero_int_k(int* p) { *p = 0; }

hipError_t zero_flag_launch(int* p, hipStream_t st) {
  zero_int_k<<<1, 1, 0, st>>>(p);
  return hipGetLastError();
}

// complex128 -> complex64 (rounding), n elements
__global__ void __launch_bounds__(256) to_c64_k(const double2* x, float2* y, long long n) {
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride)
    y[i] = float2{(float)x[i].x, (float)x[i].y};
}

hipError_t to_c64_launch(const double2* x, float2* y, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 8192);
  to_c64_k<<<(unsigned)blocks, 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}

// Y = a X + b Y (complex a, b); X may be null (Y = b Y); b = 0 does not read Y.
__global__ void __launch_bounds__(256) axpby_k(long long n, double ar, double ai, const double2* X,
                                                double br, double bi, double2* Y) {
  const long long stride = (long long)gridDim.x * 256;
  const bool rb = (br != 0.0 || bi != 0.0);
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
    double2 v{0.0, 0.0};
    if (X) {
      const double2 x = X[i];
      v.x = ar * x.x - ai * x.y;
      v.y = ar * x.y + ai * x.x;
    }
    if (rb) {
      const double2 y = Y[i];
      v.x += br * y.x - bi * y.y;
      v.y += br * y.y + bi * y.x;
    }
    Y[i] = v;
  }
}

hipError_t axpby_launch(long long n, double ar, double ai, const double2* X, double br, double bi,
                        double2* Y, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  axpby_k<<<(unsigned)blocks, 256, 0, st>>>(n, ar, ai, X, br, bi, Y);
  return hipGetLastError();
}

// part[2*b], part[2*b+1] = partial sum over block b of conj(X_i) Y_i
__global__ void __launch_bounds__(256) dot_k(long long n, const double2* X, const double2* Y,
                                             double* part) {
  __shared__ double sr[256], si[256];
  double ar = 0.0, ai = 0.0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += stride) {
    const double2 x = X[i], y = Y[i];
    ar += x.x * y.x + x.y * y.y;
    ai += x.x * y.y - x.y * y.x;
  }
  sr[threadIdx.x] = ar;
  si[threadIdx.x] = ai;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sr[threadIdx.x] += sr[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = si[0];
  }
}

// out[0..1] = sums of the nb interleaved partials, in block order
__global__ void sum2_k(const double* part, int nb, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, b = 0.0;
  for (int i = 0; i < nb; ++i) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  out[0] = a;
  out[1] = b;
}

hipError_t dot_launch(long long n, const double2* X, const double2* Y, double* part, int nblk,
                      double* out, hipStream_t st) {
  dot_k<<<nblk, 256, 0, st>>>(n, X, Y, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  sum2_k<<<1, 64, 0, st>>>(part, nblk, out);
  return hipGetLastError();
}

// part[n*nk + k] = Re(r_n tr[P[n][k] S[k]])
__global__ void __launch_bounds__(64) wtrace_k(const double2* P, const double2* S, const double2* r,
                                               int nao, int nk, double* part, int s_per_w) {
  const int k = blockIdx.x % nk, iw = blockIdx.x / nk;
  const size_t nn = (size_t)nao * nao;
  const double2* p = P + ((size_t)iw * nk + k) * nn;
  if (s_per_w) S += (size_t)iw * nk * nn;
  double tr = 0.0, ti = 0.0;
  for (int e = threadIdx.x; e < (int)nn; e += 64) {
    const int a = e / nao, b = e % nao;
    const double2 x = p[e];
    const double2 s = S[k * nn + (size_t)b * nao + a];
    tr += x.x * s.x - x.y * s.y;
    ti += x.x * s.y + x.y * s.x;
  }
  __shared__ double sr[64], si[64];
  sr[threadIdx.x] = tr;
  si[threadIdx.x] = ti;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sr[threadIdx.x] += sr[threadIdx.x + h];
      si[threadIdx.x] += si[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = r[iw].x * sr[0] - r[iw].y * si[0];
}

hipError_t wtrace_launch(const double2* P, const double2* S, const double2* r, int nao, int nk, int nw,
                         double* part, hipStream_t st, int s_per_w) {
  wtrace_k<<<(unsigned)(nw * nk), 64, 0, st>>>(P, S, r, nao, nk, part, s_per_w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked LU pieces for (I - P0) X = P0 (one workgroup per matrix).
// A = I - P0 and B = P0 are set up by wlu_init_k; for each panel of nb
// columns, wlu_panel_k factors the panel with row pivoting (swapping whole
// rows of A and B), wlu_trsm_lower_k applies the panel's unit-lower block to
// the rows of the panel, and the trailing updates are GEMMs on the host side.
// wlu_trsm_upper_k solves one diagonal block of U during back substitution.
__global__ void __launch_bounds__(256) wlu_init_k(const double2* __restrict__ P0, double2* A,
                                                   double2* B, int n) {
  const size_t nn = (size_t)n * n;
  const double2* P = P0 + blockIdx.x * nn;
  double2* Am = A + blockIdx.x * nn;
  double2* Bm = B + blockIdx.x * nn;
  for (size_t e = threadIdx.x; e < nn; e += 256) {
    const int r = (int)(e / n), c = (int)(e % n);
    const double2 p = P[e];
    Am[e] = double2{(r == c ? 1.0 : 0.0) - p.x, -p.y};
    Bm[e] = p;
  }
}

__global__ void __launch_bounds__(256) wlu_panel_k(double2* A, double2* B, int n, int j0, int nb,
                                                    int* flag) {
  const size_t nn = (size_t)n * n;
  double2* Am = A + blockIdx.x * nn;
  double2* Bm = B + blockIdx.x * nn;
  const int tid = threadIdx.x, nt = 256;
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ double2 pinv_s;
  const int j1 = min(j0 + nb, n);
  for (int j = j0; j < j1; ++j) {
    double best = -1.0;
    int bi = j;
    for (int r = j + tid; r < n; r += nt) {
      const double2 a = Am[(size_t)r * n + j];
      const double v = fabs(a.x) + fabs(a.y);
      if (v > best) { best = v; bi = r; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s) {
        const double o = sv[tid + s];
        const int oi = si[tid + s];
        if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = si[0];
    if (tid == 0 && !(sv[0] > 0.0)) atomicOr(flag, 1);
    if (p != j) {
      for (int c = tid; c < n; c += nt) {
        double2 t = Am[(size_t)j * n + c];
        Am[(size_t)j * n + c] = Am[(size_t)p * n + c];
        Am[(size_t)p * n + c] = t;
        t = Bm[(size_t)j * n + c];
        Bm[(size_t)j * n + c] = Bm[(size_t)p * n + c];
        Bm[(size_t)p * n + c] = t;
      }
    }
    __syncthreads();
    if (tid == 0) {
      const double2 a = Am[(size_t)j * n + j];
      const double den = a.x * a.x + a.y * a.y;
      pinv_s = den > 0.0 ? double2{a.x / den, -a.y / den} : double2{0.0, 0.0};
    }
    __syncthreads();
    const double2 pi = pinv_s;
    for (int r = j + 1 + tid; r < n; r += nt) {
      const double2 a = Am[(size_t)r * n + j];
      Am[(size_t)r * n + j] = double2{a.x * pi.x - a.y * pi.y, a.x * pi.y + a.y * pi.x};
    }
    __syncthreads();
    // rank-1 update of the rest of the panel
    const int w = j1 - j - 1;
    if (w > 0) {
      const size_t cnt = (size_t)(n - j - 1) * w;
      for (size_t e = tid; e < cnt; e += nt) {
        const int r = j + 1 + (int)(e / w), c = j + 1 + (int)(e % w);
        const double2 l = Am[(size_t)r * n + j];
        const double2 u = Am[(size_t)j * n + c];
        double2 a = Am[(size_t)r * n + c];
        a.x -= l.x * u.x - l.y * u.y;
        a.y -= l.x * u.y + l.y * u.x;
        Am[(size_t)r * n + c] = a;
      }
    }
    __syncthreads();
  }
}

// rows j0+1 .. j0+nb-1: U12 and B rows of the panel <- L11^{-1} (unit lower)
__global__ void __launch_bounds__(256) wlu_trsm_lower_k(double2* A, double2* B, int n, int j0, int nb) {
  const size_t nn = (size_t)n * n;
  double2* Am = A + blockIdx.x * nn;
  double2* Bm = B + blockIdx.x * nn;
  const int j1 = min(j0 + nb, n);
  const int ca = n - j1;               // trailing columns of A
  for (int r = j0 + 1; r < j1; ++r) {
    for (int e = threadIdx.x; e < ca + n; e += 256) {
      double2* M = e < ca ? Am : Bm;
      const int c = e < ca ? j1 + e : e - ca;
      double2 x = M[(size_t)r * n + c];
      for (int i = j0; i < r; ++i) {
        const double2 l = Am[(size_t)r * n + i];
        const double2 u = M[(size_t)i * n + c];
        x.x -= l.x * u.x - l.y * u.y;
        x.y -= l.x * u.y + l.y * u.x;
      }
      M[(size_t)r * n + c] = x;
    }
    __syncthreads();
  }
}

// rows j0 .. j1-1 of B <- U11^{-1} B (upper, back substitution within the block)
__global__ void __launch_bounds__(256) wlu_trsm_upper_k(const double2* A, double2* B, int n, int j0,
                                                         int nb) {
  const size_t nn = (size_t)n * n;
  const double2* Am = A + blockIdx.x * nn;
  double2* Bm = B + blockIdx.x * nn;
  const int j1 = min(j0 + nb, n);
  for (int r = j1 - 1; r >= j0; --r) {
    const double2 d = Am[(size_t)r * n + r];
    const double den = d.x * d.x + d.y * d.y;
    const double2 di = den > 0.0 ? double2{d.x / den, -d.y / den} : double2{0.0, 0.0};
    for (int c = threadIdx.x; c < n; c += 256) {
      double2 x = Bm[(size_t)r * n + c];
      for (int i = r + 1; i < j1; ++i) {
        const double2 u = Am[(size_t)r * n + i];
        const double2 y = Bm[(size_t)i * n + c];
        x.x -= u.x * y.x - u.y * y.y;
        x.y -= u.x * y.y + u.y * y.x;
      }
      Bm[(size_t)r * n + c] = double2{x.x * di.x - x.y * di.y, x.x * di.y + x.y * di.x};
    }
    __syncthreads();
  }
}

hipError_t wlu_launch(int which, const double2* P0, double2* A, double2* B, int n, int j0, int nb,
                      long long nmat, int* flag, hipStream_t st) {
  if (nmat <= 0) return hipSuccess;
  const unsigned g = (unsigned)nmat;
  switch (which) {
    case 0: wlu_init_k<<<g, 256, 0, st>>>(P0, A, B, n); break;
    case 1: wlu_panel_k<<<g, 256, 0, st>>>(A, B, n, j0, nb, flag); break;
    case 2: wlu_trsm_lower_k<<<g, 256, 0, st>>>(A, B, n, j0, nb); break;
    case 3: wlu_trsm_upper_k<<<g, 256, 0, st>>>(A, B, n, j0, nb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
