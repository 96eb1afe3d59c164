// C ABI of the density-fitted GW hot path: context, argument checks, and the
// mapping of every equation onto the device kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/gw.h"
#include "grids.h"
#include "gw_kernels.h"
#include "ir.h"

// Fixed scratch for gw_polarization_noalloc: a file-scope device array, one
// copy per GPU for the life of the process.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress and kept in g_scratch_dev.
static const size_t kScratchBytes = size_t(128) << 20;   // 128 MiB
static __device__ __align__(256) char scratch[kScratchBytes];
static const int kMaxDevices = 64;
static char* g_scratch_dev[kMaxDevices] = {};
static std::mutex g_scratch_mu;

struct gw_ctx {
  gw_dims d;
  int nk = 0;
  long long n2 = 0;      // nao^2
  long long sv = 0;      // complex elements of one V^{k,k+q} block: naux * nao^2
  hipStream_t st = nullptr;
  int device = 0;
  char* scratch = nullptr;   // this device's copy of the fixed scratch array (see below)
  bool grids = false;
  std::vector<double> tau, x, w;
  std::vector<long long> nF, nB;
  std::vector<gwgrid::cd> TF, TFp, TB, TBp, rrow;
  std::vector<int> plus;   // host copy of the k+q table
  bool check_bounds = false;
  int tile_cfg = -1;       // tile configuration of the large contractions (-1: default)
  int prod_tiles = 0;      // 1: fp32 producers on the tiled GEMM instead of the streaming kernel
  int split_cfg = -1;      // tile configuration of the split-bf16 contractions
  int split_group = 0;     // > 0: grouped workgroup order of the split contractions
  int herm = 0;            // gw_set_hermitian: GW_HERM_* bits
  double mu_window = 0.0;  // gw_set_mu_window: electron-count window (0: exact root)
  // measurement: event pairs per kernel class while profiling is on
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[KC_COUNT];
  long long launches[KC_COUNT] = {};
  double flops[KC_COUNT] = {};
  double ms[KC_COUNT] = {};
  double2 *dTF = nullptr, *dTFp = nullptr, *dTB = nullptr, *dTBp = nullptr;
  double2 *dw = nullptr, *drrow = nullptr;
  double* dwF = nullptr;
  int *dplus = nullptr, *dminus = nullptr;
  int* dflag = nullptr;
  double* dpart = nullptr;   // nw_f * nk partials, then the reduced scalar at [nw_f*nk]
  double* dred = nullptr;    // 2 * 1024 partials + 2 results for gw_dot
  double* dphi = nullptr;    // Nk * nw_b per-matrix terms of Phi~, then their sum
  void* ws = nullptr;
  size_t ws_bytes = 0;
  int tc = 0;
  std::string err;
};

namespace {

gw_status fail(gw_ctx* c, gw_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, GW_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int mesh_index(const int* mesh, int a, int b, int c) {
  a = ((a % mesh[0]) + mesh[0]) % mesh[0];
  b = ((b % mesh[1]) + mesh[1]) % mesh[1];
  c = ((c % mesh[2]) + mesh[2]) % mesh[2];
  return (a * mesh[1] + b) * mesh[2] + c;
}

gw_status check_dims(const gw_dims* d, std::string& why) {
  if (!d) { why = "dims is NULL"; return GW_ERR_ARG; }
  for (int i = 0; i < 3; ++i)
    if (d->mesh[i] < 1 || d->mesh[i] > 64) { why = "mesh entries must be in 1..64"; return GW_ERR_ARG; }
  if (d->nao < 1 || d->nao > 60) { why = "nao must be in 1..60"; return GW_ERR_ARG; }
  if (d->naux < 1 || d->naux > 8192) { why = "naux must be in 1..8192"; return GW_ERR_ARG; }
  if (d->ntau < 2 || d->ntau > 512 || d->ntau % 2) { why = "ntau must be even, 2..512"; return GW_ERR_ARG; }
  if (d->nw_f < d->ntau || d->nw_f > 4 * d->ntau) { why = "nw_f must lie in ntau..4 ntau"; return GW_ERR_ARG; }
  if (d->nw_b < d->ntau || d->nw_b > 4 * d->ntau + 1) {
    why = "nw_b must lie in ntau..4 ntau + 1";
    return GW_ERR_ARG;
  }
  if (d->ns != 1 && d->ns != 2) { why = "ns must be 1 or 2"; return GW_ERR_ARG; }
  if (!(d->beta > 0.0) || !std::isfinite(d->beta)) { why = "beta must be positive"; return GW_ERR_ARG; }
  if (d->precision < GW_PREC_FP64 || d->precision > GW_PREC_BF16X6) {
    why = "unsupported precision";
    return GW_ERR_ARG;
  }
  const long long nk = (long long)d->mesh[0] * d->mesh[1] * d->mesh[2];
  if (nk * d->nao * (long long)d->nao * d->naux > (1LL << 31)) {
    why = "Nk * naux * nao^2 must stay below 2^31";
    return GW_ERR_ARG;
  }
  return GW_OK;
}

bool ready(gw_ctx* c) { return c && c->grids; }

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

template <class T>
gw_status upload(gw_ctx* c, T** dst, const void* src, size_t bytes) {
  HIPCHK(c, hipMalloc((void**)dst, bytes));
  HIPCHK(c, hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return GW_OK;
}

// Exact [min, max] of a mapped index over i in [0, n).
void map_range(const Map3& m, long long n, long long& lo, long long& hi) {
  lo = hi = 0;
  for (long long i = 0; i < n; ++i) {
    const unsigned a = (unsigned)(i % m.din);
    const unsigned r = (unsigned)(i / m.din);
    const long long o = (long long)(r / m.dmid) * m.sout + (long long)(r % m.dmid) * m.smid +
                        (long long)a * m.sin;
    if (i == 0 || o < lo) lo = (i == 0) ? o : std::min(lo, o);
    if (i == 0 || o > hi) hi = (i == 0) ? o : std::max(hi, o);
  }
}

// Host-side proof that a GEMM descriptor stays inside its operands: every
// touched offset of A, B and C lies in [0, ext).  Enabled by GW_DEBUG_BOUNDS.
struct Ext {
  long long lo, hi;   // valid element offsets [lo, hi) relative to the operand pointer
};

bool gemm_in_bounds(gw_ctx* c, const GemmDesc& g, Ext eA, Ext eB, Ext eC, std::string& why) {
  long long bl[3] = {0, 0, 0}, bh[3] = {0, 0, 0};
  const Map3* bm[3] = {&g.ba, &g.bb, &g.bc};
  const long long ts[3] = {g.tsA, g.tsB, g.tsC};
  for (int o = 0; o < 3; ++o)
    for (long long b = 0; b < g.batch; ++b) {
      const unsigned a = (unsigned)(b % bm[o]->din);
      const unsigned r = (unsigned)(b / bm[o]->din);
      long long off = (long long)(r / bm[o]->dmid) * bm[o]->sout +
                      (long long)(r % bm[o]->dmid) * bm[o]->smid + (long long)a * bm[o]->sin;
      if (ts[o] != 0) {
        const int tq = (int)(g.tab - c->dplus);          // tables are rows of the k+q table
        off += (long long)c->plus[(size_t)tq + (size_t)(b % g.tmod)] * ts[o];
      }
      if (b == 0 || off < bl[o]) bl[o] = (b == 0) ? off : std::min(bl[o], off);
      if (b == 0 || off > bh[o]) bh[o] = (b == 0) ? off : std::max(bh[o], off);
    }
  long long l1, h1, l2, h2;
  map_range(g.am, g.M, l1, h1);
  map_range(g.ak, g.K, l2, h2);
  if (bl[0] + l1 + l2 < eA.lo || bh[0] + h1 + h2 >= eA.hi) {
    why = "A out of bounds: [" + std::to_string(bl[0] + l1 + l2) + ", " + std::to_string(bh[0] + h1 + h2) +
          "] vs [" + std::to_string(eA.lo) + ", " + std::to_string(eA.hi) + ")";
    return false;
  }
  map_range(g.bk, g.K, l1, h1);
  map_range(g.bn, g.N, l2, h2);
  if (bl[1] + l1 + l2 < eB.lo || bh[1] + h1 + h2 >= eB.hi) {
    why = "B out of bounds: [" + std::to_string(bl[1] + l1 + l2) + ", " + std::to_string(bh[1] + h1 + h2) +
          "] vs [" + std::to_string(eB.lo) + ", " + std::to_string(eB.hi) + ")";
    return false;
  }
  map_range(g.cm, g.M, l1, h1);
  map_range(g.cn, g.N, l2, h2);
  if (bl[2] + l1 + l2 < eC.lo || bh[2] + h1 + h2 >= eC.hi) {
    why = "C out of bounds: [" + std::to_string(bl[2] + l1 + l2) + ", " + std::to_string(bh[2] + h1 + h2) +
          "] vs [" + std::to_string(eC.lo) + ", " + std::to_string(eC.hi) + ")";
    return false;
  }
  return true;
}

gw_status prof_begin(gw_ctx* c, int kc, hipEvent_t* e0) {
  if (!c->prof) return GW_OK;
  HIPCHK(c, hipEventCreate(e0));
  HIPCHK(c, hipEventRecord(*e0, c->st));
  (void)kc;
  return GW_OK;
}

gw_status prof_end(gw_ctx* c, int kc, hipEvent_t e0, double flops) {
  if (!c->prof) return GW_OK;
  hipEvent_t e1;
  HIPCHK(c, hipEventCreate(&e1));
  HIPCHK(c, hipEventRecord(e1, c->st));
  c->ev[kc].push_back({e0, e1});
  c->launches[kc] += 1;
  c->flops[kc] += flops;
  return GW_OK;
}

gw_status run(gw_ctx* c, const GemmDesc& g, Ext eA, Ext eB, Ext eC) {
  if (c->check_bounds) {
    std::string why;
    if (!gemm_in_bounds(c, g, eA, eB, eC, why))
      return fail(c, GW_ERR_ARG, "internal descriptor check: " + why);
  }
  hipEvent_t e0 = nullptr;
  gw_status s = prof_begin(c, g.tag, &e0);
  if (s != GW_OK) return s;
  GemmDesc gg = g;
  // tile shapes measured best on MI355X at naux = 250: 64x64 for the
  // polarization contraction, 64x96 on the three-product (Gauss) form for
  // the self-energy one
  if (g.tag == KC_POL_PRODUCER || g.tag == KC_SE_PRODUCER) gg.cfg = c->prod_tiles;
  else gg.cfg = c->tile_cfg >= 0 ? c->tile_cfg : (g.tag == KC_SE_CONTRACT ? 7 : 0);
  hipError_t e = zgemm_launch(gg, c->st);
  if (e != hipSuccess) return fail(c, GW_ERR_DEVICE, std::string("zgemm: ") + hipGetErrorString(e));
  // MFMA flops executed: 8 real flops per complex multiply-add, 6 on the
  // three-product form; with g.tri only the entries on and above the diagonal
  const double outs = g.tri ? 0.5 * g.M * (g.M + 1.0) : (double)g.M * g.N;
  const double per = zgemm_three_product(gg) ? 6.0 : 8.0;
  return prof_end(c, g.tag, e0, per * outs * g.K * g.batch);
}

// Split-bf16 contraction: eA, eB, eC the valid element ranges of the
// operands; k_true the K that the algorithmic flops count.
gw_status run_split(gw_ctx* c, const SplitDesc& d, Ext eA, Ext eB, Ext eC) {
  if (c->check_bounds) {
    auto span = [&](const Map3& bm, const Map3& rm, int rows, long long ks, long long& lo, long long& hi) {
      long long l1, h1, l2, h2;
      map_range(bm, d.batch, l1, h1);
      map_range(rm, rows, l2, h2);
      lo = l1 + l2 + std::min(0LL, (long long)(d.K - 1) * ks);
      hi = h1 + h2 + std::max(0LL, (long long)(d.K - 1) * ks);
    };
    long long la, ha, lb, hb, lc, hc, l1, h1;
    span(d.ba, d.am, d.M, d.aks, la, ha);
    span(d.bb, d.bn, d.N, d.bks, lb, hb);
    span(d.bc, d.cm, d.M, 0, lc, hc);
    map_range(d.cn, d.N, l1, h1);
    lc += l1;
    hc += h1;
    if (la < eA.lo || ha >= eA.hi || lb < eB.lo || hb >= eB.hi || lc < eC.lo || hc >= eC.hi)
      return fail(c, GW_ERR_ARG, "internal descriptor check: split contraction out of bounds");
  }
  hipEvent_t e0 = nullptr;
  gw_status s = prof_begin(c, d.tag, &e0);
  if (s != GW_OK) return s;
  SplitDesc dd = d;
  dd.cfg = c->split_cfg;
  if (c->split_group > 0) {
    dd.batch_fastest = 2;
    dd.group = c->split_group;
  }
  hipError_t e = bsgemm_launch(dd, c->st);
  if (e != hipSuccess) return fail(c, GW_ERR_DEVICE, std::string("bsgemm: ") + hipGetErrorString(e));
  const double outs = d.tri ? 0.5 * d.M * (d.M + 1.0) : (double)d.M * d.N;
  return prof_end(c, d.tag, e0, 8.0 * outs * d.K * d.batch);
}

gw_status read_flag(gw_ctx* c, const char* what) {
  int f = 0;
  HIPCHK(c, hipMemcpyAsync(&f, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (f) return fail(c, GW_ERR_SINGULAR, std::string(what) + ": zero pivot");
  return GW_OK;
}

// Electron count of G at mu (no G written unless Gout is given).
gw_status count_at(gw_ctx* c, const gw_z* H0, const gw_z* S, const gw_z* Sinf, const gw_z* Siw,
                   double mu, gw_z* Gout, double* ne) {
  DysonArgs a{};
  a.H0 = (const double2*)H0;
  a.S = (const double2*)S;
  a.Sinf = (const double2*)Sinf;
  a.Siw = (const double2*)Siw;
  a.wF = c->dwF;
  a.rrow = c->drrow;
  a.mu = mu;
  a.nk = c->nk;
  a.nao = c->d.nao;
  a.G = (double2*)Gout;
  a.part = c->dpart;
  a.flag = c->dflag;
  HIPCHK(c, dyson_launch(a, c->d.nw_f, c->st));
  const long long np = (long long)c->d.nw_f * c->nk;
  HIPCHK(c, sum_launch(c->dpart, np, -(double)c->d.ns / c->nk, c->dpart + np, c->st));
  HIPCHK(c, hipMemcpyAsync(ne, c->dpart + np, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (!std::isfinite(*ne)) return fail(c, GW_ERR_NONFINITE, "electron count is not finite");
  return GW_OK;
}

}  // namespace

extern "C" {

const char* gw_status_string(gw_status s) {
  switch (s) {
    case GW_OK: return "ok";
    case GW_ERR_ARG: return "invalid argument";
    case GW_ERR_DEVICE: return "HIP runtime error";
    case GW_ERR_SINGULAR: return "singular matrix";
    case GW_ERR_NOCONV: return "no convergence";
    case GW_ERR_WORKSPACE: return "workspace missing or too small";
    case GW_ERR_STATE: return "grids not built";
    case GW_ERR_NONFINITE: return "non-finite value";
  }
  return "unknown status";
}

const char* gw_last_error(const gw_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

gw_status gw_create(const gw_dims* d, void* hip_stream, gw_ctx** out) {
  if (!out) return GW_ERR_ARG;
  *out = nullptr;
  std::string why;
  if (check_dims(d, why) != GW_OK) return GW_ERR_ARG;
  gw_ctx* c = new (std::nothrow) gw_ctx();
  if (!c) return GW_ERR_DEVICE;
  c->d = *d;
  c->nk = d->mesh[0] * d->mesh[1] * d->mesh[2];
  c->n2 = (long long)d->nao * d->nao;
  c->sv = (long long)d->naux * c->n2;
  c->st = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return GW_ERR_DEVICE; }
  if (c->device < 0 || c->device >= kMaxDevices) { delete c; return GW_ERR_DEVICE; }
  {
    // once per device, with that device current: the device address of its scratch copy
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[c->device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) { delete c; return GW_ERR_DEVICE; }
      g_scratch_dev[c->device] = (char*)p;
    }
    c->scratch = g_scratch_dev[c->device];
  }
  std::vector<int> plus((size_t)c->nk * c->nk), minus((size_t)c->nk * c->nk);
  const int* m = d->mesh;
  for (int q = 0; q < c->nk; ++q)
    for (int k = 0; k < c->nk; ++k) {
      const int qa = q / (m[1] * m[2]), qb = (q / m[2]) % m[1], qc = q % m[2];
      const int ka = k / (m[1] * m[2]), kb = (k / m[2]) % m[1], kc = k % m[2];
      plus[(size_t)q * c->nk + k] = mesh_index(m, ka + qa, kb + qb, kc + qc);
      minus[(size_t)q * c->nk + k] = mesh_index(m, ka - qa, kb - qb, kc - qc);
    }
  c->plus = plus;
  {
    const char* e = std::getenv("GW_DEBUG_BOUNDS");
    c->check_bounds = e && e[0] == '1';
    const char* t = std::getenv("GW_TILE_CFG");
    c->tile_cfg = t ? std::atoi(t) : -1;
    const char* pt = std::getenv("GW_PROD_TILES");
    c->prod_tiles = pt && pt[0] == '1' ? 1 : 0;
    const char* u = std::getenv("GW_SPLIT_CFG");
    c->split_cfg = u ? std::atoi(u) : -1;
    const char* gg = std::getenv("GW_SPLIT_GROUP");
    c->split_group = gg ? std::atoi(gg) : 0;
  }
  if (upload(c, &c->dplus, plus.data(), plus.size() * sizeof(int)) != GW_OK ||
      upload(c, &c->dminus, minus.data(), minus.size() * sizeof(int)) != GW_OK ||
      hipMalloc((void**)&c->dflag, sizeof(int)) != hipSuccess ||
      hipMemset(c->dflag, 0, sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&c->dpart, ((size_t)d->nw_f * c->nk + 8) * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&c->dred, (2 * 1024 + 8) * sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&c->dphi, ((size_t)d->nw_b * c->nk + 8) * sizeof(double)) != hipSuccess) {
    gw_destroy(c);
    return GW_ERR_DEVICE;
  }
  *out = c;
  return GW_OK;
}

gw_status gw_destroy(gw_ctx* c) {
  if (!c) return GW_ERR_ARG;
  for (int k = 0; k < KC_COUNT; ++k)
    for (auto& p : c->ev[k]) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
  void* ptrs[] = {c->dTF, c->dTFp, c->dTB, c->dTBp, c->dw, c->drrow, c->dwF,
                  c->dplus, c->dminus, c->dflag, c->dpart, c->dred, c->dphi};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete c;
  return GW_OK;
}

struct HostGrids {
  std::vector<double> tau, x, w;
  std::vector<long long> nF, nB;
  std::vector<gwgrid::cd> TF, TFp, TB, TBp, rrow;
  std::vector<double> wf;
};

// Derived tables: fermionic frequencies and the electron-count row r = w TFp.
static void finish_grids(double beta, HostGrids& g) {
  const int nt = (int)g.tau.size(), nwf = (int)g.nF.size();
  g.wf.assign(nwf, 0.0);
  for (int n = 0; n < nwf; ++n) g.wf[n] = gwgrid::matsubara(g.nF[n], beta, 0);
  g.rrow.assign(nwf, 0.0);
  for (int n = 0; n < nwf; ++n) {
    gwgrid::cd s = 0.0;
    for (int i = 0; i < nt; ++i) s += g.w[i] * g.TFp[(size_t)i * nwf + n];
    g.rrow[n] = s;
  }
}

static gw_status make_grids(double beta, int nt, const long long* nF, const long long* nB,
                            HostGrids& g, std::string& why) {
  if (!(beta > 0.0) || !std::isfinite(beta) || nt < 2 || nt > 512 || nt % 2) {
    why = "beta must be positive and ntau even in 2..512";
    return GW_ERR_ARG;
  }
  const int nwf = nt, nwb = nt + 1;
  try {
    g.tau.assign(nt, 0.0);
    g.x.assign(nt, 0.0);
    gwgrid::tau_nodes(beta, nt, g.tau.data(), g.x.data());
    if (nF) g.nF.assign(nF, nF + nwf); else g.nF = gwgrid::select_sparse(beta, nt, 0);
    if (nB) g.nB.assign(nB, nB + nwb); else g.nB = gwgrid::select_sparse(beta, nt, 1);
    for (size_t i = 1; i < g.nF.size(); ++i)
      if (g.nF[i] <= g.nF[i - 1]) { why = "nF must be strictly increasing"; return GW_ERR_ARG; }
    for (size_t i = 1; i < g.nB.size(); ++i)
      if (g.nB[i] <= g.nB[i - 1]) { why = "nB must be strictly increasing"; return GW_ERR_ARG; }
    std::vector<double> wf(nwf), wb(nwb);
    for (int n = 0; n < nwf; ++n) wf[n] = gwgrid::matsubara(g.nF[n], beta, 0);
    for (int n = 0; n < nwb; ++n) wb[n] = gwgrid::matsubara(g.nB[n], beta, 1);
    g.TF.assign((size_t)nwf * nt, 0.0);
    g.TB.assign((size_t)nwb * nt, 0.0);
    g.TFp.assign((size_t)nt * nwf, 0.0);
    g.TBp.assign((size_t)nt * nwb, 0.0);
    gwgrid::transform(beta, nt, g.x.data(), wf.data(), nwf, g.TF.data());
    gwgrid::transform(beta, nt, g.x.data(), wb.data(), nwb, g.TB.data());
    if (gwgrid::pinv_qr(g.TF.data(), nwf, nt, g.TFp.data()) ||
        gwgrid::pinv_qr(g.TB.data(), nwb, nt, g.TBp.data())) {
      why = "transform matrix is rank deficient for these frequencies";
      return GW_ERR_ARG;
    }
    g.w.assign(nt, 0.0);
    gwgrid::beta_row(nt, g.x.data(), g.w.data());
    finish_grids(beta, g);
  } catch (const std::exception& e) {
    why = e.what();
    return GW_ERR_ARG;
  }
  return GW_OK;
}

gw_status gw_grids_host(double beta, int ntau, const long long* nF, const long long* nB,
                        double* tau, long long* nF_out, long long* nB_out, gw_z* TF, gw_z* TFp,
                        gw_z* TB, gw_z* TBp, double* w) {
  HostGrids g;
  std::string why;
  gw_status s = make_grids(beta, ntau, nF, nB, g, why);
  if (s != GW_OK) return s;
  if (tau) std::memcpy(tau, g.tau.data(), g.tau.size() * 8);
  if (nF_out) std::memcpy(nF_out, g.nF.data(), g.nF.size() * 8);
  if (nB_out) std::memcpy(nB_out, g.nB.data(), g.nB.size() * 8);
  if (TF) std::memcpy(TF, g.TF.data(), g.TF.size() * 16);
  if (TFp) std::memcpy(TFp, g.TFp.data(), g.TFp.size() * 16);
  if (TB) std::memcpy(TB, g.TB.data(), g.TB.size() * 16);
  if (TBp) std::memcpy(TBp, g.TBp.data(), g.TBp.size() * 16);
  if (w) std::memcpy(w, g.w.data(), g.w.size() * 8);
  return GW_OK;
}

// Keep the host tables in the context and upload the device copies.
static gw_status install_grids(gw_ctx* c, HostGrids& g) {
  c->tau = g.tau; c->x = g.x; c->w = g.w; c->nF = g.nF; c->nB = g.nB;
  c->TF = g.TF; c->TFp = g.TFp; c->TB = g.TB; c->TBp = g.TBp; c->rrow = g.rrow;
  std::vector<gwgrid::cd> wz(c->w.begin(), c->w.end());
  void* olds[] = {c->dTF, c->dTFp, c->dTB, c->dTBp, c->dw, c->drrow, c->dwF};
  for (void* p : olds)
    if (p) (void)hipFree(p);
  c->dTF = c->dTFp = c->dTB = c->dTBp = c->dw = c->drrow = nullptr;
  c->dwF = nullptr;
  c->grids = false;
  gw_status s;
  if ((s = upload(c, &c->dTF, c->TF.data(), c->TF.size() * 16)) != GW_OK) return s;
  if ((s = upload(c, &c->dTFp, c->TFp.data(), c->TFp.size() * 16)) != GW_OK) return s;
  if ((s = upload(c, &c->dTB, c->TB.data(), c->TB.size() * 16)) != GW_OK) return s;
  if ((s = upload(c, &c->dTBp, c->TBp.data(), c->TBp.size() * 16)) != GW_OK) return s;
  if ((s = upload(c, &c->dw, wz.data(), wz.size() * 16)) != GW_OK) return s;
  if ((s = upload(c, &c->drrow, c->rrow.data(), c->rrow.size() * 16)) != GW_OK) return s;
  if ((s = upload(c, &c->dwF, g.wf.data(), g.wf.size() * 8)) != GW_OK) return s;
  c->grids = true;
  return GW_OK;
}

gw_status gw_build_grids(gw_ctx* c, const long long* nF, const long long* nB) {
  if (!c) return GW_ERR_ARG;
  if (c->d.nw_f != c->d.ntau || c->d.nw_b != c->d.ntau + 1)
    return fail(c, GW_ERR_ARG, "gw_build_grids needs nw_f = ntau and nw_b = ntau + 1");
  HostGrids g;
  std::string why;
  gw_status s = make_grids(c->d.beta, c->d.ntau, nF, nB, g, why);
  if (s != GW_OK) return fail(c, s, why);
  return install_grids(c, g);
}

gw_status gw_set_grids(gw_ctx* c, const double* tau, const long long* nF, const long long* nB,
                       const gw_z* TF, const gw_z* TFp, const gw_z* TB, const gw_z* TBp,
                       const double* w) {
  if (!c) return GW_ERR_ARG;
  if (!tau || !nF || !nB || !TF || !TFp || !TB || !TBp || !w) return fail(c, GW_ERR_ARG, "NULL table");
  const int nt = c->d.ntau, nwf = c->d.nw_f, nwb = c->d.nw_b;
  const double beta = c->d.beta;
  for (int i = 0; i < nt; ++i) {
    if (!std::isfinite(tau[i]) || !(tau[i] > 0.0) || !(tau[i] < beta))
      return fail(c, GW_ERR_ARG, "tau nodes must lie in (0, beta)");
    if (i > 0 && !(tau[i] > tau[i - 1])) return fail(c, GW_ERR_ARG, "tau nodes must increase");
    if (std::fabs(tau[nt - 1 - i] - (beta - tau[i])) > 1e-12 * beta)
      return fail(c, GW_ERR_ARG, "tau nodes must be mirrored: tau[ntau-1-i] = beta - tau[i]");
    if (!std::isfinite(w[i])) return fail(c, GW_ERR_ARG, "density row is not finite");
  }
  for (int n = 1; n < nwf; ++n)
    if (nF[n] <= nF[n - 1]) return fail(c, GW_ERR_ARG, "nF must be strictly increasing");
  for (int n = 1; n < nwb; ++n)
    if (nB[n] <= nB[n - 1]) return fail(c, GW_ERR_ARG, "nB must be strictly increasing");
  auto finite = [](const gw_z* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(a[i].re) || !std::isfinite(a[i].im)) return false;
    return true;
  };
  const size_t nfT = (size_t)nwf * nt, nbT = (size_t)nwb * nt;
  if (!finite(TF, nfT) || !finite(TFp, nfT) || !finite(TB, nbT) || !finite(TBp, nbT))
    return fail(c, GW_ERR_ARG, "transform table is not finite");
  HostGrids g;
  try {
    g.tau.assign(tau, tau + nt);
    g.x.resize(nt);
    for (int i = 0; i < nt; ++i) g.x[i] = 2.0 * tau[i] / beta - 1.0;
    g.w.assign(w, w + nt);
    g.nF.assign(nF, nF + nwf);
    g.nB.assign(nB, nB + nwb);
    auto cz = [](const gw_z* a, size_t n) {
      std::vector<gwgrid::cd> v(n);
      for (size_t i = 0; i < n; ++i) v[i] = gwgrid::cd(a[i].re, a[i].im);
      return v;
    };
    g.TF = cz(TF, nfT); g.TFp = cz(TFp, nfT); g.TB = cz(TB, nbT); g.TBp = cz(TBp, nbT);
    finish_grids(beta, g);
  } catch (const std::exception& e) {
    return fail(c, GW_ERR_ARG, e.what());
  }
  return install_grids(c, g);
}

// ------------------------------------------------ IR grids (Sec. IV.C) ---
static gw_status check_ir(double lambda, double eps) {
  if (!(lambda >= 1.0 && lambda <= 1e5) || !(eps >= 1e-14 && eps <= 1e-2)) return GW_ERR_ARG;
  return GW_OK;
}

gw_status gw_ir_size(double lambda, double eps, int* ntau) {
  if (!ntau || check_ir(lambda, eps) != GW_OK) return GW_ERR_ARG;
  try {
    *ntau = gwir::ir_size(lambda, eps);
  } catch (const std::exception&) {
    return GW_ERR_ARG;
  }
  return GW_OK;
}

static gw_status make_ir(double beta, double lambda, double eps, int ntau, HostGrids& g, std::string& why) {
  if (!(beta > 0.0) || !std::isfinite(beta) || check_ir(lambda, eps) != GW_OK) {
    why = "beta must be positive, lambda in 1..1e5 and eps in 1e-14..1e-2";
    return GW_ERR_ARG;
  }
  try {
    gwir::IRTables t;
    if (gwir::ir_size(lambda, eps) != ntau) {
      why = "ntau differs from the IR basis size (gw_ir_size)";
      return GW_ERR_ARG;
    }
    gwir::ir_grids(beta, lambda, eps, t);
    g.tau = t.tau; g.x = t.x; g.w = t.w; g.nF = t.nF; g.nB = t.nB;
    g.TF = t.TF; g.TFp = t.TFp; g.TB = t.TB; g.TBp = t.TBp;
    finish_grids(beta, g);
  } catch (const std::exception& e) {
    why = e.what();
    return GW_ERR_ARG;
  }
  return GW_OK;
}

gw_status gw_ir_grids_host(double beta, double lambda, double eps, int ntau, double* tau, long long* nF,
                           long long* nB, gw_z* TF, gw_z* TFp, gw_z* TB, gw_z* TBp, double* w) {
  HostGrids g;
  std::string why;
  gw_status s = make_ir(beta, lambda, eps, ntau, g, why);
  if (s != GW_OK) return s;
  if (tau) std::memcpy(tau, g.tau.data(), g.tau.size() * 8);
  if (nF) std::memcpy(nF, g.nF.data(), g.nF.size() * 8);
  if (nB) std::memcpy(nB, g.nB.data(), g.nB.size() * 8);
  if (TF) std::memcpy(TF, g.TF.data(), g.TF.size() * 16);
  if (TFp) std::memcpy(TFp, g.TFp.data(), g.TFp.size() * 16);
  if (TB) std::memcpy(TB, g.TB.data(), g.TB.size() * 16);
  if (TBp) std::memcpy(TBp, g.TBp.data(), g.TBp.size() * 16);
  if (w) std::memcpy(w, g.w.data(), g.w.size() * 8);
  return GW_OK;
}

gw_status gw_build_ir_grids(gw_ctx* c, double lambda, double eps) {
  if (!c) return GW_ERR_ARG;
  const int nt = c->d.ntau;
  if (c->d.nw_f != nt || c->d.nw_b != nt + 1)
    return fail(c, GW_ERR_ARG, "IR grids need nw_f = ntau and nw_b = ntau + 1");
  HostGrids g;
  std::string why;
  gw_status s = make_ir(c->d.beta, lambda, eps, nt, g, why);
  if (s != GW_OK) return fail(c, s, why);
  return install_grids(c, g);
}

gw_status gw_get_grids(const gw_ctx* cc, double* tau, long long* nF, long long* nB, gw_z* TF,
                       gw_z* TFp, gw_z* TB, gw_z* TBp, double* w) {
  gw_ctx* c = const_cast<gw_ctx*>(cc);
  if (!c) return GW_ERR_ARG;
  if (!c->grids) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (tau) std::memcpy(tau, c->tau.data(), c->tau.size() * 8);
  if (nF) std::memcpy(nF, c->nF.data(), c->nF.size() * 8);
  if (nB) std::memcpy(nB, c->nB.data(), c->nB.size() * 8);
  if (TF) std::memcpy(TF, c->TF.data(), c->TF.size() * 16);
  if (TFp) std::memcpy(TFp, c->TFp.data(), c->TFp.size() * 16);
  if (TB) std::memcpy(TB, c->TB.data(), c->TB.size() * 16);
  if (TBp) std::memcpy(TBp, c->TBp.data(), c->TBp.size() * 16);
  if (w) std::memcpy(w, c->w.data(), c->w.size() * 8);
  return GW_OK;
}

// Bytes of the polarization / self-energy chains for a tau chunk: two
// intermediates of tc x Nk x naux x nao^2 (plus complex64 copies of two G
// arrays in mixed precision).
// complex64 V and chain intermediates (GW_PREC_FP32, GW_PREC_BF16X3, GW_PREC_BF16X6)
static bool lowp(const gw_ctx* c) { return c->d.precision != GW_PREC_FP64; }
// split-bf16 operands of the two large contractions (GW_PREC_BF16X3, GW_PREC_BF16X6)
static bool splitbf(const gw_ctx* c) {
  return c->d.precision == GW_PREC_BF16X3 || c->d.precision == GW_PREC_BF16X6;
}
static int nsplit(const gw_ctx* c) { return c->d.precision == GW_PREC_BF16X6 ? 3 : 2; }
// Chain workspace: two tau-chunk regions (X and Zt, or Vt and L); in the
// low-precision modes two complex64 copies of G after them.
static size_t region_bytes(const gw_ctx* c, int tc) {
  return align256((size_t)tc * c->nk * c->sv * (lowp(c) ? 8 : 16));
}
static size_t gslot_bytes(const gw_ctx* c) { return align256((size_t)c->d.ntau * c->nk * c->n2 * 8); }

// complex64 P~ of one tau chunk (split mode, after the G copies)
static size_t pchunk_bytes(const gw_ctx* c, int tc) {
  return align256((size_t)tc * c->d.naux * (size_t)c->d.naux * 8);
}

static size_t chain_bytes(const gw_ctx* c, int tc) {
  return 2 * region_bytes(c, tc) + (lowp(c) ? 2 * gslot_bytes(c) : 0) + (splitbf(c) ? pchunk_bytes(c, tc) : 0);
}

static size_t screened_bytes(const gw_ctx* c, int nq) {
  return align256((size_t)nq * c->d.nw_b * c->d.naux * (size_t)c->d.naux * 16);
}

static size_t hf_bytes(const gw_ctx* c) {
  return align256((size_t)c->nk * c->sv * 16) + align256((size_t)c->nk * c->n2 * 16) +
         align256((size_t)c->d.naux * 16);
}

// Per-q polarization buffers of the whole-chain calls (gw_sigma per q,
// gw_sigma_jvp, gw_sigma_vjp): two tau arrays and four frequency arrays of
// naux^2 complex numbers, at the end of the workspace.
static size_t perq_tau_bytes(const gw_ctx* c) {
  return align256((size_t)c->d.ntau * c->d.naux * (size_t)c->d.naux * 16);
}
static size_t perq_w_bytes(const gw_ctx* c) { return screened_bytes(c, 1); }
static size_t perq_bytes(const gw_ctx* c) { return 2 * perq_tau_bytes(c) + 4 * perq_w_bytes(c); }

// Front region the sub-calls of the whole-chain calls use.
static size_t sigma_front_bytes(const gw_ctx* c, int tc) {
  return std::max({chain_bytes(c, tc), screened_bytes(c, 1), hf_bytes(c)});
}

size_t gw_workspace_bytes(const gw_ctx* c, int op, int tau_chunk) {
  if (!c) return 0;
  switch (op) {
    case GW_OP_DYSON_JVP:
      return 2 * align256((size_t)c->d.nw_f * c->nk * c->n2 * 16);
    case GW_OP_POLARIZATION:
    case GW_OP_SELF_ENERGY:
      if (tau_chunk < 1 || tau_chunk > c->d.ntau) return 0;
      return chain_bytes(c, tau_chunk);
    case GW_OP_SCREENED_W:
      if (tau_chunk < 1) return 0;
      return screened_bytes(c, tau_chunk);
    case GW_OP_HF:
      return hf_bytes(c);
    case GW_OP_SIGMA:
      if (tau_chunk < 1 || tau_chunk > c->d.ntau) return 0;
      return sigma_front_bytes(c, tau_chunk) + perq_bytes(c);
    case GW_OP_THERMO: {
      const size_t nb = (size_t)c->d.nw_f * c->nk;
      return align256(nb * c->n2 * 16) + 3 * align256(nb * 8) + align256((size_t)c->nk * c->n2 * 16) +
             align256((size_t)c->d.nw_f * 16) + align256((size_t)c->nk * 3 * 8);
    }
  }
  return 0;
}

gw_status gw_set_workspace(gw_ctx* c, void* dev, size_t bytes, int tau_chunk) {
  if (!c) return GW_ERR_ARG;
  if (tau_chunk < 1 || tau_chunk > c->d.ntau)
    return fail(c, GW_ERR_ARG, "tau_chunk must be in 1..ntau");
  if (bytes && !dev) return fail(c, GW_ERR_ARG, "workspace pointer is NULL");
  if (((uintptr_t)dev) & 255) return fail(c, GW_ERR_ARG, "workspace must be 256-byte aligned");
  c->ws = dev;
  c->ws_bytes = bytes;
  c->tc = tau_chunk;
  return GW_OK;
}

gw_status gw_mix(gw_ctx* c, long long n, double alpha, const gw_z* X, gw_z* Y, double* maxdiff) {
  if (!c) return GW_ERR_ARG;
  if (!Y || n < 0) return fail(c, GW_ERR_ARG, "bad gw_mix arguments");
  if (!std::isfinite(alpha)) return fail(c, GW_ERR_ARG, "alpha is not finite");
  if (n == 0) {
    if (maxdiff) *maxdiff = 0.0;
    return GW_OK;
  }
  // partial maxima reuse the electron-count scratch (nw_f * nk + 8 doubles)
  const int cap = c->d.nw_f * c->nk + 7;
  const int nblk = (int)std::max(1LL, std::min<long long>({(n + 255) / 256, 2048LL, (long long)cap - 1}));
  HIPCHK(c, mix_launch(n, alpha, (const double2*)X, (double2*)Y, maxdiff ? c->dpart : nullptr, nblk,
                       c->st));
  if (maxdiff) {
    HIPCHK(c, hipMemcpyAsync(maxdiff, c->dpart + nblk, sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (!std::isfinite(*maxdiff)) return fail(c, GW_ERR_NONFINITE, "gw_mix: non-finite element");
  }
  return GW_OK;
}

gw_status gw_profile_enable(gw_ctx* c, int on) {
  if (!c) return GW_ERR_ARG;
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int k = 0; k < KC_COUNT; ++k) {
    for (auto& p : c->ev[k]) {
      (void)hipEventDestroy(p.first);
      (void)hipEventDestroy(p.second);
    }
    c->ev[k].clear();
    if (on) {
      c->launches[k] = 0;
      c->flops[k] = 0.0;
      c->ms[k] = 0.0;
    }
  }
  c->prof = on != 0;
  return GW_OK;
}

gw_status gw_profile_read(gw_ctx* c, int kc, long long* launches, double* ms, double* flops) {
  if (!c) return GW_ERR_ARG;
  if (kc < 0 || kc >= KC_COUNT) return fail(c, GW_ERR_ARG, "kernel class out of range");
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (auto& p : c->ev[kc]) {
    float t = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&t, p.first, p.second));
    c->ms[kc] += t;
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  c->ev[kc].clear();
  if (launches) *launches = c->launches[kc];
  if (ms) *ms = c->ms[kc];
  if (flops) *flops = c->flops[kc];
  return GW_OK;
}

gw_status gw_synchronize(gw_ctx* c) {
  if (!c) return GW_ERR_ARG;
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GW_OK;
}

// ------------------------------------------------------------- Eq. tilde_P0_tau
// Mixed-precision context: V and the chain intermediates are complex64, G is
// rounded to complex64 once per call, the MFMAs run in fp32 and the long
// contractions add each 512-element chunk of their K sum into fp64.
static const int kMixedChunk = 512;

// Scratch of one chain call: base pointer, bytes and tau chunk (the
// context's workspace, or another region of device memory).
struct Work {
  char* base;
  size_t bytes;
  int tc;
};
static Work ctx_work(gw_ctx* c) { return Work{(char*)c->ws, c->ws_bytes, c->tc}; }

// complex64 copy of G in slot 0 or 1 of the mixed-precision workspace
static gw_status g_to_c64(gw_ctx* c, const Work& w, const gw_z* G, void** Gc, int slot = 0) {
  const size_t off = 2 * region_bytes(c, w.tc) + (size_t)slot * gslot_bytes(c);
  *Gc = w.base + off;
  HIPCHK(c, to_c64_launch((const double2*)G, (float2*)*Gc, (long long)c->d.ntau * c->nk * c->n2, c->st));
  return GW_OK;
}

static gw_status pol_impl(gw_ctx* c, const Work& w, const void* V, const gw_z* G, const gw_z* Gb,
                          int q0, int nq, gw_z* P0, bool accumulate, bool two_slot);

gw_status gw_set_hermitian(gw_ctx* c, int mode) {
  if (!c) return GW_ERR_ARG;
  if (mode & ~(GW_HERM_FORWARD | GW_HERM_TWO_SLOT)) return fail(c, GW_ERR_ARG, "unknown Hermitian-mode bits");
  c->herm = mode;
  return GW_OK;
}

gw_status gw_set_mu_window(gw_ctx* c, double ne_tol) {
  if (!c) return GW_ERR_ARG;
  if (!std::isfinite(ne_tol) || ne_tol < 0.0) return fail(c, GW_ERR_ARG, "ne_tol must be finite and >= 0");
  c->mu_window = ne_tol;
  return GW_OK;
}

gw_status gw_polarization(gw_ctx* c, const void* V, const gw_z* G, int q0, int nq, gw_z* P0) {
  if (!c) return GW_ERR_ARG;
  return pol_impl(c, ctx_work(c), V, G, G, q0, nq, P0, false, false);
}

gw_status gw_polarization2(gw_ctx* c, const void* V, const gw_z* Ga, const gw_z* Gb, int q0, int nq,
                           int accumulate, gw_z* P0) {
  if (!c) return GW_ERR_ARG;
  return pol_impl(c, ctx_work(c), V, Ga, Gb, q0, nq, P0, accumulate != 0, true);
}

// gw_polarization on the fixed scratch array instead of the caller's
// workspace: the largest tau chunk whose intermediates fit is used.  Makes
// no allocation (profiling events are not recorded during the call).
gw_status gw_polarization_noalloc(gw_ctx* c, const void* V, const gw_z* G, int q0, int nq, gw_z* P0) {
  if (!c) return GW_ERR_ARG;
  if (!c->scratch) return fail(c, GW_ERR_DEVICE, "scratch address not set up");
  int tc = 0;
  for (int t = c->d.ntau; t >= 1; t = (t == 1) ? 0 : (t + 1) / 2)
    if (chain_bytes(c, t) <= kScratchBytes) { tc = t; break; }
  if (tc == 0)
    return fail(c, GW_ERR_WORKSPACE,
                "gw_polarization_noalloc: one tau slice of the intermediates needs " +
                    std::to_string(chain_bytes(c, 1)) + " bytes, above the fixed scratch of " +
                    std::to_string(kScratchBytes) + " bytes");
  const bool prof = c->prof;
  c->prof = false;
  const gw_status s = pol_impl(c, Work{c->scratch, kScratchBytes, tc}, V, G, G, q0, nq, P0, false, false);
  c->prof = prof;
  return s;
}

// One tau chunk of Eq. tilde_P0_tau in the split-bf16 modes (GW_PREC_BF16X3 / X6).
// The complex64 producers write X and Zt with K = (k, d, b) contiguous per
// row, so that the contraction's loader reads whole K-runs:
//   X2[tl][Q][k n2 + d nao + b]  = sum_a V[q][k][Q][d][a] G[t0+tl][k+q][a][b]
//   Z2[tl][Q'][k n2 + d nao + b] = sum_c G[nt-1-t0-tl][k][c][d] conj(V[q][k][Q'][c][b])
//   P0[iq][t0+tl][Q][Q'] (+)= -(ns/nk) sum_K X2[tl][Q][K] Z2[tl][Q'][K]   (bf16x3)
// Gd and Gbd are the complex64 copies of the two G slots.
static gw_status pol_split_chunk(gw_ctx* c, const char* Aq, const char* Gd, const char* Gbd, char* X, char* Z,
                                 int q, int iq, int t0, int tcur, int tc, gw_z* P0, bool accumulate,
                                 bool herm) {
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux, nt = c->d.ntau;
  const long long n2 = c->n2, sv = c->sv;
  const long long K = (long long)nk * n2, ldr = (long long)naux * K;
  GemmDesc g = gemm_desc();
  g.A = Aq; g.B = Gd + (size_t)t0 * nk * n2 * 8; g.C = X;
  g.M = naux * nao; g.N = tcur * nao; g.K = nao; g.batch = nk;
  g.am = aff(nao); g.ak = aff(1);
  g.bk = aff(nao); g.bn = two(nao, 1, (long long)nk * n2);
  g.cm = two(nao, nao, K); g.cn = two(nao, 1, ldr);
  g.ba = aff(sv); g.bb = aff(0); g.bc = aff(n2);
  g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsB = n2;   // G^{k+q}
  g.ta = g.tb = g.tc = 1; g.f32 = 1;
  g.tag = KC_POL_PRODUCER;
  gw_status s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)tc * ldr});
  if (s != GW_OK) return s;
  g = gemm_desc();
  // rows over tr = tcur-1-tl: G read with a positive stride (uniform-K loop)
  g.A = Gbd + (size_t)(nt - t0 - tcur) * nk * n2 * 8; g.B = Aq; g.C = Z + (size_t)(tcur - 1) * ldr * 8;
  g.M = tcur * nao; g.N = naux * nao; g.K = nao; g.batch = nk;
  g.am = two(nao, 1, (long long)nk * n2); g.ak = aff(nao);
  g.bk = aff(nao); g.bn = two(nao, 1, n2); g.conjB = 1;
  g.cm = two(nao, nao, -ldr); g.cn = two(nao, 1, K);
  g.ba = aff(n2); g.bb = aff(sv); g.bc = aff(n2);
  g.ta = g.tb = g.tc = 1; g.f32 = 1;
  g.tag = KC_POL_PRODUCER;
  if ((s = run(c, g, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)nk * sv},
               Ext{-(long long)(tcur - 1) * ldr, (long long)(tc - tcur + 1) * ldr})) != GW_OK)
    return s;
  SplitDesc d = split_desc();
  d.A = X; d.B = Z; d.C = (double2*)P0 + ((long long)iq * nt + t0) * naux * naux;
  d.M = naux; d.N = naux; d.K = (int)K; d.batch = tcur;
  d.ta = d.tb = 1; d.tc = 0;
  d.am = aff(K); d.aks = 1; d.bn = aff(K); d.bks = 1;
  d.ba = d.bb = aff(ldr); d.bc = aff((long long)naux * naux);
  d.cm = aff(naux); d.cn = aff(1);
  d.alpha_r = -(double)c->d.ns / nk;
  if (accumulate) { d.beta_zero = 0; d.beta_r = 1.0; }
  d.tri = herm ? 1 : 0; d.kchunk = kMixedChunk; d.nsplit = nsplit(c);
  d.tag = KC_POL_CONTRACT;
  if ((s = run_split(c, d, Ext{0, (long long)tcur * ldr}, Ext{0, (long long)tcur * ldr},
                     Ext{0, (long long)tcur * naux * naux})) != GW_OK)
    return s;
  if (herm) HIPCHK(c, herm_fill_launch((double2*)d.C, naux, tcur, c->st));
  return GW_OK;
}

// G fills the tau slot (G^{k+q}(tau_i)), Gb the mirrored slot (G^k(tau_{ntau-1-i})).
static gw_status pol_impl(gw_ctx* c, const Work& w, const void* V, const gw_z* G, const gw_z* Gb,
                          int q0, int nq, gw_z* P0, bool accumulate, bool two_slot) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built");
  if (q0 < 0 || nq < 0 || q0 + nq > c->nk) return fail(c, GW_ERR_ARG, "q range outside the mesh");
  if (nq == 0) return GW_OK;
  if (!V || !G || !Gb || !P0) return fail(c, GW_ERR_ARG, "NULL array");
  const int tc = w.tc;
  if (!w.base || tc < 1 || tc > c->d.ntau || w.bytes < chain_bytes(c, tc))
    return fail(c, GW_ERR_WORKSPACE, "polarization workspace too small");
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux, nt = c->d.ntau;
  const long long n2 = c->n2, sv = c->sv;
  const long long S = (long long)nk * sv;                // one tau slice of X or Zt
  const bool f32 = lowp(c);
  const bool sb = splitbf(c);
  const size_t ez = f32 ? 8 : 16;                        // bytes of V / X / Zt / G elements
  char* X = w.base;
  char* Z = w.base + region_bytes(c, tc);
  const char* Vd = (const char*)V;
  const char* Gd = (const char*)G;
  const char* Gbd = (const char*)Gb;
  if (f32) {
    void* Gc = nullptr;
    gw_status s = g_to_c64(c, w, G, &Gc);
    if (s != GW_OK) return s;
    Gd = Gbd = (const char*)Gc;
    if (Gb != G) {
      if ((s = g_to_c64(c, w, Gb, &Gc, 1)) != GW_OK) return s;
      Gbd = (const char*)Gc;
    }
  }
  const int t = f32 ? 1 : 0;
  // P0^q(tau) is Hermitian when G^k(tau) is and V^{k+q,k}(Q) = V^{k,k+q}(Q)^H,
  // and so is each two-slot term P0[Ga, Gb] for Hermitian Ga, Gb: then only
  // the tiles on and above the diagonal are contracted (accumulating into an
  // upper triangle and refilling the lower one keeps a Hermitian sum).
  const bool herm = (c->herm & (two_slot ? GW_HERM_TWO_SLOT : GW_HERM_FORWARD)) != 0;
  for (int q = q0; q < q0 + nq; ++q) {
    const char* Aq = Vd + (size_t)q * nk * sv * ez;
    for (int t0 = 0; t0 < nt; t0 += tc) {
      const int tcur = std::min(tc, nt - t0);
      if (sb) {
        gw_status s = pol_split_chunk(c, Aq, Gd, Gbd, X, Z, q, q - q0, t0, tcur, tc, P0, accumulate, herm);
        if (s != GW_OK) return s;
        continue;
      }
      // X[tl][k][Q][d][b] = sum_a V[q][k][Q][d][a] G[t0+tl][k+q][a][b]
      GemmDesc g = gemm_desc();
      g.A = Aq; g.B = Gd + (size_t)t0 * nk * n2 * ez; g.C = X;
      g.M = naux * nao; g.N = tcur * nao; g.K = nao; g.batch = nk;
      g.am = aff(nao); g.ak = aff(1);
      g.bk = aff(nao); g.bn = two(nao, 1, (long long)nk * n2);
      g.cm = aff(nao); g.cn = two(nao, 1, S);
      g.ba = aff(sv); g.bb = aff(0); g.bc = aff(sv);
      g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsB = n2;   // G^{k+q}
      g.ta = g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_POL_PRODUCER;
      gw_status s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)tc * S});
      if (s != GW_OK) return s;
      // Zt[tl][k][Q'][d][b] = sum_c G[nt-1-t0-tl][k][c][d] conj(V[q][k][Q'][c][b])
      // Rows run over tr = tcur-1-tl, so that G is read with a positive
      // stride (the uniform-K loop needs non-negative operand strides) and
      // the rows are written backwards.
      g = gemm_desc();
      g.A = Gbd + (size_t)(nt - t0 - tcur) * nk * n2 * ez; g.B = Aq;
      g.C = Z + (size_t)(tcur - 1) * S * ez;
      g.M = tcur * nao; g.N = naux * nao; g.K = nao; g.batch = nk;
      g.am = two(nao, 1, (long long)nk * n2); g.ak = aff(nao);
      g.bk = aff(nao); g.bn = two(nao, 1, n2); g.conjB = 1;
      g.cm = two(nao, nao, -S); g.cn = two(nao, 1, n2);
      g.ba = aff(n2); g.bb = aff(sv); g.bc = aff(sv);
      g.ta = g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_POL_PRODUCER;
      if ((s = run(c, g, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)nk * sv},
                   Ext{-(long long)(tcur - 1) * S, (long long)(tc - tcur + 1) * S})) != GW_OK) return s;
      // P0[q-q0][t0+tl][Q][Q'] = -(ns/nk) sum_{k,e} X[tl][k][Q][e] Zt[tl][k][Q'][e]
      g = gemm_desc();
      g.A = X; g.B = Z; g.C = (double2*)P0 + ((long long)(q - q0) * nt + t0) * naux * naux;
      g.M = naux; g.N = naux; g.K = nk * (int)n2; g.batch = tcur;
      g.am = aff(n2); g.ak = two((unsigned)n2, 1, sv);
      g.bk = two((unsigned)n2, 1, sv); g.bn = aff(n2);
      g.cm = aff(naux); g.cn = aff(1);
      g.ba = aff(S); g.bb = aff(S); g.bc = aff((long long)naux * naux);
      g.alpha_r = -(double)c->d.ns / nk;
      if (accumulate) { g.beta_zero = 0; g.beta_r = 1.0; }
      g.ta = g.tb = t; g.tc = 0; g.f32 = t; g.kchunk = f32 ? kMixedChunk : 0;
      g.tag = KC_POL_CONTRACT;
      g.tri = herm ? 1 : 0;
      if ((s = run(c, g, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * naux * naux})) != GW_OK) return s;
      if (herm) HIPCHK(c, herm_fill_launch((double2*)g.C, naux, tcur, c->st));
    }
  }
  return GW_OK;
}

// ------------------------------------------------------------- transforms
static gw_status transform(gw_ctx* c, int stat, const gw_z* Xin, long long batch, long long R,
                           gw_z* Xout, bool forward) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (stat != GW_FERMION && stat != GW_BOSON) return fail(c, GW_ERR_ARG, "stat must be 0 or 1");
  if (batch < 0 || R < 0 || batch > 65535 || R > 0x7fffffffLL)
    return fail(c, GW_ERR_ARG, "batch or R out of range");
  if (batch == 0 || R == 0) return GW_OK;
  if (!Xin || !Xout) return fail(c, GW_ERR_ARG, "NULL array");
  const int nt = c->d.ntau;
  const int nw = stat == GW_FERMION ? c->d.nw_f : c->d.nw_b;
  const int rows = forward ? nw : nt, inner = forward ? nt : nw;
  GemmDesc g = gemm_desc();
  g.A = forward ? (stat == GW_FERMION ? c->dTF : c->dTB) : (stat == GW_FERMION ? c->dTFp : c->dTBp);
  g.B = (const double2*)Xin;
  g.C = (double2*)Xout;
  g.M = rows; g.N = (int)R; g.K = inner; g.batch = (int)batch;
  g.am = aff(inner); g.ak = aff(1);
  g.bk = aff(R); g.bn = aff(1);
  g.cm = aff(R); g.cn = aff(1);
  g.ba = aff(0); g.bb = aff((long long)inner * R); g.bc = aff((long long)rows * R);
  g.tag = KC_TRANSFORM;
  return run(c, g, Ext{0, (long long)rows * inner}, Ext{0, batch * inner * R}, Ext{0, batch * rows * R});
}

gw_status gw_tau_to_iw(gw_ctx* c, int stat, const gw_z* X_tau, long long batch, long long R,
                       gw_z* X_iw) {
  return transform(c, stat, X_tau, batch, R, X_iw, true);
}

gw_status gw_iw_to_tau(gw_ctx* c, int stat, const gw_z* X_iw, long long batch, long long R,
                       gw_z* X_tau) {
  return transform(c, stat, X_iw, batch, R, X_tau, false);
}

// ------------------------------------------------------------- Eq. tilde_P_omega
gw_status gw_screened_W(gw_ctx* c, const gw_z* P0, int nq, gw_z* Pt) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (nq < 0 || nq > c->nk) return fail(c, GW_ERR_ARG, "nq out of range");
  if (nq == 0) return GW_OK;
  if (!P0 || !Pt) return fail(c, GW_ERR_ARG, "NULL array");
  if (P0 == Pt) return fail(c, GW_ERR_ARG, "Pt_iw may not alias P0_iw");
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_SCREENED_W, nq))
    return fail(c, GW_ERR_WORKSPACE, "screened_W workspace too small");
  HIPCHK(c, zero_flag_launch(c->dflag, c->st));
  hipEvent_t e0 = nullptr;
  gw_status s = prof_begin(c, KC_WDYSON, &e0);
  if (s != GW_OK) return s;
  // Blocked right-looking LU with row pivoting inside each panel of kNb
  // columns; the trailing updates of A and of the right-hand side and the
  // blocked back substitution are batched GEMMs over all nq * nw_b matrices.
  const int n = c->d.naux, kNb = 32;
  const long long nmat = (long long)nq * c->d.nw_b, nn = (long long)n * n;
  double2* Am = (double2*)c->ws;
  double2* Bm = (double2*)Pt;
  HIPCHK(c, wlu_launch(0, (const double2*)P0, Am, Bm, n, 0, kNb, nmat, c->dflag, c->st));
  auto gemm = [&](double2* X, long long xo, double2* Y, long long yo, double2* Z, long long zo, int M,
                  int N, int K) -> gw_status {
    if (M <= 0 || N <= 0 || K <= 0) return GW_OK;
    GemmDesc g = gemm_desc();
    g.A = X + xo; g.B = Y + yo; g.C = Z + zo;
    g.M = M; g.N = N; g.K = K; g.batch = (int)nmat;
    g.am = aff(n); g.ak = aff(1); g.bk = aff(n); g.bn = aff(1); g.cm = aff(n); g.cn = aff(1);
    g.ba = g.bb = g.bc = aff(nn);
    g.alpha_r = -1.0; g.beta_zero = 0; g.beta_r = 1.0;
    g.tag = KC_OTHER;                 // timed as part of the whole solve (KC_WDYSON)
    const long long span = nmat * nn;
    return run(c, g, Ext{-xo, span - xo}, Ext{-yo, span - yo}, Ext{-zo, span - zo});
  };
  for (int j0 = 0; j0 < n; j0 += kNb) {
    const int j1 = std::min(j0 + kNb, n), w = j1 - j0, rest = n - j1;
    HIPCHK(c, wlu_launch(1, nullptr, Am, Bm, n, j0, kNb, nmat, c->dflag, c->st));
    HIPCHK(c, wlu_launch(2, nullptr, Am, Bm, n, j0, kNb, nmat, c->dflag, c->st));
    // A22 -= L21 U12 ;  B2 -= L21 B1
    if ((s = gemm(Am, (long long)j1 * n + j0, Am, (long long)j0 * n + j1, Am, (long long)j1 * n + j1,
                  rest, rest, w)) != GW_OK) return s;
    if ((s = gemm(Am, (long long)j1 * n + j0, Bm, (long long)j0 * n, Bm, (long long)j1 * n,
                  rest, n, w)) != GW_OK) return s;
  }
  const int nblk = (n + kNb - 1) / kNb;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j0 = b * kNb, w = std::min(kNb, n - j0);
    HIPCHK(c, wlu_launch(3, nullptr, Am, Bm, n, j0, kNb, nmat, c->dflag, c->st));
    // B[0:j0] -= U[0:j0, j0:j0+w] B[j0:j0+w]
    if ((s = gemm(Am, (long long)j0, Bm, (long long)j0 * n, Bm, 0, j0, n, w)) != GW_OK) return s;
  }
  const double nd = n;
  if ((s = prof_end(c, KC_WDYSON, e0, (32.0 / 3.0) * nd * nd * nd * nmat)) != GW_OK) return s;
  return read_flag(c, "screened_W");
}

// ------------------------------------------------------ Eq. tilde_Phi_GW
gw_status gw_screened_W_phi(gw_ctx* c, const gw_z* P0, int nq, gw_z* Pt, double* phi) {
  if (!c) return GW_ERR_ARG;
  if (!phi) return fail(c, GW_ERR_ARG, "NULL phi");
  *phi = 0.0;
  gw_status s = gw_screened_W(c, P0, nq, Pt);
  if (s != GW_OK || nq == 0) return s;
  // The LU of I - P0 is still packed in the workspace.  Weights of the
  // Matsubara sum: value at tau = 0 of the least-squares fit, i.e. the
  // beta^- row reversed (mirrored nodes) times TBp; real part, scaled by
  // 1 / (2 Nk).  dred[1..nw_b] holds the weights, dphi the per-matrix terms
  // and, after them, their sum.
  const int nt = c->d.ntau, nwb = c->d.nw_b;
  if (nwb + 1 > 2 * 1024 + 8) return fail(c, GW_ERR_ARG, "gw_screened_W_phi supports nw_b <= 2055");
  std::vector<double> up((size_t)nwb + 1, 0.0);
  for (int n = 0; n < nwb; ++n) {
    double r = 0.0;
    for (int i = 0; i < nt; ++i) r += c->w[nt - 1 - i] * c->TBp[(size_t)i * nwb + n].real();
    up[1 + n] = r / (2.0 * c->nk);
  }
  HIPCHK(c, hipMemcpyAsync(c->dred, up.data(), up.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
  const long long nmat = (long long)nq * nwb;
  HIPCHK(c, phi_terms_launch((const double2*)c->ws, (const double2*)P0, c->d.naux, nmat, c->dred + 1,
                             nwb, c->dphi, c->dphi + nmat, c->st));
  HIPCHK(c, hipMemcpyAsync(phi, c->dphi + nmat, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GW_OK;
}

// ------------------------------------------------------------- Eq. tilde_sigma2
gw_status gw_self_energy(gw_ctx* c, const void* V, const gw_z* G, const gw_z* Pt, int q0, int nq,
                         gw_z* Sig) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (q0 < 0 || nq < 0 || q0 + nq > c->nk) return fail(c, GW_ERR_ARG, "q range outside the mesh");
  if (nq == 0) return GW_OK;
  if (!V || !G || !Pt || !Sig) return fail(c, GW_ERR_ARG, "NULL array");
  const int tc = c->tc;
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_SELF_ENERGY, tc))
    return fail(c, GW_ERR_WORKSPACE, "self-energy workspace too small");
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux, nt = c->d.ntau;
  const long long n2 = c->n2, sv = c->sv;
  const long long S = (long long)nk * sv;
  const bool f32 = lowp(c);
  const bool sb = splitbf(c);
  const size_t ez = f32 ? 8 : 16;
  char* Vt = (char*)c->ws;
  char* L = (char*)c->ws + region_bytes(c, tc);
  const char* Vd = (const char*)V;
  const char* Gd = (const char*)G;
  if (f32) {
    void* Gc = nullptr;
    gw_status s = g_to_c64(c, ctx_work(c), G, &Gc);
    if (s != GW_OK) return s;
    Gd = (const char*)Gc;
  }
  const int t = f32 ? 1 : 0;
  const bool kmajor = f32;   // layouts of Vt and L (see the final contraction)
  for (int q = q0; q < q0 + nq; ++q) {
    const char* Aq = Vd + (size_t)q * nk * sv * ez;
    for (int t0 = 0; t0 < nt; t0 += tc) {
      const int tcur = std::min(tc, nt - t0);
      // Vt[tl][Q][kk][b][j] = sum_Q' Pt[q][t0+tl][Q][Q'] V[q][kk][Q'][b][j]
      // (fp64), or Vt[tl][kk][Q][b][j] (mixed): see the final contraction
      if (sb) {
        // bf16x3: rows Q of P~ (complex64 copy, K = Q' contiguous), columns
        // (kk, b, j) of the V slab read in place (K = Q' with stride n2)
        float2* Pc = (float2*)((char*)c->ws + 2 * region_bytes(c, tc) + 2 * gslot_bytes(c));
        HIPCHK(c, to_c64_launch((const double2*)Pt + ((long long)(q - q0) * nt + t0) * naux * naux, Pc,
                                (long long)tcur * naux * naux, c->st));
        SplitDesc d = split_desc();
        d.A = Pc;
        d.B = Aq; d.C = Vt;
        d.M = naux; d.N = nk * (int)n2; d.K = naux; d.batch = tcur;
        d.ta = 1; d.tb = 1; d.tc = 1;
        d.am = aff(naux); d.aks = 1; d.ba = aff((long long)naux * naux);
        d.bn = two((unsigned)n2, 1, sv); d.bks = n2; d.bb = aff(0);
        d.cm = aff(n2); d.cn = two((unsigned)n2, 1, sv); d.bc = aff(S);
        d.batch_fastest = 1;                    // every tau reads the same V slab
        d.kchunk = kMixedChunk; d.nsplit = nsplit(c);
        d.tag = KC_SE_CONTRACT;
        gw_status s = run_split(c, d, Ext{0, (long long)tcur * naux * naux}, Ext{0, (long long)nk * sv},
                                Ext{0, (long long)tcur * S});
        if (s != GW_OK) return s;
      } else {
        GemmDesc g = gemm_desc();
        g.A = (const double2*)Pt + ((long long)(q - q0) * nt + t0) * naux * naux;
        g.B = Aq; g.C = Vt;
        g.M = naux; g.N = nk * (int)n2; g.K = naux; g.batch = tcur;
        g.am = aff(naux); g.ak = aff(1);
        g.bk = aff(n2); g.bn = two((unsigned)n2, 1, sv);
        if (kmajor) { g.cm = aff(n2); g.cn = two((unsigned)n2, 1, sv); }
        else { g.cm = aff((long long)nk * n2); g.cn = aff(1); }
        g.ba = aff((long long)naux * naux); g.bb = aff(0); g.bc = aff(S);
        g.ta = 0; g.tb = g.tc = t; g.f32 = t;
        // groups of 8 tiles walk every tau: their V tiles and each tau's P~
        // panels stay in L2 (measured at si-4x4x4: fetch 49 -> 29 GB per q,
        // 25.6 vs 25.9 ms; groups of 16: 21 GB, 26.1 ms)
        g.batch_fastest = 2;
        g.group = 8;
        g.tag = KC_SE_CONTRACT;
        gw_status s = run(c, g, Ext{0, (long long)tcur * naux * naux}, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * S});
        if (s != GW_OK) return s;
      }
      // L[tl][kk][Q][i][b] (fp64) or L[tl][kk][i][Q][b] (mixed)
      //   = sum_a conj(V[q][kk][Q][a][i]) G[t0+tl][kk][a][b]
      gw_status s;
      GemmDesc g = gemm_desc();
      g.A = Aq; g.B = Gd + (size_t)t0 * nk * n2 * ez; g.C = L;
      g.M = naux * nao; g.N = tcur * nao; g.K = nao; g.batch = nk;
      g.am = two(nao, 1, n2); g.ak = aff(nao); g.conjA = 1;
      g.bk = aff(nao); g.bn = two(nao, 1, (long long)nk * n2);
      g.cm = kmajor ? two(nao, (long long)naux * nao, nao) : aff(nao);
      g.cn = two(nao, 1, S);
      g.ba = aff(sv); g.bb = aff(n2); g.bc = aff(sv);
      g.ta = g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_SE_PRODUCER;
      if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)tcur * S})) != GW_OK) return s;
      // Sig[t0+tl][kk+q][i][j] += -(1/nk) sum_{Q,b} L(i, (Q, b)) Vt((Q, b), j)
      // In the mixed layouts K = (Q, b) is contiguous in L and has stride nao
      // in Vt, so the uniform-K loop applies (fp32 MFMA steps are short
      // enough for the per-lane index carries of the other layout to show:
      // 6.6 vs 8.8 ms per q); the fp64 contraction streams at the HBM read
      // rate either way and is faster with its operands' k-points adjacent
      // (7.3 vs 8.1 ms per q).
      g = gemm_desc();
      g.A = L; g.B = Vt; g.C = (double2*)Sig + (long long)t0 * nk * n2;
      g.M = nao; g.N = nao; g.K = naux * nao; g.batch = tcur * nk;
      if (kmajor) {
        g.am = aff((long long)naux * nao); g.ak = aff(1);
        g.bk = aff(nao); g.bn = aff(1);
        g.bb = two(nk, sv, S);
      } else {
        g.am = aff(nao); g.ak = two(nao, 1, n2);
        g.bk = two(nao, nao, (long long)nk * n2); g.bn = aff(1);
        g.bb = two(nk, n2, S);
      }
      g.cm = aff(nao); g.cn = aff(1);
      g.ba = two(nk, sv, S); g.bc = two(nk, 0, (long long)nk * n2);
      g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsC = n2;
      g.alpha_r = -1.0 / nk;
      g.beta_zero = 0; g.beta_r = 1.0;
      g.ta = g.tb = t; g.tc = 0; g.f32 = t; g.kchunk = f32 ? kMixedChunk : 0;
      g.tag = KC_SE_FINAL;
      if ((s = run(c, g, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * nk * n2})) != GW_OK) return s;
    }
  }
  return GW_OK;
}

// ------------------------------------------------------------- density
static gw_status gamma_of(gw_ctx* c, const gw_z* G, double2* gamma) {
  GemmDesc g = gemm_desc();
  g.A = c->dw; g.B = (const double2*)G; g.C = gamma;
  g.M = 1; g.N = c->nk * (int)c->n2; g.K = c->d.ntau;
  g.am = aff(0); g.ak = aff(1); g.bk = aff((long long)c->nk * c->n2); g.bn = aff(1);
  g.cm = aff(0); g.cn = aff(1);
  g.alpha_r = -1.0;
  g.tag = KC_HF;
  return run(c, g, Ext{0, (long long)c->d.ntau}, Ext{0, (long long)c->d.ntau * c->nk * c->n2}, Ext{0, (long long)c->nk * c->n2});
}

gw_status gw_density(gw_ctx* c, const gw_z* G, const gw_z* S, gw_z* gamma, double* n_out) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (!G || !gamma || (n_out && !S)) return fail(c, GW_ERR_ARG, "NULL array");
  gw_status s = gamma_of(c, G, (double2*)gamma);
  if (s != GW_OK || !n_out) return s;
  HIPCHK(c, trace_launch((const double2*)gamma, (const double2*)S, c->d.nao, c->nk, c->dpart, c->st));
  HIPCHK(c, sum_launch(c->dpart, c->nk, (double)c->d.ns / c->nk, c->dpart + c->nk, c->st));
  HIPCHK(c, hipMemcpyAsync(n_out, c->dpart + c->nk, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GW_OK;
}

// ------------------------------------------------------------- Eqs. HF_J, HF_K
gw_status gw_hf(gw_ctx* c, const void* V, const gw_z* G, gw_z* gamma_out, gw_z* Sinf) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (!V || !G || !Sinf) return fail(c, GW_ERR_ARG, "NULL array");
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_HF, 1))
    return fail(c, GW_ERR_WORKSPACE, "HF workspace too small");
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux;
  const long long n2 = c->n2, sv = c->sv;
  double2* T1 = (double2*)c->ws;
  double2* gam = (double2*)((char*)c->ws + align256((size_t)nk * sv * 16));
  double2* vq = (double2*)((char*)gam + align256((size_t)nk * n2 * 16));
  if (gamma_out) gam = (double2*)gamma_out;
  const char* Vd = (const char*)V;
  const int tv = lowp(c) ? 1 : 0;   // V storage type
  const size_t ez = tv ? 8 : 16;
  gw_status s = gamma_of(c, G, gam);
  if (s != GW_OK) return s;
  // v[Q] = (ns/nk) sum_{k',b,a} V[0][k'][Q][b][a] gamma[k'][a][b]
  GemmDesc g = gemm_desc();
  g.A = Vd; g.B = gam; g.C = vq;
  g.M = naux; g.N = 1; g.K = nk * (int)n2;
  g.am = aff(n2); g.ak = two((unsigned)n2, 1, sv);
  g.bk = three(nao, nao, nao, 1, n2); g.bn = aff(0);
  g.cm = aff(1); g.cn = aff(0);
  g.alpha_r = (double)c->d.ns / nk;
  g.ta = tv;
  g.tag = KC_HF;
  if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2}, Ext{0, (long long)naux})) != GW_OK) return s;
  // J[k][e] = sum_Q v[Q] V[0][k][Q][e]
  g = gemm_desc();
  g.A = vq; g.B = Vd; g.C = (double2*)Sinf;
  g.M = 1; g.N = nk * (int)n2; g.K = naux;
  g.am = aff(0); g.ak = aff(1);
  g.bk = aff(n2); g.bn = two((unsigned)n2, 1, sv);
  g.cm = aff(0); g.cn = aff(1);
  g.tb = tv;
  g.tag = KC_HF;
  if ((s = run(c, g, Ext{0, (long long)naux}, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2})) != GW_OK) return s;
  for (int q = 0; q < nk; ++q) {
    const char* Aq = Vd + (size_t)q * nk * sv * ez;
    // T1[k][Q][i][b] = sum_a V[q][k][Q][i][a] gamma[k+q][a][b]
    g = gemm_desc();
    g.A = Aq; g.B = gam; g.C = T1;
    g.M = naux * nao; g.N = nao; g.K = nao; g.batch = nk;
    g.am = aff(nao); g.ak = aff(1); g.bk = aff(nao); g.bn = aff(1);
    g.cm = aff(nao); g.cn = aff(1);
    g.ba = aff(sv); g.bb = aff(0); g.bc = aff(sv);
    g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsB = n2;
    g.ta = tv;
    g.tag = KC_HF;
    if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2}, Ext{0, (long long)nk * sv})) != GW_OK) return s;
    // Sinf[k][i][j] += -(1/nk) sum_{Q,b} T1[k][Q][i][b] conj(V[q][k][Q][j][b])
    g = gemm_desc();
    g.A = T1; g.B = Aq; g.C = (double2*)Sinf;
    g.M = nao; g.N = nao; g.K = naux * nao; g.batch = nk;
    g.am = aff(nao); g.ak = two(nao, 1, n2);
    g.bk = two(nao, 1, n2); g.bn = aff(nao); g.conjB = 1;
    g.cm = aff(nao); g.cn = aff(1);
    g.ba = aff(sv); g.bb = aff(sv); g.bc = aff(n2);
    g.alpha_r = -1.0 / nk;
    g.beta_zero = 0; g.beta_r = 1.0;
    g.tb = tv;
    g.tag = KC_HF;
    if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2})) != GW_OK) return s;
  }
  return GW_OK;
}

// ------------------------------------------------------------- Eq. Dyson
gw_status gw_dyson_G(gw_ctx* c, const gw_z* H0, const gw_z* S, const gw_z* Sinf, const gw_z* Siw,
                     double mu, gw_z* G) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (!H0 || !S || !G) return fail(c, GW_ERR_ARG, "NULL array");
  if (!std::isfinite(mu)) return fail(c, GW_ERR_ARG, "mu is not finite");
  HIPCHK(c, zero_flag_launch(c->dflag, c->st));
  DysonArgs a{};
  a.H0 = (const double2*)H0; a.S = (const double2*)S;
  a.Sinf = (const double2*)Sinf; a.Siw = (const double2*)Siw;
  a.wF = c->dwF; a.rrow = c->drrow; a.mu = mu; a.nk = c->nk; a.nao = c->d.nao;
  a.G = (double2*)G; a.part = nullptr; a.flag = c->dflag;
  HIPCHK(c, dyson_launch(a, c->d.nw_f, c->st));
  return read_flag(c, "dyson_G");
}

gw_status gw_find_mu(gw_ctx* c, const gw_z* H0, const gw_z* S, const gw_z* Sinf, const gw_z* Siw,
                     double n_target, double tol, double* mu_inout, gw_z* G_iw, gw_z* G_tau,
                     double* n_out) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (!H0 || !S || !mu_inout) return fail(c, GW_ERR_ARG, "NULL array");
  if (G_tau && !G_iw) return fail(c, GW_ERR_ARG, "G_tau needs G_iw");
  if (!(n_target > 0.0) || !(n_target < (double)c->d.ns * c->d.nao))
    return fail(c, GW_ERR_ARG, "n_target must lie in (0, ns*nao)");
  if (!std::isfinite(*mu_inout)) return fail(c, GW_ERR_ARG, "initial mu is not finite");
  if (!(tol > 0.0)) tol = 1e-13;
  HIPCHK(c, zero_flag_launch(c->dflag, c->st));
  const double mu0 = *mu_inout;
  double n = 0.0;
  gw_status s;
  // root of N_e(mu) = target by bracket expansion from mu0 +/- 1 Ha and bisection
  auto root = [&](double target, double* out) -> gw_status {
    double lo = mu0 - 1.0, hi = mu0 + 1.0, step = 1.0, m = 0.0;
    gw_status r;
    int it = 0;
    for (;;) {
      if ((r = count_at(c, H0, S, Sinf, Siw, lo, nullptr, &m)) != GW_OK) return r;
      if (!(m > target)) break;
      step *= 2.0;
      lo -= step;
      if (++it > 60) return fail(c, GW_ERR_NOCONV, "mu search: no lower bracket");
    }
    step = 1.0;
    it = 0;
    for (;;) {
      if ((r = count_at(c, H0, S, Sinf, Siw, hi, nullptr, &m)) != GW_OK) return r;
      if (!(m < target)) break;
      step *= 2.0;
      hi += step;
      if (++it > 60) return fail(c, GW_ERR_NOCONV, "mu search: no upper bracket");
    }
    it = 0;
    while (hi - lo > tol && it < 400) {
      const double mid = 0.5 * (lo + hi);
      if ((r = count_at(c, H0, S, Sinf, Siw, mid, nullptr, &m)) != GW_OK) return r;
      if (m < target) lo = mid; else hi = mid;
      ++it;
    }
    if (hi - lo > tol) return fail(c, GW_ERR_NOCONV, "mu search: bracket not narrowed to tol");
    *out = 0.5 * (lo + hi);
    return GW_OK;
  };
  double mu = 0.0;
  if (c->mu_window > 0.0) {
    const double w = std::min(c->mu_window, 0.5 * std::min(n_target, (double)c->d.ns * c->d.nao - n_target));
    // keep mu0 when its count is inside the window, else the window's midpoint
    if ((s = count_at(c, H0, S, Sinf, Siw, mu0, nullptr, &n)) != GW_OK) return s;
    if (std::fabs(n - n_target) <= w) {
      mu = mu0;
    } else {
      double m_lo = 0.0, m_hi = 0.0;
      if ((s = root(n_target - w, &m_lo)) != GW_OK) return s;
      if ((s = root(n_target + w, &m_hi)) != GW_OK) return s;
      mu = 0.5 * (m_lo + m_hi);
    }
  } else {
    if ((s = root(n_target, &mu)) != GW_OK) return s;
  }
  if ((s = count_at(c, H0, S, Sinf, Siw, mu, G_iw, &n)) != GW_OK) return s;
  if ((s = read_flag(c, "find_mu")) != GW_OK) return s;
  *mu_inout = mu;
  if (n_out) *n_out = n;
  if (G_tau) {
    if ((s = gw_iw_to_tau(c, GW_FERMION, G_iw, 1, (long long)c->nk * c->n2, G_tau)) != GW_OK)
      return s;
  }
  return GW_OK;
}


// =========================================================================
// Derivatives of G -> (Sigma_inf, Sigma~).  The map is holomorphic in G, so
// a vector-Jacobian product is the conjugate-transposed Jacobian applied to
// the cotangent (the convention of torch autograd for complex tensors).
// All of these need a GW_PREC_FP64 context.
// =========================================================================

// calls that never read V run in either precision
static gw_status need_grids(gw_ctx* c) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  return GW_OK;
}

gw_status gw_screened_W_lin(gw_ctx* c, const gw_z* Pt, const gw_z* X, int nq, int adjoint, gw_z* Y) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (nq < 0 || nq > c->nk) return fail(c, GW_ERR_ARG, "nq out of range");
  if (nq == 0) return GW_OK;
  if (!Pt || !X || !Y) return fail(c, GW_ERR_ARG, "NULL array");
  if (X == Y || Pt == Y) return fail(c, GW_ERR_ARG, "Y may not alias Pt or X");
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_SCREENED_W, nq))
    return fail(c, GW_ERR_WORKSPACE, "screened_W workspace too small");
  const int n = c->d.naux;
  const long long nn = (long long)n * n, nmat = (long long)nq * c->d.nw_b;
  double2* T = (double2*)c->ws;
  // T = X + op(Pt) X, then Y = T + T op(Pt), op = identity (JVP) or ^H (VJP):
  // (I + Pt) X (I + Pt) is the derivative of (I - P0)^{-1} P0 = (I - P0)^{-1} - I.
  HIPCHK(c, mix_launch(nmat * nn, 1.0, (const double2*)X, T, nullptr, 2048, c->st));
  GemmDesc g = gemm_desc();
  g.A = Pt; g.B = X; g.C = T;
  g.M = n; g.N = n; g.K = n; g.batch = (int)nmat;
  if (adjoint) { g.am = aff(1); g.ak = aff(n); g.conjA = 1; } else { g.am = aff(n); g.ak = aff(1); }
  g.bk = aff(n); g.bn = aff(1); g.cm = aff(n); g.cn = aff(1);
  g.ba = g.bb = g.bc = aff(nn);
  g.beta_zero = 0; g.beta_r = 1.0;
  g.tag = KC_OTHER;
  if ((s = run(c, g, Ext{0, nmat * nn}, Ext{0, nmat * nn}, Ext{0, nmat * nn})) != GW_OK) return s;
  HIPCHK(c, mix_launch(nmat * nn, 1.0, T, (double2*)Y, nullptr, 2048, c->st));
  g = gemm_desc();
  g.A = T; g.B = Pt; g.C = Y;
  g.M = n; g.N = n; g.K = n; g.batch = (int)nmat;
  g.am = aff(n); g.ak = aff(1);
  if (adjoint) { g.bk = aff(1); g.bn = aff(n); g.conjB = 1; } else { g.bk = aff(n); g.bn = aff(1); }
  g.cm = aff(n); g.cn = aff(1);
  g.ba = g.bb = g.bc = aff(nn);
  g.beta_zero = 0; g.beta_r = 1.0;
  g.tag = KC_OTHER;
  return run(c, g, Ext{0, nmat * nn}, Ext{0, nmat * nn}, Ext{0, nmat * nn});
}

gw_status gw_transform_adjoint(gw_ctx* c, int stat, int inverse, const gw_z* Xin, long long batch,
                               long long R, gw_z* Xout) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (stat != GW_FERMION && stat != GW_BOSON) return fail(c, GW_ERR_ARG, "stat must be 0 or 1");
  if (batch < 0 || R < 0 || batch > 65535 || R > 0x7fffffffLL)
    return fail(c, GW_ERR_ARG, "batch or R out of range");
  if (batch == 0 || R == 0) return GW_OK;
  if (!Xin || !Xout) return fail(c, GW_ERR_ARG, "NULL array");
  const int nt = c->d.ntau;
  const int nw = stat == GW_FERMION ? c->d.nw_f : c->d.nw_b;
  // inverse = 0: Xout[b][i][r] = sum_n conj(T[n][i]) Xin[b][n][r]  (adjoint of tau -> i w)
  // inverse = 1: Xout[b][n][r] = sum_i conj(Tp[i][n]) Xin[b][i][r] (adjoint of i w -> tau)
  const int rows = inverse ? nw : nt, inner = inverse ? nt : nw;
  GemmDesc g = gemm_desc();
  g.A = inverse ? (stat == GW_FERMION ? c->dTFp : c->dTBp) : (stat == GW_FERMION ? c->dTF : c->dTB);
  g.B = Xin; g.C = Xout;
  g.M = rows; g.N = (int)R; g.K = inner; g.batch = (int)batch;
  g.am = aff(1); g.ak = aff(rows); g.conjA = 1;
  g.bk = aff(R); g.bn = aff(1); g.cm = aff(R); g.cn = aff(1);
  g.ba = aff(0); g.bb = aff((long long)inner * R); g.bc = aff((long long)rows * R);
  g.tag = KC_TRANSFORM;
  return run(c, g, Ext{0, (long long)rows * inner}, Ext{0, batch * inner * R}, Ext{0, batch * rows * R});
}

// The VJP contractions in every precision: fp64, or in the complex64 modes
// V complex64, complex64 intermediates, fp32 MFMA (operands rounded on load)
// with fp64 sums of 512-term chunks for the long contractions, outputs fp64.
struct VjpMode {
  int t;        // storage type of V and of the intermediates
  size_t ez;    // their element size
  int kchunk;
};
static VjpMode vjp_mode(const gw_ctx* c) {
  const bool f32 = lowp(c);
  return VjpMode{f32 ? 1 : 0, f32 ? (size_t)8 : (size_t)16, f32 ? kMixedChunk : 0};
}

gw_status gw_self_energy_vjp(gw_ctx* c, const void* V, const gw_z* G, const gw_z* Pt,
                             const gw_z* Sbar, int q0, int nq, gw_z* Gbar, gw_z* Ptbar) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (q0 < 0 || nq < 0 || q0 + nq > c->nk) return fail(c, GW_ERR_ARG, "q range outside the mesh");
  if (nq == 0) return GW_OK;
  if (!V || !G || !Pt || !Sbar || !Gbar || !Ptbar) return fail(c, GW_ERR_ARG, "NULL array");
  const int tc = c->tc;
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_SELF_ENERGY, tc))
    return fail(c, GW_ERR_WORKSPACE, "self-energy workspace too small");
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux, nt = c->d.ntau;
  const long long n2 = c->n2, sv = c->sv, S = (long long)nk * sv;
  const VjpMode vm = vjp_mode(c);
  const int t = vm.t;
  char* R0 = (char*)c->ws;
  char* R1 = (char*)c->ws + region_bytes(c, tc);
  for (int q = q0; q < q0 + nq; ++q) {
    const char* Aq = (const char*)V + (size_t)q * nk * sv * vm.ez;
    for (int t0 = 0; t0 < nt; t0 += tc) {
      const int tcur = std::min(tc, nt - t0);
      const gw_z* Ptq = Pt + ((long long)(q - q0) * nt + t0) * naux * naux;
      // R0 = Vt[tl][Q][kk][b][j] = sum_Q' Pt[Q][Q'] V[q][kk][Q'][b][j]
      GemmDesc g = gemm_desc();
      g.A = Ptq; g.B = Aq; g.C = R0;
      g.M = naux; g.N = nk * (int)n2; g.K = naux; g.batch = tcur;
      g.am = aff(naux); g.ak = aff(1); g.bk = aff(n2); g.bn = two((unsigned)n2, 1, sv);
      g.cm = aff((long long)nk * n2); g.cn = aff(1);
      g.ba = aff((long long)naux * naux); g.bb = aff(0); g.bc = aff(S);
      g.ta = 0; g.tb = g.tc = t; g.f32 = t;
      g.batch_fastest = 1;
      g.tag = KC_SE_CONTRACT;
      if ((s = run(c, g, Ext{0, (long long)tcur * naux * naux}, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * S})) != GW_OK) return s;
      // R1 = L'[tl][kk][Q][a][j] = sum_i V[q][kk][Q][a][i] Sbar[t][kk+q][i][j]
      g = gemm_desc();
      g.A = Aq; g.B = Sbar + (size_t)t0 * nk * n2; g.C = R1;
      g.M = naux * nao; g.N = tcur * nao; g.K = nao; g.batch = nk;
      g.am = aff(nao); g.ak = aff(1); g.bk = aff(nao); g.bn = two(nao, 1, (long long)nk * n2);
      g.cm = aff(nao); g.cn = two(nao, 1, S);
      g.ba = aff(sv); g.bb = aff(0); g.bc = aff(sv);
      g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsB = n2;
      g.ta = g.tc = t; g.tb = 0; g.f32 = t;
      g.tag = KC_SE_PRODUCER;
      if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)tcur * S})) != GW_OK) return s;
      // Gbar[t][kk][a][b] += -(1/nk) sum_{Q,j} L'[tl][kk][Q][a][j] conj(Vt[tl][Q][kk][b][j])
      g = gemm_desc();
      g.A = R1; g.B = R0; g.C = Gbar + (size_t)t0 * nk * n2;
      g.M = nao; g.N = nao; g.K = naux * nao; g.batch = tcur * nk;
      g.am = aff(nao); g.ak = two(nao, 1, n2);
      g.bk = two(nao, 1, (long long)nk * n2); g.bn = aff(nao); g.conjB = 1;
      g.cm = aff(nao); g.cn = aff(1);
      g.ba = two(nk, sv, S); g.bb = two(nk, n2, S); g.bc = two(nk, n2, (long long)nk * n2);
      g.alpha_r = -1.0 / nk; g.beta_zero = 0; g.beta_r = 1.0;
      g.ta = g.tb = t; g.tc = 0; g.f32 = t; g.kchunk = vm.kchunk;
      g.tag = KC_SE_FINAL;
      if ((s = run(c, g, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * nk * n2})) != GW_OK) return s;
      // R0 = Y[tl][kk][Q'][a][j] = sum_b G[t][kk][a][b] V[q][kk][Q'][b][j]
      g = gemm_desc();
      g.A = G + (size_t)t0 * nk * n2; g.B = Aq; g.C = R0;
      g.M = tcur * nao; g.N = naux * nao; g.K = nao; g.batch = nk;
      g.am = two(nao, nao, (long long)nk * n2); g.ak = aff(1);
      g.bk = aff(nao); g.bn = two(nao, 1, n2);
      g.cm = two(nao, nao, S); g.cn = two(nao, 1, n2);
      g.ba = aff(n2); g.bb = aff(sv); g.bc = aff(sv);
      g.ta = 0; g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_SE_PRODUCER;
      if ((s = run(c, g, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * S})) != GW_OK) return s;
      // Ptbar[q][t][Q][Q'] = -(1/nk) sum_{kk,a,j} L'[tl][kk][Q][a][j] conj(Y[tl][kk][Q'][a][j])
      g = gemm_desc();
      g.A = R1; g.B = R0; g.C = Ptbar + ((long long)(q - q0) * nt + t0) * naux * naux;
      g.M = naux; g.N = naux; g.K = nk * (int)n2; g.batch = tcur;
      g.am = aff(n2); g.ak = two((unsigned)n2, 1, sv);
      g.bk = two((unsigned)n2, 1, sv); g.bn = aff(n2); g.conjB = 1;
      g.cm = aff(naux); g.cn = aff(1);
      g.ba = aff(S); g.bb = aff(S); g.bc = aff((long long)naux * naux);
      g.alpha_r = -1.0 / nk;
      g.ta = g.tb = t; g.tc = 0; g.f32 = t; g.kchunk = vm.kchunk;
      g.tag = KC_POL_CONTRACT;
      if ((s = run(c, g, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * naux * naux})) != GW_OK) return s;
    }
  }
  return GW_OK;
}

gw_status gw_polarization_vjp(gw_ctx* c, const void* V, const gw_z* G, const gw_z* P0bar, int q0,
                              int nq, gw_z* Gbar) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (q0 < 0 || nq < 0 || q0 + nq > c->nk) return fail(c, GW_ERR_ARG, "q range outside the mesh");
  if (nq == 0) return GW_OK;
  if (!V || !G || !P0bar || !Gbar) return fail(c, GW_ERR_ARG, "NULL array");
  const int tc = c->tc;
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_POLARIZATION, tc))
    return fail(c, GW_ERR_WORKSPACE, "polarization workspace too small");
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux, nt = c->d.ntau;
  const long long n2 = c->n2, sv = c->sv, S = (long long)nk * sv;
  const double sc = -(double)c->d.ns / nk;
  const VjpMode vm = vjp_mode(c);
  const int t = vm.t;
  char* R0 = (char*)c->ws;
  char* R1 = (char*)c->ws + region_bytes(c, tc);
  for (int q = q0; q < q0 + nq; ++q) {
    const char* Aq = (const char*)V + (size_t)q * nk * sv * vm.ez;
    for (int t0 = 0; t0 < nt; t0 += tc) {
      const int tcur = std::min(tc, nt - t0);
      const gw_z* Pb = P0bar + ((long long)(q - q0) * nt + t0) * naux * naux;
      // --- tau slot: Gbar[t][k+q] += sc sum_{Q,d} conj(V[q][k][Q][d][a]) U[Q][k][d][b]
      // R1 = W[tl][k][Q'][d][b] = sum_c conj(G[nt-1-t][k][c][d]) V[q][k][Q'][c][b]
      GemmDesc g = gemm_desc();
      g.A = G + (size_t)(nt - 1 - t0) * nk * n2; g.B = Aq; g.C = R1;
      g.M = tcur * nao; g.N = naux * nao; g.K = nao; g.batch = nk;
      g.am = two(nao, 1, -(long long)nk * n2); g.ak = aff(nao); g.conjA = 1;
      g.bk = aff(nao); g.bn = two(nao, 1, n2);
      g.cm = two(nao, nao, S); g.cn = two(nao, 1, n2);
      g.ba = aff(n2); g.bb = aff(sv); g.bc = aff(sv);
      g.ta = 0; g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_POL_PRODUCER;
      if ((s = run(c, g, Ext{-(long long)(tcur - 1) * nk * n2, (long long)nk * n2}, Ext{0, (long long)nk * sv}, Ext{0, (long long)tc * S})) != GW_OK) return s;
      // R0 = U[tl][Q][k][e] = sum_Q' Pbar[Q][Q'] W[tl][k][Q'][e]
      g = gemm_desc();
      g.A = Pb; g.B = R1; g.C = R0;
      g.M = naux; g.N = nk * (int)n2; g.K = naux; g.batch = tcur;
      g.am = aff(naux); g.ak = aff(1); g.bk = aff(n2); g.bn = two((unsigned)n2, 1, sv);
      g.cm = aff((long long)nk * n2); g.cn = aff(1);
      g.ba = aff((long long)naux * naux); g.bb = aff(S); g.bc = aff(S);
      g.ta = 0; g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_SE_CONTRACT;
      if ((s = run(c, g, Ext{0, (long long)tcur * naux * naux}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * S})) != GW_OK) return s;
      // Gbar[t0+tl][k+q][a][b] += sc sum_{Q,d} conj(V[q][k][Q][d][a]) U[tl][Q][k][d][b]
      g = gemm_desc();
      g.A = Aq; g.B = R0; g.C = Gbar + (size_t)t0 * nk * n2;
      g.M = nao; g.N = nao; g.K = naux * nao; g.batch = tcur * nk;
      g.am = aff(1); g.ak = two(nao, nao, n2); g.conjA = 1;
      g.bk = two(nao, nao, (long long)nk * n2); g.bn = aff(1);
      g.cm = aff(nao); g.cn = aff(1);
      g.ba = two(nk, sv, 0); g.bb = two(nk, n2, S); g.bc = two(nk, 0, (long long)nk * n2);
      g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsC = n2;
      g.alpha_r = sc; g.beta_zero = 0; g.beta_r = 1.0;
      g.ta = g.tb = t; g.tc = 0; g.f32 = t; g.kchunk = vm.kchunk;
      g.tag = KC_SE_FINAL;
      if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * nk * n2})) != GW_OK) return s;
      // --- mirrored slot: Gbar[nt-1-t][k] += sc sum_{Q',b} V[q][k][Q'][c][b] T[Q'][k][d][b]
      // R1 = X[tl][k][Q][d][b] = sum_a V[q][k][Q][d][a] G[t][k+q][a][b]
      g = gemm_desc();
      g.A = Aq; g.B = G + (size_t)t0 * nk * n2; g.C = R1;
      g.M = naux * nao; g.N = tcur * nao; g.K = nao; g.batch = nk;
      g.am = aff(nao); g.ak = aff(1); g.bk = aff(nao); g.bn = two(nao, 1, (long long)nk * n2);
      g.cm = aff(nao); g.cn = two(nao, 1, S);
      g.ba = aff(sv); g.bb = aff(0); g.bc = aff(sv);
      g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsB = n2;
      g.ta = g.tc = t; g.tb = 0; g.f32 = t;
      g.tag = KC_POL_PRODUCER;
      if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * nk * n2}, Ext{0, (long long)tc * S})) != GW_OK) return s;
      // R0 = T[tl][Q'][k][e] = sum_Q Pbar[Q][Q'] conj(X[tl][k][Q][e])
      g = gemm_desc();
      g.A = Pb; g.B = R1; g.C = R0;
      g.M = naux; g.N = nk * (int)n2; g.K = naux; g.batch = tcur;
      g.am = aff(1); g.ak = aff(naux); g.bk = aff(n2); g.bn = two((unsigned)n2, 1, sv); g.conjB = 1;
      g.cm = aff((long long)nk * n2); g.cn = aff(1);
      g.ba = aff((long long)naux * naux); g.bb = aff(S); g.bc = aff(S);
      g.ta = 0; g.tb = g.tc = t; g.f32 = t;
      g.tag = KC_SE_CONTRACT;
      if ((s = run(c, g, Ext{0, (long long)tcur * naux * naux}, Ext{0, (long long)tcur * S}, Ext{0, (long long)tcur * S})) != GW_OK) return s;
      // Gbar[nt-1-t0-tl][k][c][d] += sc sum_{Q',b} V[q][k][Q'][c][b] T[tl][Q'][k][d][b]
      g = gemm_desc();
      g.A = Aq; g.B = R0; g.C = Gbar + (size_t)(nt - 1 - t0) * nk * n2;
      g.M = nao; g.N = nao; g.K = naux * nao; g.batch = tcur * nk;
      g.am = aff(nao); g.ak = two(nao, 1, n2);
      g.bk = two(nao, 1, (long long)nk * n2); g.bn = aff(nao);
      g.cm = aff(nao); g.cn = aff(1);
      g.ba = two(nk, sv, 0); g.bb = two(nk, n2, S); g.bc = two(nk, n2, -(long long)nk * n2);
      g.alpha_r = sc; g.beta_zero = 0; g.beta_r = 1.0;
      g.ta = g.tb = t; g.tc = 0; g.f32 = t; g.kchunk = vm.kchunk;
      g.tag = KC_SE_FINAL;
      if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)tcur * S}, Ext{-(long long)(tcur - 1) * nk * n2, (long long)nk * n2})) != GW_OK) return s;
    }
  }
  return GW_OK;
}

gw_status gw_hf_vjp(gw_ctx* c, const void* V, const gw_z* Sbar, gw_z* Gbar) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (!V || !Sbar || !Gbar) return fail(c, GW_ERR_ARG, "NULL array");
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_HF, 1))
    return fail(c, GW_ERR_WORKSPACE, "HF workspace too small");
  const int nk = c->nk, nao = c->d.nao, naux = c->d.naux, nt = c->d.ntau;
  const long long n2 = c->n2, sv = c->sv;
  // complex64 V is read in fp64 arithmetic, as in gw_hf
  const int tv = lowp(c) ? 1 : 0;
  const size_t ez = tv ? 8 : 16;
  const char* Vd = (const char*)V;
  double2* T2 = (double2*)c->ws;
  double2* gb = (double2*)((char*)c->ws + align256((size_t)nk * sv * 16));
  double2* vb = (double2*)((char*)gb + align256((size_t)nk * n2 * 16));
  // vbar[Q] = sum_{k,e} conj(V[0][k][Q][e]) Sbar[k][e]
  GemmDesc g = gemm_desc();
  g.A = Vd; g.B = Sbar; g.C = vb;
  g.M = naux; g.N = 1; g.K = nk * (int)n2;
  g.am = aff(n2); g.ak = two((unsigned)n2, 1, sv); g.conjA = 1;
  g.bk = aff(1); g.bn = aff(0); g.cm = aff(1); g.cn = aff(0);
  g.ta = tv;
  g.tag = KC_HF;
  if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2}, Ext{0, (long long)naux})) != GW_OK) return s;
  // gbar[k'][a][b] = (ns/nk) sum_Q conj(V[0][k'][Q][b][a]) vbar[Q]
  g = gemm_desc();
  g.A = vb; g.B = Vd; g.C = gb;
  g.M = 1; g.N = nk * (int)n2; g.K = naux;
  g.am = aff(0); g.ak = aff(1);
  g.bk = aff(n2); g.bn = three(nao, nao, nao, 1, sv); g.conjB = 1;
  g.cm = aff(0); g.cn = aff(1);
  g.alpha_r = (double)c->d.ns / nk;
  g.tb = tv;
  g.tag = KC_HF;
  if ((s = run(c, g, Ext{0, (long long)naux}, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2})) != GW_OK) return s;
  for (int q = 0; q < nk; ++q) {
    const char* Aq = Vd + (size_t)q * nk * sv * ez;
    // T2[k][Q][b][i] = sum_j V[q][k][Q][j][b] Sbar[k][i][j]
    g = gemm_desc();
    g.A = Aq; g.B = Sbar; g.C = T2;
    g.M = naux * nao; g.N = nao; g.K = nao; g.batch = nk;
    g.am = two(nao, 1, n2); g.ak = aff(nao); g.bk = aff(1); g.bn = aff(nao);
    g.cm = aff(nao); g.cn = aff(1);
    g.ba = aff(sv); g.bb = aff(n2); g.bc = aff(sv);
    g.ta = tv;
    g.tag = KC_HF;
    if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2}, Ext{0, (long long)nk * sv})) != GW_OK) return s;
    // gbar[k+q][a][b] += -(1/nk) sum_{Q,i} conj(V[q][k][Q][i][a]) T2[k][Q][b][i]
    g = gemm_desc();
    g.A = Aq; g.B = T2; g.C = gb;
    g.M = nao; g.N = nao; g.K = naux * nao; g.batch = nk;
    g.am = aff(1); g.ak = two(nao, nao, n2); g.conjA = 1;
    g.bk = two(nao, 1, n2); g.bn = aff(nao);
    g.cm = aff(nao); g.cn = aff(1);
    g.ba = aff(sv); g.bb = aff(sv); g.bc = aff(0);
    g.tab = c->dplus + (size_t)q * nk; g.tmod = nk; g.tsC = n2;
    g.alpha_r = -1.0 / nk; g.beta_zero = 0; g.beta_r = 1.0;
    g.ta = tv;
    g.tag = KC_HF;
    if ((s = run(c, g, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * sv}, Ext{0, (long long)nk * n2})) != GW_OK) return s;
  }
  // Gbar[t] += -w_t gbar   (gamma = -sum_t w_t G(t), w real)
  g = gemm_desc();
  g.A = c->dw; g.B = gb; g.C = Gbar;
  g.M = nt; g.N = nk * (int)n2; g.K = 1;
  g.am = aff(1); g.ak = aff(0); g.bk = aff(0); g.bn = aff(1);
  g.cm = aff((long long)nk * n2); g.cn = aff(1);
  g.alpha_r = -1.0; g.beta_zero = 0; g.beta_r = 1.0;
  g.tag = KC_HF;
  return run(c, g, Ext{0, (long long)nt}, Ext{0, (long long)nk * n2}, Ext{0, (long long)nt * nk * n2});
}


// ---------------------------------------------------------------- vectors
gw_status gw_axpby(gw_ctx* c, long long n, double ar, double ai, const gw_z* X, double br, double bi,
                   gw_z* Y) {
  if (!c) return GW_ERR_ARG;
  if (n < 0 || !Y) return fail(c, GW_ERR_ARG, "bad gw_axpby arguments");
  HIPCHK(c, axpby_launch(n, ar, ai, (const double2*)X, br, bi, (double2*)Y, c->st));
  return GW_OK;
}

gw_status gw_dot(gw_ctx* c, long long n, const gw_z* X, const gw_z* Y, double* out) {
  if (!c) return GW_ERR_ARG;
  if (n < 0 || !X || !Y || !out) return fail(c, GW_ERR_ARG, "bad gw_dot arguments");
  if (n == 0) {
    out[0] = out[1] = 0.0;
    return GW_OK;
  }
  const int nblk = (int)std::min<long long>((n + 255) / 256, 1024);
  HIPCHK(c, dot_launch(n, (const double2*)X, (const double2*)Y, c->dred, nblk, c->dred + 2 * 1024,
                       c->st));
  HIPCHK(c, hipMemcpyAsync(out, c->dred + 2 * 1024, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return GW_OK;
}

gw_status gw_hermitize(gw_ctx* c, gw_z* X, int n, long long nmat) {
  if (!c) return GW_ERR_ARG;
  if (n < 1 || n > 8192 || nmat < 0 || nmat > 65535) return fail(c, GW_ERR_ARG, "bad gw_hermitize sizes");
  if (nmat == 0) return GW_OK;
  if (!X) return fail(c, GW_ERR_ARG, "NULL array");
  HIPCHK(c, herm_avg_launch((double2*)X, n, nmat, c->st));
  return GW_OK;
}

// ------------------------------------------------- finite-size corrections
gw_status gw_finite_size(gw_ctx* c, const gw_z* S, double chi, const gw_z* gamma, gw_z* Sig_inf,
                         const gw_z* G_tau, const double* head, gw_z* Sig_tau) {
  if (!c) return GW_ERR_ARG;
  const int nao = c->d.nao, nk = c->nk, nt = c->d.ntau;
  if (nao > 64) return fail(c, GW_ERR_ARG, "gw_finite_size needs nao <= 64");
  if (!std::isfinite(chi)) return fail(c, GW_ERR_ARG, "chi is not finite");
  if (!S) return fail(c, GW_ERR_ARG, "NULL S");
  if (!gamma != !Sig_inf) return fail(c, GW_ERR_ARG, "gamma and Sig_inf go together");
  if (!G_tau != !Sig_tau || (G_tau && !head))
    return fail(c, GW_ERR_ARG, "G_tau, head and Sig_tau go together");
  if (head)
    for (int i = 0; i < nt; ++i)
      if (!std::isfinite(head[i])) return fail(c, GW_ERR_ARG, "head is not finite");
  if (gamma)
    HIPCHK(c, sxs_add_launch((const double2*)S, (const double2*)gamma, (double2*)Sig_inf, nao, nk, nk,
                             -chi, c->st));
  if (G_tau) {
    // Sigma~(tau_i) += -chi head_i S G(tau_i) S: one launch per tau node
    const size_t slab = (size_t)nk * c->n2;
    for (int i = 0; i < nt; ++i) {
      if (head[i] == 0.0) continue;
      HIPCHK(c, sxs_add_launch((const double2*)S, (const double2*)G_tau + i * slab,
                               (double2*)Sig_tau + i * slab, nao, nk, nk, -chi * head[i], c->st));
    }
  }
  return GW_OK;
}

// ---------------------------------------------------------------- Dyson JVP
gw_status gw_dyson_jvp(gw_ctx* c, const gw_z* S, const gw_z* G_iw, const gw_z* dSinf,
                       const gw_z* dSig_iw, int fixed_mu, gw_z* dG_iw, double* dmu) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (!S || !G_iw || !dG_iw) return fail(c, GW_ERR_ARG, "NULL array");
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_DYSON_JVP, 1))
    return fail(c, GW_ERR_WORKSPACE, "dyson_jvp workspace too small");
  const int nk = c->nk, nao = c->d.nao, nw = c->d.nw_f;
  const long long n2 = c->n2, tot = (long long)nw * nk * n2;
  double2* T = (double2*)c->ws;
  double2* P2 = (double2*)((char*)c->ws + align256((size_t)tot * 16));
  const int nb = nw * nk;
  // one product X Y over all (n, k); Y's batch offset is given by its map
  auto prod = [&](const void* A, Map3 ba, const void* B, Map3 bb, void* C, bool acc) -> gw_status {
    GemmDesc g = gemm_desc();
    g.A = A; g.B = B; g.C = C;
    g.M = nao; g.N = nao; g.K = nao; g.batch = nb;
    g.am = aff(nao); g.ak = aff(1); g.bk = aff(nao); g.bn = aff(1);
    g.cm = aff(nao); g.cn = aff(1);
    g.ba = ba; g.bb = bb; g.bc = aff(n2);
    if (acc) { g.beta_zero = 0; g.beta_r = 1.0; }
    g.tag = KC_OTHER;
    const long long eb = bb.sin == n2 ? tot : (long long)nk * n2;
    return run(c, g, Ext{0, tot}, Ext{0, eb}, Ext{0, tot});
  };
  const Map3 per_nk = aff(n2);                  // batch b = n*nk + k -> b * n2
  const Map3 per_k = two(nk, n2, 0);            // -> k * n2
  // dG = G (dSinf + dSig(i w)) G - dmu G S G  (Eq. Dyson differentiated)
  bool have = false;
  if (dSig_iw) {
    if ((s = prod(G_iw, per_nk, dSig_iw, per_nk, T, false)) != GW_OK) return s;
    have = true;
  }
  if (dSinf) {
    if ((s = prod(G_iw, per_nk, dSinf, per_k, T, have)) != GW_OK) return s;
    have = true;
  }
  if (!have) HIPCHK(c, axpby_launch(tot, 0.0, 0.0, nullptr, 0.0, 0.0, T, c->st));
  if ((s = prod(T, per_nk, G_iw, per_nk, dG_iw, false)) != GW_OK) return s;
  double m = 0.0;
  if (!fixed_mu) {
    // dmu keeps N_e = -(ns/Nk) sum Re(r_n tr[G S]) fixed:
    // dmu = sum Re(r_n tr[G dSig G S]) / sum Re(r_n tr[G S G S])
    if ((s = prod(G_iw, per_nk, S, per_k, T, false)) != GW_OK) return s;
    if ((s = prod(T, per_nk, G_iw, per_nk, P2, false)) != GW_OK) return s;
    double t1 = 0.0, t2 = 0.0;
    HIPCHK(c, wtrace_launch((const double2*)dG_iw, (const double2*)S, c->drrow, nao, nk, nw, c->dpart, c->st));
    HIPCHK(c, sum_launch(c->dpart, nb, 1.0, c->dpart + nb, c->st));
    HIPCHK(c, hipMemcpyAsync(&t1, c->dpart + nb, sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    HIPCHK(c, wtrace_launch(P2, (const double2*)S, c->drrow, nao, nk, nw, c->dpart, c->st));
    HIPCHK(c, sum_launch(c->dpart, nb, 1.0, c->dpart + nb, c->st));
    HIPCHK(c, hipMemcpyAsync(&t2, c->dpart + nb, sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (!(t2 != 0.0)) return fail(c, GW_ERR_SINGULAR, "dyson_jvp: dN/dmu is zero");
    m = t1 / t2;
    HIPCHK(c, axpby_launch(tot, -m, 0.0, P2, 1.0, 0.0, (double2*)dG_iw, c->st));
  }
  if (dmu) *dmu = m;
  return GW_OK;
}

// =========================================================================
// Whole-chain calls: one Sigma[G] + Pi evaluation and its JVP / VJP, the
// composition of the calls above (Sec. III, Algorithm 1).
// =========================================================================

// Per-q buffers at the end of the workspace (the front is left to the
// sub-calls): two tau arrays and four frequency arrays of naux^2 numbers.
struct PerQ {
  gw_z *ta, *tb, *w0, *w1, *w2, *w3;
};

static gw_status perq_bufs(gw_ctx* c, PerQ& p) {
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_SIGMA, c->tc))
    return fail(c, GW_ERR_WORKSPACE, "workspace too small for the whole-chain calls (GW_OP_SIGMA)");
  char* b = (char*)c->ws + ((c->ws_bytes - perq_bytes(c)) & ~size_t(255));
  const size_t tb = perq_tau_bytes(c), wb = perq_w_bytes(c);
  p.ta = (gw_z*)b;
  p.tb = (gw_z*)(b + tb);
  p.w0 = (gw_z*)(b + 2 * tb);
  p.w1 = (gw_z*)(b + 2 * tb + wb);
  p.w2 = (gw_z*)(b + 2 * tb + 2 * wb);
  p.w3 = (gw_z*)(b + 2 * tb + 3 * wb);
  return GW_OK;
}

static gw_status zero_z(gw_ctx* c, gw_z* Y, long long n) {
  HIPCHK(c, axpby_launch(n, 0.0, 0.0, nullptr, 0.0, 0.0, (double2*)Y, c->st));
  return GW_OK;
}

// P~^q of G rebuilt for one q: P0^q(tau) -> P0^q(i Omega) (p.w0) ->
// P~^q(i Omega) (p.w1) -> P~^q(tau) (p.ta).  phi (may be NULL) accumulates
// this q's Phi~ term.
static gw_status pt_one_q(gw_ctx* c, const void* V, const gw_z* G, int q, const PerQ& p, double* phi) {
  gw_status s;
  if ((s = pol_impl(c, ctx_work(c), V, G, G, q, 1, p.ta, false, false)) != GW_OK) return s;
  if ((s = gw_tau_to_iw(c, GW_BOSON, p.ta, 1, (long long)c->d.naux * c->d.naux, p.w0)) != GW_OK) return s;
  if (phi) {
    double f = 0.0;
    if ((s = gw_screened_W_phi(c, p.w0, 1, p.w1, &f)) != GW_OK) return s;
    *phi += f;
  } else if ((s = gw_screened_W(c, p.w0, 1, p.w1)) != GW_OK) {
    return s;
  }
  return gw_iw_to_tau(c, GW_BOSON, p.w1, 1, (long long)c->d.naux * c->d.naux, p.ta);
}

gw_status gw_sigma(gw_ctx* c, const void* V, const gw_z* G, gw_z* gamma, gw_z* Sinf, gw_z* Stau,
                   gw_z* P_tau, gw_z* P0_iw, gw_z* Pt_iw, double* phi) {
  if (!c) return GW_ERR_ARG;
  if (!ready(c)) return fail(c, GW_ERR_STATE, "grids not built (gw_build_grids or gw_set_grids)");
  if (!V || !G || !Sinf || !Stau) return fail(c, GW_ERR_ARG, "NULL array");
  const bool stored = P_tau || P0_iw || Pt_iw;
  if (stored && !(P_tau && P0_iw && Pt_iw))
    return fail(c, GW_ERR_ARG, "P_tau, P0_iw and Pt_iw are given all together or not at all");
  if (phi) *phi = 0.0;
  const int nk = c->nk, naux = c->d.naux;
  const long long nn = (long long)naux * naux;
  PerQ p{};
  gw_status s;
  if (!stored && (s = perq_bufs(c, p)) != GW_OK) return s;
  if ((s = gw_hf(c, V, G, gamma, Sinf)) != GW_OK) return s;
  if ((s = zero_z(c, Stau, (long long)c->d.ntau * nk * c->n2)) != GW_OK) return s;
  double ph = 0.0;
  if (stored) {
    if ((s = pol_impl(c, ctx_work(c), V, G, G, 0, nk, P_tau, false, false)) != GW_OK) return s;
    if ((s = gw_tau_to_iw(c, GW_BOSON, P_tau, nk, nn, P0_iw)) != GW_OK) return s;
    // screened-interaction solves in q-batches as large as the workspace holds
    const size_t per = screened_bytes(c, 1);
    const int qb = (int)std::max<size_t>(1, std::min<size_t>((size_t)nk, c->ws_bytes / per));
    for (int q0 = 0; q0 < nk; q0 += qb) {
      const int nq = std::min(qb, nk - q0);
      const size_t off = (size_t)q0 * c->d.nw_b * nn;
      if (phi) {
        double f = 0.0;
        if ((s = gw_screened_W_phi(c, P0_iw + off, nq, Pt_iw + off, &f)) != GW_OK) return s;
        ph += f;
      } else if ((s = gw_screened_W(c, P0_iw + off, nq, Pt_iw + off)) != GW_OK) {
        return s;
      }
    }
    if ((s = gw_iw_to_tau(c, GW_BOSON, Pt_iw, nk, nn, P_tau)) != GW_OK) return s;
    if ((s = gw_self_energy(c, V, G, P_tau, 0, nk, Stau)) != GW_OK) return s;
  } else {
    for (int q = 0; q < nk; ++q) {
      if ((s = pt_one_q(c, V, G, q, p, phi ? &ph : nullptr)) != GW_OK) return s;
      if ((s = gw_self_energy(c, V, G, p.ta, q, 1, Stau)) != GW_OK) return s;
    }
  }
  if (phi) {
    HIPCHK(c, hipStreamSynchronize(c->st));
    *phi = ph;
  }
  return GW_OK;
}

// Shared checks of the derivative calls; sets *stored.
static gw_status deriv_args(gw_ctx* c, const void* V, const gw_z* G, const gw_z* Pt_tau,
                            const gw_z* Pt_iw, bool* stored) {
  if (!V || !G) return fail(c, GW_ERR_ARG, "NULL array");
  if (!Pt_tau != !Pt_iw) return fail(c, GW_ERR_ARG, "Pt_tau and Pt_iw are given together or not at all");
  *stored = Pt_tau != nullptr;
  return GW_OK;
}

gw_status gw_sigma_jvp(gw_ctx* c, const void* V, const gw_z* G, const gw_z* Pt_tau, const gw_z* Pt_iw,
                       const gw_z* dG, gw_z* dSinf, gw_z* dStau) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  bool stored = false;
  if ((s = deriv_args(c, V, G, Pt_tau, Pt_iw, &stored)) != GW_OK) return s;
  if (!dG || !dSinf || !dStau) return fail(c, GW_ERR_ARG, "NULL array");
  PerQ p{};
  if ((s = perq_bufs(c, p)) != GW_OK) return s;
  const int nk = c->nk, nt = c->d.ntau, nwb = c->d.nw_b;
  const long long nn = (long long)c->d.naux * c->d.naux;
  // dSigma_inf = HF[gamma(dG)] (linear in G)
  if ((s = gw_hf(c, V, dG, nullptr, dSinf)) != GW_OK) return s;
  if ((s = zero_z(c, dStau, (long long)nt * nk * c->n2)) != GW_OK) return s;
  for (int q = 0; q < nk; ++q) {
    const gw_z* pt = stored ? Pt_tau + (size_t)q * nt * nn : p.ta;
    const gw_z* pw = stored ? Pt_iw + (size_t)q * nwb * nn : p.w1;
    if (!stored && (s = pt_one_q(c, V, G, q, p, nullptr)) != GW_OK) return s;
    // dP0 = P0[dG, G] + P0[G, dG]
    if ((s = pol_impl(c, ctx_work(c), V, dG, G, q, 1, p.tb, false, true)) != GW_OK) return s;
    if ((s = pol_impl(c, ctx_work(c), V, G, dG, q, 1, p.tb, true, true)) != GW_OK) return s;
    // dP~(i Omega) = (I + P~) dP0(i Omega) (I + P~)
    if ((s = gw_tau_to_iw(c, GW_BOSON, p.tb, 1, nn, p.w2)) != GW_OK) return s;
    if ((s = gw_screened_W_lin(c, pw, p.w2, 1, 0, p.w3)) != GW_OK) return s;
    if ((s = gw_iw_to_tau(c, GW_BOSON, p.w3, 1, nn, p.tb)) != GW_OK) return s;
    // dSigma~ += Sigma~[dP~, G] + Sigma~[P~, dG]
    if ((s = gw_self_energy(c, V, G, p.tb, q, 1, dStau)) != GW_OK) return s;
    if ((s = gw_self_energy(c, V, dG, pt, q, 1, dStau)) != GW_OK) return s;
  }
  return GW_OK;
}

gw_status gw_sigma_vjp(gw_ctx* c, const void* V, const gw_z* G, const gw_z* Pt_tau, const gw_z* Pt_iw,
                       const gw_z* Sinf_bar, const gw_z* Stau_bar, gw_z* G_bar) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  bool stored = false;
  if ((s = deriv_args(c, V, G, Pt_tau, Pt_iw, &stored)) != GW_OK) return s;
  if (!Sinf_bar || !Stau_bar || !G_bar) return fail(c, GW_ERR_ARG, "NULL array");
  PerQ p{};
  if ((s = perq_bufs(c, p)) != GW_OK) return s;
  const int nk = c->nk, nt = c->d.ntau, nwb = c->d.nw_b;
  const long long nn = (long long)c->d.naux * c->d.naux;
  if ((s = zero_z(c, G_bar, (long long)nt * nk * c->n2)) != GW_OK) return s;
  for (int q = 0; q < nk; ++q) {
    const gw_z* pt = stored ? Pt_tau + (size_t)q * nt * nn : p.ta;
    const gw_z* pw = stored ? Pt_iw + (size_t)q * nwb * nn : p.w1;
    if (!stored && (s = pt_one_q(c, V, G, q, p, nullptr)) != GW_OK) return s;
    // Sigma~ = SE[P~, G]: G part into G_bar, P~ part into P_bar (p.tb)
    if ((s = gw_self_energy_vjp(c, V, G, pt, Stau_bar, q, 1, G_bar, p.tb)) != GW_OK) return s;
    // back through i Omega -> tau, the screened-interaction solve, tau -> i Omega
    if ((s = gw_transform_adjoint(c, GW_BOSON, 1, p.tb, 1, nn, p.w2)) != GW_OK) return s;
    if ((s = gw_screened_W_lin(c, pw, p.w2, 1, 1, p.w3)) != GW_OK) return s;
    if ((s = gw_transform_adjoint(c, GW_BOSON, 0, p.w3, 1, nn, p.tb)) != GW_OK) return s;
    // both G slots of the polarization
    if ((s = gw_polarization_vjp(c, V, G, p.tb, q, 1, G_bar)) != GW_OK) return s;
  }
  return gw_hf_vjp(c, V, Sinf_bar, G_bar);
}

// ------------------------------------------- thermodynamics (Sec. III.C) ---
// Eigenvalues of the Hermitian pencil (H, S), S positive definite: Cholesky
// S = L L^H, A = L^{-1} H L^{-H}, cyclic complex Jacobi rotations on A.
static bool pencil_eigenvalues(const gwgrid::cd* H, const gwgrid::cd* S, int n, double* ev) {
  using cd = gwgrid::cd;
  std::vector<cd> L((size_t)n * n, 0.0), A((size_t)n * n), X((size_t)n * n);
  for (int j = 0; j < n; ++j) {
    double d = S[(size_t)j * n + j].real();
    for (int p = 0; p < j; ++p) d -= std::norm(L[(size_t)j * n + p]);
    if (!(d > 0.0)) return false;
    L[(size_t)j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      cd v = S[(size_t)i * n + j];
      for (int p = 0; p < j; ++p) v -= L[(size_t)i * n + p] * std::conj(L[(size_t)j * n + p]);
      L[(size_t)i * n + j] = v / L[(size_t)j * n + j];
    }
  }
  // X = L^{-1} M for a square M (forward substitution per column)
  auto lsolve = [&](const std::vector<cd>& M, std::vector<cd>& out) {
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        cd v = M[(size_t)i * n + c];
        for (int p = 0; p < i; ++p) v -= L[(size_t)i * n + p] * out[(size_t)p * n + c];
        out[(size_t)i * n + c] = v / L[(size_t)i * n + i];
      }
  };
  std::vector<cd> Hm(H, H + (size_t)n * n), Y((size_t)n * n);
  lsolve(Hm, X);                                       // X = L^{-1} H
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Y[(size_t)i * n + j] = std::conj(X[(size_t)j * n + i]);
  lsolve(Y, A);                                        // A = L^{-1} X^H = (X L^{-H})^H
  for (int i = 0; i < n; ++i)                          // A is Hermitian: make it exactly so
    for (int j = i; j < n; ++j) {
      const cd v = 0.5 * (A[(size_t)i * n + j] + std::conj(A[(size_t)j * n + i]));
      A[(size_t)i * n + j] = v;
      A[(size_t)j * n + i] = std::conj(v);
    }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += std::norm(A[(size_t)i * n + j]);
        if (i != j) off += std::norm(A[(size_t)i * n + j]);
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd b = A[(size_t)p * n + q];
        const double ab = std::abs(b);
        if (ab == 0.0) continue;
        const cd ph = b / ab;                           // e^{i phi}
        const double a = A[(size_t)p * n + p].real(), d = A[(size_t)q * n + q].real();
        const double tau = (d - a) / (2.0 * ab);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < n; ++k) {                   // A <- A U
          const cd x = A[(size_t)k * n + p], y = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = c * x - sn * std::conj(ph) * y;
          A[(size_t)k * n + q] = sn * x + c * std::conj(ph) * y;
        }
        for (int k = 0; k < n; ++k) {                   // A <- U^H A
          const cd x = A[(size_t)p * n + k], y = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = c * x - sn * ph * y;
          A[(size_t)q * n + k] = sn * x + c * ph * y;
        }
      }
  }
  for (int i = 0; i < n; ++i) ev[i] = A[(size_t)i * n + i].real();
  return true;
}

gw_status gw_thermodynamics(gw_ctx* c, const gw_z* H0, const gw_z* S, const gw_z* Sinf, const gw_z* Siw,
                            double mu, double phi_tilde, gw_thermo* out) {
  gw_status s = need_grids(c);
  if (s != GW_OK) return s;
  if (!H0 || !S || !out) return fail(c, GW_ERR_ARG, "NULL array");
  if (!std::isfinite(mu) || !std::isfinite(phi_tilde)) return fail(c, GW_ERR_ARG, "mu or phi_tilde is not finite");
  if (!c->ws || c->ws_bytes < gw_workspace_bytes(c, GW_OP_THERMO, 1))
    return fail(c, GW_ERR_WORKSPACE, "thermodynamics workspace too small (GW_OP_THERMO)");
  const int nk = c->nk, nao = c->d.nao, nw = c->d.nw_f, ns = c->d.ns;
  const long long n2 = c->n2, nb = (long long)nw * nk;
  char* p = (char*)c->ws;
  double2* Giw = (double2*)p;                     // G(i w) [n][k][i][j]
  p += align256((size_t)nb * n2 * 16);
  double* ld = (double*)p;                        // ln|det M|
  p += align256((size_t)nb * 8);
  double* ldr = (double*)p;                       // ln|det M_ref|
  p += align256((size_t)nb * 8);
  double* tr = (double*)p;                        // per-(n, k) weighted traces
  p += align256((size_t)nb * 8);
  double2* gam = (double2*)p;                     // gamma [k][i][j]
  p += align256((size_t)nk * n2 * 16);
  double2* cw = (double2*)p;                      // (c_n, 0): c_n = -Re r_n
  p += align256((size_t)nw * 16);
  double* trk = (double*)p;                       // per-k traces
  // Dyson at mu with and without Sigma~ (log-determinants), G(i w) kept
  HIPCHK(c, zero_flag_launch(c->dflag, c->st));
  DysonArgs a{};
  a.H0 = (const double2*)H0; a.S = (const double2*)S; a.Sinf = (const double2*)Sinf;
  a.Siw = (const double2*)Siw; a.wF = c->dwF; a.rrow = c->drrow; a.mu = mu; a.nk = nk; a.nao = nao;
  a.flag = c->dflag; a.G = Giw; a.logdet = ld;
  HIPCHK(c, dyson_launch(a, nw, c->st));
  a.Siw = nullptr; a.G = nullptr; a.logdet = ldr;
  HIPCHK(c, dyson_launch(a, nw, c->st));
  if ((s = read_flag(c, "thermodynamics")) != GW_OK) return s;
  // gamma = -G(beta^-) = -sum_n r_n G(i w_n)
  GemmDesc g = gemm_desc();
  g.A = c->drrow; g.B = Giw; g.C = gam;
  g.M = 1; g.N = nk * (int)n2; g.K = nw;
  g.am = aff(0); g.ak = aff(1); g.bk = aff((long long)nk * n2); g.bn = aff(1);
  g.cm = aff(0); g.cn = aff(1);
  g.alpha_r = -1.0;
  g.tag = KC_OTHER;
  if ((s = run(c, g, Ext{0, (long long)nw}, Ext{0, nb * n2}, Ext{0, (long long)nk * n2})) != GW_OK) return s;
  // Matsubara-sum weights of decaying fermionic functions: c_n = -Re r_n
  std::vector<double2> cwh(nw);
  std::vector<double> cnh(nw);
  for (int n = 0; n < nw; ++n) {
    cnh[n] = -c->rrow[n].real();
    cwh[n] = double2{cnh[n], 0.0};
  }
  HIPCHK(c, hipMemcpyAsync(cw, cwh.data(), nw * sizeof(double2), hipMemcpyHostToDevice, c->st));
  if (Siw) HIPCHK(c, wtrace_launch((const double2*)Siw, Giw, cw, nao, nk, nw, tr, c->st, 1));
  // per-k traces tr[gamma X] for X = S, H0, Sigma_inf
  std::vector<double> t_s(nk), t_h(nk), t_x(nk, 0.0), t_dyn(nb, 0.0), lm(nb), lr(nb);
  HIPCHK(c, trace_launch(gam, (const double2*)S, nao, nk, trk, c->st));
  HIPCHK(c, hipMemcpyAsync(t_s.data(), trk, nk * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, trace_launch(gam, (const double2*)H0, nao, nk, trk + nk, c->st));
  HIPCHK(c, hipMemcpyAsync(t_h.data(), trk + nk, nk * sizeof(double), hipMemcpyDeviceToHost, c->st));
  if (Sinf) {
    HIPCHK(c, trace_launch(gam, (const double2*)Sinf, nao, nk, trk + 2 * nk, c->st));
    HIPCHK(c, hipMemcpyAsync(t_x.data(), trk + 2 * nk, nk * sizeof(double), hipMemcpyDeviceToHost, c->st));
  }
  if (Siw) HIPCHK(c, hipMemcpyAsync(t_dyn.data(), tr, nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(lm.data(), ld, nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(lr.data(), ldr, nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
  // the static pencil (H0 + Sigma_inf, S) on the host
  std::vector<gwgrid::cd> hh((size_t)nk * n2), ss((size_t)nk * n2), xx((size_t)nk * n2, 0.0);
  HIPCHK(c, hipMemcpyAsync(hh.data(), H0, hh.size() * 16, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(ss.data(), S, ss.size() * 16, hipMemcpyDeviceToHost, c->st));
  if (Sinf) HIPCHK(c, hipMemcpyAsync(xx.data(), Sinf, xx.size() * 16, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  const double beta = c->d.beta, pre = (double)ns / nk;
  double free_sum = 0.0;
  std::vector<double> ev(nao);
  for (int k = 0; k < nk; ++k) {
    std::vector<gwgrid::cd> hk(hh.begin() + (size_t)k * n2, hh.begin() + (size_t)(k + 1) * n2);
    for (long long e = 0; e < n2; ++e) hk[e] += xx[(size_t)k * n2 + e];
    if (!pencil_eigenvalues(hk.data(), &ss[(size_t)k * n2], nao, ev.data()))
      return fail(c, GW_ERR_ARG, "S is not positive definite");
    for (int i = 0; i < nao; ++i) {
      const double xi = ev[i] - mu;
      free_sum += std::max(-xi, 0.0) + std::log1p(std::exp(-beta * std::fabs(xi))) / beta;
    }
  }
  double ln_dyn = 0.0, sg_dyn = 0.0, ne = 0.0, e1 = 0.0, xs = 0.0;
  for (int n = 0; n < nw; ++n)
    for (int k = 0; k < nk; ++k) {
      const size_t i = (size_t)n * nk + k;
      ln_dyn += cnh[n] * (lm[i] - lr[i]);
      sg_dyn += t_dyn[i];
    }
  for (int k = 0; k < nk; ++k) {
    ne += t_s[k];
    e1 += t_h[k];
    xs += t_x[k];
  }
  gw_thermo o{};
  o.tr_ln = pre * (free_sum + ln_dyn);
  o.tr_sigma_g = pre * (xs + sg_dyn);
  o.phi_inf = 0.5 * pre * xs;
  o.phi_tilde = phi_tilde;
  o.omega = o.phi_inf + o.phi_tilde - o.tr_ln - o.tr_sigma_g;
  o.e_one_body = pre * e1;
  o.e_gm = o.e_one_body + 0.5 * o.tr_sigma_g;
  o.n_e = pre * ne;
  if (!std::isfinite(o.omega) || !std::isfinite(o.e_gm))
    return fail(c, GW_ERR_NONFINITE, "thermodynamics: non-finite result");
  *out = o;
  return GW_OK;
}

}  // extern "C"
