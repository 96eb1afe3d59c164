// Intermediate-representation (IR) grids with sparse sampling on both
// imaginary axes (Sec. IV.C of the paper: dynamical quantities are expanded
// in the IR basis, whose dimensionless cutoff lambda exceeds beta times the
// bandwidth, and sampled sparsely in tau and in Matsubara frequency).
//
// The basis is the singular-value expansion of the logistic kernel
//   K(x, y) = exp(-lambda y (x + 1) / 2) / (1 + exp(-lambda y)),
// x = 2 tau / beta - 1, y = omega / omega_max, lambda = beta omega_max, i.e.
// e^{-omega tau} / (1 + e^{-beta omega}); one basis serves fermionic and
// bosonic functions (a bosonic spectral function enters times
// coth(beta omega / 2)).  Steps:
//  1. K sampled on composite Gauss-Legendre rules (segments halving towards
//     x = +-1 and towards y = 0) and weighted, A = sqrt(wx) K sqrt(wy);
//  2. A = Q R P^T by Householder QR with column pivoting, truncated at the
//     numerical rank, then the SVD of R by one-sided (Hestenes) Jacobi
//     rotations of the columns of R^T: singular values s_l and right
//     singular vectors v_l;
//  3. L = number of s_l above eps s_0, rounded up to even; basis functions
//     by the Nystrom extension u_l(x) = (1 / s_l) sum_j K(x, y_j) sqrt(wy_j)
//     v_{jl}, whose Matsubara transforms are closed forms: -1 / (i nu - omega)
//     per kernel column (fermionic nu), -tanh(beta omega / 2) / (i nu - omega)
//     (bosonic nu);
//  4. tau points: the L roots of u_L (sign changes on a fine composite grid
//     and bisection), mirrored in pairs;
//  5. Matsubara points: symmetric pairs chosen greedily by the largest
//     residual of their transform rows (columns scaled to unit norm over the
//     candidates |n| < 4 lambda / pi + 4 L), L fermionic and L + 1 bosonic;
//  6. tables T = Uhat U(tau)^{-1}, Tp = U(tau) Uhat^+, w = u(1) U(tau)^{-1}.
#include "ir.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>

namespace gwir {
namespace {

using gwgrid::cd;

double kernel(double x, double y, double lam) {
  const double e = y >= 0.0 ? -0.5 * lam * y * (x + 1.0) : 0.5 * lam * y * (1.0 - x);
  return std::exp(e) / (1.0 + std::exp(-lam * std::fabs(y)));
}

void segments(double lam, std::vector<double>& bx, std::vector<double>& by) {
  const int m = (int)std::ceil(std::log2(lam)) + 2;
  std::vector<double> px{0.0, 1.0}, py{0.0};
  for (int j = 1; j < m; ++j) px.push_back(1.0 - std::ldexp(1.0, -j));
  for (int j = 0; j < m; ++j) py.push_back(std::ldexp(1.0, -j));
  auto mirror = [](std::vector<double> p) {
    std::vector<double> out;
    for (double v : p) {
      out.push_back(v);
      if (v > 0.0) out.push_back(-v);
    }
    std::sort(out.begin(), out.end());
    out.erase(std::unique(out.begin(), out.end()), out.end());
    return out;
  };
  bx = mirror(px);
  by = mirror(py);
}

void composite(const std::vector<double>& br, int npts, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> t, tw;
  gwgrid::gauss_legendre(npts, t, tw);
  x.clear();
  w.clear();
  for (size_t s = 0; s + 1 < br.size(); ++s) {
    const double a = br[s], b = br[s + 1];
    for (int i = 0; i < npts; ++i) {
      x.push_back(0.5 * (b - a) * t[i] + 0.5 * (b + a));
      w.push_back(0.5 * (b - a) * tw[i]);
    }
  }
}

// Right singular vectors and singular values of the m x n row-major A, for
// the singular values above 1e-15 s_0: pivoted Householder QR, then one-sided
// Jacobi on the columns of R^T.  s sorted descending; V column-major (n x r).
void svd_right(std::vector<double> A, int m, int n, std::vector<double>& s, std::vector<double>& V) {
  std::vector<int> perm(n);
  for (int j = 0; j < n; ++j) perm[j] = j;
  std::vector<double> cn(n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) cn[j] += A[(size_t)i * n + j] * A[(size_t)i * n + j];
  const int kmax = std::min(m, n);
  int r = 0;
  double r00 = 0.0;
  for (int k = 0; k < kmax; ++k) {
    // pivot: largest remaining column norm (recomputed to avoid drift)
    int p = k;
    double best = -1.0;
    for (int j = k; j < n; ++j) {
      double t = 0.0;
      for (int i = k; i < m; ++i) t += A[(size_t)i * n + j] * A[(size_t)i * n + j];
      cn[j] = t;
      if (t > best) { best = t; p = j; }
    }
    if (p != k) {
      for (int i = 0; i < m; ++i) std::swap(A[(size_t)i * n + k], A[(size_t)i * n + p]);
      std::swap(perm[k], perm[p]);
    }
    const double norm = std::sqrt(best);
    if (k == 0) r00 = norm;
    if (!(norm > 1e-15 * r00)) break;
    // Householder reflector zeroing A[k+1:, k]
    const double a0 = A[(size_t)k * n + k];
    const double alpha = a0 >= 0.0 ? -norm : norm;
    std::vector<double> v(m - k);
    v[0] = a0 - alpha;
    for (int i = k + 1; i < m; ++i) v[i - k] = A[(size_t)i * n + k];
    double vn = 0.0;
    for (double t : v) vn += t * t;
    if (vn > 0.0)
      for (int j = k; j < n; ++j) {
        double d = 0.0;
        for (int i = k; i < m; ++i) d += v[i - k] * A[(size_t)i * n + j];
        const double f = 2.0 * d / vn;
        for (int i = k; i < m; ++i) A[(size_t)i * n + j] -= f * v[i - k];
      }
    r = k + 1;
  }
  // M = R^T (n x r, column c = row c of R), columns rotated until orthogonal
  std::vector<double> M((size_t)n * r, 0.0);
  for (int c = 0; c < r; ++c)
    for (int j = c; j < n; ++j) M[(size_t)c * n + j] = A[(size_t)c * n + j];
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int i = 0; i < r; ++i)
      for (int j = i + 1; j < r; ++j) {
        double* mi = &M[(size_t)i * n];
        double* mj = &M[(size_t)j * n];
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int t = 0; t < n; ++t) {
          al += mi[t] * mi[t];
          be += mj[t] * mj[t];
          ga += mi[t] * mj[t];
        }
        if (!(std::fabs(ga) > 1e-15 * std::sqrt(al * be))) continue;
        rotated = true;
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + tt * tt), sn = c * tt;
        for (int t = 0; t < n; ++t) {
          const double a = mi[t], b = mj[t];
          mi[t] = c * a - sn * b;
          mj[t] = sn * a + c * b;
        }
      }
    if (!rotated) break;
  }
  std::vector<std::pair<double, int>> order(r);
  for (int c = 0; c < r; ++c) {
    double t = 0.0;
    for (int j = 0; j < n; ++j) t += M[(size_t)c * n + j] * M[(size_t)c * n + j];
    order[c] = {std::sqrt(t), c};
  }
  std::sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  s.assign(r, 0.0);
  V.assign((size_t)n * r, 0.0);
  for (int l = 0; l < r; ++l) {
    s[l] = order[l].first;
    const double* mc = &M[(size_t)order[l].second * n];
    for (int j = 0; j < n; ++j) V[(size_t)l * n + perm[j]] = mc[j] / s[l];   // undo the pivoting
  }
}

// Singular-value expansion of the kernel for one (lambda, eps).
struct Sve {
  double lam = 0.0, eps = 0.0;
  int L = 0;
  std::vector<double> bx, y;   // x breakpoints; y nodes
  std::vector<double> s;       // singular values
  std::vector<double> coef;    // Nystrom coefficients, (L + 1) columns of ny, column-major
};

Sve make_sve(double lam, double eps) {
  Sve b;
  b.lam = lam;
  b.eps = eps;
  std::vector<double> by, x, wx, wy;
  segments(lam, b.bx, by);
  composite(b.bx, 16, x, wx);
  composite(by, 16, b.y, wy);
  const int m = (int)x.size(), n = (int)b.y.size();
  std::vector<double> A((size_t)m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) A[(size_t)i * n + j] = std::sqrt(wx[i]) * kernel(x[i], b.y[j], lam) * std::sqrt(wy[j]);
  std::vector<double> V;
  svd_right(std::move(A), m, n, b.s, V);
  int L = 0;
  while (L < (int)b.s.size() && b.s[L] > eps * b.s[0]) ++L;
  L += L % 2;
  if (L + 1 > (int)b.s.size()) throw std::runtime_error("IR basis: eps below the attainable rank");
  b.L = L;
  b.coef.assign((size_t)(L + 1) * n, 0.0);
  for (int l = 0; l <= L; ++l)
    for (int j = 0; j < n; ++j) b.coef[(size_t)l * n + j] = std::sqrt(wy[j]) * V[(size_t)l * n + j] / b.s[l];
  return b;
}

const Sve& sve_cached(double lam, double eps) {
  static std::mutex mu;
  static std::map<std::pair<double, double>, Sve> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(lam, eps);
  auto it = cache.find(key);
  if (it == cache.end()) it = cache.emplace(key, make_sve(lam, eps)).first;
  return it->second;
}

// u_l(x) for l < nl
void ueval(const Sve& b, double x, int l0, int nl, double* out) {
  const int ny = (int)b.y.size();
  std::vector<double> k(ny);
  for (int j = 0; j < ny; ++j) k[j] = kernel(x, b.y[j], b.lam);
  for (int l = 0; l < nl; ++l) {
    const double* c = &b.coef[(size_t)(l0 + l) * ny];
    double t = 0.0;
    for (int j = 0; j < ny; ++j) t += k[j] * c[j];
    out[l] = t;
  }
}

double uL(const Sve& b, double x) {
  double v = 0.0;
  ueval(b, x, b.L, 1, &v);
  return v;
}

// Roots of u_L in (-1, 1), mirrored from the positive half.
std::vector<double> tau_roots(const Sve& b) {
  std::vector<double> g, gw;
  composite(b.bx, 64, g, gw);
  for (double v : b.bx) g.push_back(v);
  std::sort(g.begin(), g.end());
  std::vector<double> pts;
  for (double v : g)
    if (v > 0.0) pts.push_back(v);
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  std::vector<double> f(pts.size());
  for (size_t i = 0; i < pts.size(); ++i) f[i] = uL(b, pts[i]);
  std::vector<double> pos;
  for (size_t i = 0; i + 1 < pts.size(); ++i) {
    if (!((f[i] < 0.0 && f[i + 1] > 0.0) || (f[i] > 0.0 && f[i + 1] < 0.0))) continue;
    double a = pts[i], c = pts[i + 1], fa = f[i];
    for (int it = 0; it < 64; ++it) {
      const double mid = 0.5 * (a + c), fm = uL(b, mid);
      if ((fm < 0.0) == (fa < 0.0)) { a = mid; fa = fm; } else { c = mid; }
    }
    pos.push_back(0.5 * (a + c));
  }
  if ((int)(2 * pos.size()) != b.L) throw std::runtime_error("IR basis: u_L does not have L roots");
  std::vector<double> x;
  for (auto it = pos.rbegin(); it != pos.rend(); ++it) x.push_back(-*it);
  for (double v : pos) x.push_back(v);
  return x;
}

// Matsubara transforms of u_0 .. u_{L-1} at one frequency nu.
void uhat_row(const Sve& b, double beta, double nu, int stat, cd* row) {
  const int ny = (int)b.y.size();
  const double wmax = b.lam / beta;
  std::vector<cd> f(ny);
  for (int j = 0; j < ny; ++j) {
    const double om = b.y[j] * wmax;
    const cd z(-om, nu);
    f[j] = (stat == 0 ? -1.0 : -std::tanh(0.5 * beta * om)) / z;
  }
  for (int l = 0; l < b.L; ++l) {
    const double* c = &b.coef[(size_t)l * ny];
    cd t = 0.0;
    for (int j = 0; j < ny; ++j) t += f[j] * c[j];
    row[l] = t;
  }
}

std::vector<long long> select_matsubara(const Sve& b, double beta, int stat, int count) {
  const int L = b.L;
  const long long N = (long long)std::ceil(4.0 * b.lam / M_PI) + 4LL * L;
  const long long nc = 2 * N;                       // candidates -N .. N-1
  std::vector<cd> R((size_t)nc * L);
  for (long long i = 0; i < nc; ++i) {
    const long long n = i - N;
    uhat_row(b, beta, gwgrid::matsubara(n, beta, stat), stat, &R[(size_t)i * L]);
  }
  for (int l = 0; l < L; ++l) {
    double t = 0.0;
    for (long long i = 0; i < nc; ++i) t += std::norm(R[(size_t)i * L + l]);
    const double inv = 1.0 / std::sqrt(t);
    for (long long i = 0; i < nc; ++i) R[(size_t)i * L + l] *= inv;
  }
  auto row = [&](long long n) { return &R[(size_t)(n + N) * L]; };
  auto nrm2 = [&](long long n) {
    double t = 0.0;
    const cd* r = row(n);
    for (int l = 0; l < L; ++l) t += std::norm(r[l]);
    return t;
  };
  // groups: fermionic {n, -n-1}; bosonic {0} first, then {m, -m}
  std::vector<std::vector<long long>> groups;
  if (stat == 0)
    for (long long n = 0; n < N; ++n) groups.push_back({n, -n - 1});
  else {
    groups.push_back({0});
    for (long long m = 1; m < N; ++m) groups.push_back({m, -m});
  }
  std::vector<char> used(groups.size(), 0);
  std::vector<long long> chosen;
  std::vector<cd> q(L);
  while ((int)chosen.size() < count) {
    size_t best = 0;
    double bv = -1.0;
    for (size_t g = 0; g < groups.size(); ++g) {
      if (used[g]) continue;
      double t = 0.0;
      for (long long n : groups[g]) t += nrm2(n);
      if (t > bv) { bv = t; best = g; }
    }
    if (bv <= 0.0) throw std::runtime_error("IR Matsubara selection: no candidate left");
    used[best] = 1;
    for (long long n : groups[best]) {
      const cd* r = row(n);
      const double nr = std::sqrt(nrm2(n));
      for (int l = 0; l < L; ++l) q[l] = r[l] / nr;
      // project the new direction out of every candidate row
      for (long long i = 0; i < nc; ++i) {
        cd* x = &R[(size_t)i * L];
        cd d = 0.0;
        for (int l = 0; l < L; ++l) d += std::conj(q[l]) * x[l];
        for (int l = 0; l < L; ++l) x[l] -= d * q[l];
      }
      chosen.push_back(n);
    }
  }
  std::sort(chosen.begin(), chosen.end());
  return chosen;
}

// Inverse of the n x n real row-major matrix by Gauss-Jordan with partial pivoting.
std::vector<double> inverse(std::vector<double> a, int n) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[(size_t)r * n + c]) > std::fabs(a[(size_t)p * n + c])) p = r;
    if (!(std::fabs(a[(size_t)p * n + c]) > 0.0)) throw std::runtime_error("IR: singular sampling matrix");
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)p * n + j], a[(size_t)c * n + j]);
        std::swap(inv[(size_t)p * n + j], inv[(size_t)c * n + j]);
      }
    const double d = 1.0 / a[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      a[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    }
  }
  return inv;
}

}  // namespace

int ir_size(double lam, double eps) { return sve_cached(lam, eps).L; }

void ir_grids(double beta, double lam, double eps, IRTables& t) {
  const Sve& b = sve_cached(lam, eps);
  const int L = b.L;
  t.x = tau_roots(b);
  t.tau.resize(L);
  for (int i = 0; i < L; ++i) t.tau[i] = 0.5 * beta * (t.x[i] + 1.0);
  t.nF = select_matsubara(b, beta, 0, L);
  t.nB = select_matsubara(b, beta, 1, L + 1);
  std::vector<double> U((size_t)L * L);
  for (int i = 0; i < L; ++i) ueval(b, t.x[i], 0, L, &U[(size_t)i * L]);
  const std::vector<double> Ui = inverse(U, L);
  auto tables = [&](const std::vector<long long>& idx, int stat, std::vector<cd>& T, std::vector<cd>& Tp) {
    const int nw = (int)idx.size();
    std::vector<cd> Uh((size_t)nw * L);
    for (int r = 0; r < nw; ++r) uhat_row(b, beta, gwgrid::matsubara(idx[r], beta, stat), stat, &Uh[(size_t)r * L]);
    T.assign((size_t)nw * L, 0.0);
    for (int r = 0; r < nw; ++r)
      for (int k = 0; k < L; ++k) {
        const cd a = Uh[(size_t)r * L + k];
        for (int c = 0; c < L; ++c) T[(size_t)r * L + c] += a * Ui[(size_t)k * L + c];
      }
    std::vector<cd> P((size_t)L * nw);          // Uhat^+ (L x nw)
    if (gwgrid::pinv_qr(Uh.data(), nw, L, P.data())) throw std::runtime_error("IR: rank-deficient Matsubara sampling");
    Tp.assign((size_t)L * nw, 0.0);
    for (int i = 0; i < L; ++i)
      for (int k = 0; k < L; ++k) {
        const double a = U[(size_t)i * L + k];
        for (int c = 0; c < nw; ++c) Tp[(size_t)i * nw + c] += a * P[(size_t)k * nw + c];
      }
  };
  tables(t.nF, 0, t.TF, t.TFp);
  tables(t.nB, 1, t.TB, t.TBp);
  std::vector<double> u1(L);
  ueval(b, 1.0, 0, L, u1.data());
  t.w.assign(L, 0.0);
  for (int k = 0; k < L; ++k)
    for (int c = 0; c < L; ++c) t.w[c] += u1[k] * Ui[(size_t)k * L + c];
}

}  // namespace gwir
