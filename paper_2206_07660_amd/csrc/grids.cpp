// Host-side discretisation of the imaginary-time and Matsubara axes.
//
// A function on [0, beta] is represented by its values at the tau nodes (the
// roots of T_ntau mapped to [0, beta]); between nodes it is the Lagrange
// interpolant.  The Fourier pair of the paper (Eqs. tau_to_iw / iw_to_tau and
// P0t_to_P0w / Piw_to_Pt) then becomes a pair of small dense matrices:
//   T[n][i] = int_0^beta L_i(tau) exp(i nu_n tau) d tau,
//   Tp      = least-squares inverse of T.
// L_i is evaluated in barycentric form; the integral uses Gauss-Legendre
// quadrature with enough points to resolve the oscillation; the least-squares
// inverse uses a complex Householder QR.  Nothing here touches the GPU.
#include "grids.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace gwgrid {

static const double kPi = 3.14159265358979323846;

void tau_nodes(double beta, int n, double* tau, double* x) {
  const int h = n / 2;
  for (int i = 0; i < n; ++i) x[i] = -std::cos((2.0 * i + 1.0) * kPi / (2.0 * n));
  for (int i = 0; i < h; ++i) x[n - 1 - i] = -x[i];           // exact mirror
  if (n % 2) x[h] = 0.0;
  for (int i = 0; i < n; ++i) tau[i] = 0.5 * beta * (1.0 + x[i]);
  for (int i = 0; i < h; ++i) tau[n - 1 - i] = beta - tau[i];
}

void gauss_legendre(int m, std::vector<double>& xs, std::vector<double>& ws) {
  // Newton iteration on P_m from the asymptotic guess; P_m and P_m' by the
  // three-term recurrence.
  xs.assign(m, 0.0);
  ws.assign(m, 0.0);
  for (int i = 0; i < (m + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (m + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= m; ++l) {
        double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      if (m == 1) { p1 = z; p0 = 1.0; }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16 * std::max(1.0, std::fabs(z))) {
        // one more evaluation of the derivative at the converged point
        p0 = 1.0; p1 = z;
        for (int l = 2; l <= m; ++l) {
          double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
          p0 = p1;
          p1 = p2;
        }
        dp = m * (z * p1 - p0) / (z * z - 1.0);
        break;
      }
    }
    double w = 2.0 / ((1.0 - z * z) * dp * dp);
    xs[i] = -z;
    xs[m - 1 - i] = z;
    ws[i] = w;
    ws[m - 1 - i] = w;
  }
  if (m % 2) xs[m / 2] = 0.0;
}

// Barycentric weights lambda_i = 1 / prod_{j != i} (x_i - x_j), each factor
// scaled by 2 (capacity of [-1, 1]) to keep the products in range.
static std::vector<double> bary_weights(const double* x, int n) {
  std::vector<double> lam(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (j != i) lam[i] /= 2.0 * (x[i] - x[j]);
  double mx = 0.0;
  for (double v : lam) mx = std::max(mx, std::fabs(v));
  for (double& v : lam) v /= mx;
  return lam;
}

// L[i] = L_i(y) for all i (second barycentric form; exact at nodes).
static void lagrange_at(const double* x, const std::vector<double>& lam, int n, double y,
                        double* L) {
  for (int i = 0; i < n; ++i)
    if (y == x[i]) {
      for (int j = 0; j < n; ++j) L[j] = (i == j) ? 1.0 : 0.0;
      return;
    }
  double den = 0.0;
  for (int i = 0; i < n; ++i) {
    L[i] = lam[i] / (y - x[i]);
    den += L[i];
  }
  for (int i = 0; i < n; ++i) L[i] /= den;
}

double matsubara(long long idx, double beta, int stat) {
  return stat == 0 ? (2.0 * idx + 1.0) * kPi / beta : 2.0 * idx * kPi / beta;
}

void transform(double beta, int ntau, const double* x, const double* nu, int nw, cd* T) {
  double numax = 0.0;
  for (int n = 0; n < nw; ++n) numax = std::max(numax, std::fabs(nu[n]));
  const int m = ntau + (int)std::ceil(beta * numax / 2.0) + 200;
  std::vector<double> xg, wg;
  gauss_legendre(m, xg, wg);
  std::vector<double> lam = bary_weights(x, ntau);
  std::vector<double> Lm((size_t)m * ntau);
  for (int g = 0; g < m; ++g) lagrange_at(x, lam, ntau, xg[g], &Lm[(size_t)g * ntau]);
  std::vector<cd> row(ntau);
  for (int n = 0; n < nw; ++n) {
    std::fill(row.begin(), row.end(), cd(0.0, 0.0));
    for (int g = 0; g < m; ++g) {
      const double t = 0.5 * beta * (1.0 + xg[g]);
      const cd ph = std::polar(wg[g] * 0.5 * beta, nu[n] * t);
      const double* L = &Lm[(size_t)g * ntau];
      for (int i = 0; i < ntau; ++i) row[i] += ph * L[i];
    }
    for (int i = 0; i < ntau; ++i) T[(size_t)n * ntau + i] = row[i];
  }
}

void beta_row(int ntau, const double* x, double* w) {
  std::vector<double> lam = bary_weights(x, ntau);
  lagrange_at(x, lam, ntau, 1.0, w);
}

// Least-squares inverse of a full-column-rank m x n matrix (m >= n) by
// Householder QR: A = Q R, Tp = R^{-1} Q^H (n x m).
int pinv_qr(const cd* A, int m, int n, cd* Tp) {
  if (m < n) return 1;
  std::vector<cd> R(A, A + (size_t)m * n);
  std::vector<cd> Qh((size_t)m * m, cd(0.0, 0.0));    // accumulates Q^H, starts at I
  for (int i = 0; i < m; ++i) Qh[(size_t)i * m + i] = 1.0;
  std::vector<cd> v(m);
  for (int j = 0; j < n; ++j) {
    double nrm = 0.0;
    for (int i = j; i < m; ++i) nrm += std::norm(R[(size_t)i * n + j]);
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return 2;
    cd a = R[(size_t)j * n + j];
    cd phase = (std::abs(a) > 0.0) ? a / std::abs(a) : cd(1.0, 0.0);
    // v = x + phase * ||x|| e_1 ; H = I - 2 v v^H / (v^H v)
    for (int i = 0; i < m; ++i) v[i] = 0.0;
    for (int i = j; i < m; ++i) v[i] = R[(size_t)i * n + j];
    v[j] += phase * nrm;
    double vv = 0.0;
    for (int i = j; i < m; ++i) vv += std::norm(v[i]);
    // apply to R columns j..n-1
    for (int c = j; c < n; ++c) {
      cd s = 0.0;
      for (int i = j; i < m; ++i) s += std::conj(v[i]) * R[(size_t)i * n + c];
      s *= 2.0 / vv;
      for (int i = j; i < m; ++i) R[(size_t)i * n + c] -= s * v[i];
    }
    // apply to Qh (all columns)
    for (int c = 0; c < m; ++c) {
      cd s = 0.0;
      for (int i = j; i < m; ++i) s += std::conj(v[i]) * Qh[(size_t)i * m + c];
      s *= 2.0 / vv;
      for (int i = j; i < m; ++i) Qh[(size_t)i * m + c] -= s * v[i];
    }
  }
  // back substitution R[0:n,0:n] X = Qh[0:n, :]
  for (int c = 0; c < m; ++c) {
    for (int i = n - 1; i >= 0; --i) {
      cd s = Qh[(size_t)i * m + c];
      for (int l = i + 1; l < n; ++l) s -= R[(size_t)i * n + l] * Tp[(size_t)l * m + c];
      cd d = R[(size_t)i * n + i];
      if (std::abs(d) == 0.0) return 3;
      Tp[(size_t)i * m + c] = s / d;
    }
  }
  return 0;
}

std::vector<long long> select_sparse(double beta, int ntau, int stat) {
  if (ntau % 2) throw std::invalid_argument("ntau must be even");
  std::vector<double> tau(ntau), x(ntau);
  tau_nodes(beta, ntau, tau.data(), x.data());
  const int nc = 4 * ntau;
  std::vector<double> nu(2 * nc);
  for (int c = 0; c < nc; ++c) {
    nu[2 * c] = matsubara(c, beta, stat);
    nu[2 * c + 1] = matsubara(stat == 0 ? -c - 1 : -c, beta, stat);
  }
  std::vector<cd> rows((size_t)2 * nc * ntau);
  transform(beta, ntau, x.data(), nu.data(), 2 * nc, rows.data());
  std::vector<double> norm2(2 * nc);
  for (int r = 0; r < 2 * nc; ++r) {
    double s = 0.0;
    for (int i = 0; i < ntau; ++i) s += std::norm(rows[(size_t)r * ntau + i]);
    norm2[r] = s;
  }
  std::vector<cd> basis;   // orthonormal rows, ntau each
  int nb = 0;
  auto project_out = [&](std::vector<cd>& r) {
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<cd> coef(nb);
      for (int b = 0; b < nb; ++b) {
        cd s = 0.0;
        for (int i = 0; i < ntau; ++i) s += std::conj(basis[(size_t)b * ntau + i]) * r[i];
        coef[b] = s;
      }
      for (int b = 0; b < nb; ++b)
        for (int i = 0; i < ntau; ++i) r[i] -= coef[b] * basis[(size_t)b * ntau + i];
    }
  };
  auto add = [&](int r) {
    std::vector<cd> v(rows.begin() + (size_t)r * ntau, rows.begin() + (size_t)(r + 1) * ntau);
    project_out(v);
    double s = 0.0;
    for (auto& z : v) s += std::norm(z);
    s = std::sqrt(s);
    for (auto& z : v) z /= s;
    basis.insert(basis.end(), v.begin(), v.end());
    ++nb;
  };
  std::vector<char> taken(nc, 0);
  std::vector<long long> chosen;
  if (stat == 1) {
    add(0);
    taken[0] = 1;
    chosen.push_back(0);
  }
  for (int p = 0; p < ntau / 2; ++p) {
    std::vector<double> res(nc, -1.0);
    double best = -1.0;
    for (int c = 0; c < nc; ++c) {
      if (taken[c]) continue;
      double tot = 0.0;
      for (int s = 0; s < 2; ++s) {
        const int r = 2 * c + s;
        std::vector<cd> v(rows.begin() + (size_t)r * ntau, rows.begin() + (size_t)(r + 1) * ntau);
        if (nb) {
          // single classical projection, as a residual estimate
          std::vector<cd> coef(nb);
          for (int b = 0; b < nb; ++b) {
            cd z = 0.0;
            for (int i = 0; i < ntau; ++i) z += std::conj(basis[(size_t)b * ntau + i]) * v[i];
            coef[b] = z;
          }
          for (int b = 0; b < nb; ++b)
            for (int i = 0; i < ntau; ++i) v[i] -= coef[b] * basis[(size_t)b * ntau + i];
        }
        double e = 0.0;
        for (auto& z : v) e += std::norm(z);
        tot += e / norm2[r];
      }
      res[c] = tot;
      best = std::max(best, tot);
    }
    int pick = -1;
    for (int c = 0; c < nc; ++c)
      if (!taken[c] && res[c] >= best * (1.0 - 1e-9)) { pick = c; break; }
    taken[pick] = 1;
    chosen.push_back(pick);
    add(2 * pick);
    add(2 * pick + 1);
  }
  std::vector<long long> pos;
  for (long long c : chosen)
    if (c > 0 || stat == 0) pos.push_back(c);
  std::sort(pos.begin(), pos.end());
  std::vector<long long> out;
  for (int i = (int)pos.size() - 1; i >= 0; --i) out.push_back(stat == 0 ? -pos[i] - 1 : -pos[i]);
  if (stat == 1) out.push_back(0);
  for (long long c : pos) out.push_back(c);
  return out;
}

}  // namespace gwgrid
