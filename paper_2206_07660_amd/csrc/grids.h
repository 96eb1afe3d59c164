// Host-side discretisation of the imaginary-time and Matsubara axes
// (see grids.cpp).  Plain C++; no GPU code.
#pragma once
#include <complex>
#include <vector>

namespace gwgrid {
using cd = std::complex<double>;

// Chebyshev-root nodes on [0, beta], ascending, mirrored: tau[n-1-i] = beta - tau[i].
// x[i] = 2 tau[i] / beta - 1.
void tau_nodes(double beta, int n, double* tau, double* x);
// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int m, std::vector<double>& xs, std::vector<double>& ws);
// nu of Matsubara index idx: stat 0 fermionic (2n+1) pi / beta, 1 bosonic 2 n pi / beta.
double matsubara(long long idx, double beta, int stat);
// T[n][i] = int_0^beta L_i(tau) exp(i nu_n tau) d tau (row-major nw x ntau).
void transform(double beta, int ntau, const double* x, const double* nu, int nw, cd* T);
// w[i] = L_i(tau = beta).
void beta_row(int ntau, const double* x, double* w);
// Least-squares inverse (n x m) of a full-column-rank m x n matrix; 0 on success.
int pinv_qr(const cd* A, int m, int n, cd* Tp);
// Greedy symmetric sparse Matsubara index set, sorted ascending
// (stat 0: ntau entries {n, -n-1}; stat 1: ntau + 1 entries {0, m, -m}).
std::vector<long long> select_sparse(double beta, int ntau, int stat);
}  // namespace gwgrid
