// Host-side intermediate-representation grids (see ir.cpp).  Plain C++; no GPU code.
#pragma once
#include <vector>

#include "grids.h"

namespace gwir {

// Tables in the layout of the Chebyshev grids: ntau = L nodes, L fermionic
// and L + 1 bosonic Matsubara indices, T (nw x L), Tp (L x nw), density row w.
struct IRTables {
  std::vector<double> tau, x, w;
  std::vector<long long> nF, nB;
  std::vector<gwgrid::cd> TF, TFp, TB, TBp;
};

// Basis size L (even) for the cutoff lam and the singular-value threshold eps
// (cached per (lam, eps)); throws std::runtime_error on failure.
int ir_size(double lam, double eps);
// Sampling points and tables for beta; throws std::runtime_error on failure.
void ir_grids(double beta, double lam, double eps, IRTables& t);

}  // namespace gwir
