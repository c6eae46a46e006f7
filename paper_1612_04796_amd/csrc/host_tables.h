// Host-side set-up numerics of the p-multigrid hierarchy: GLL / GL rules, 1D SIPG
// blocks, restricted 1D eigenpairs, hat weights, interpolation and the level-0
// global eigenpairs.  Pure C++ (no HIP); used by the context set-up and by the
// host-only table queries of the C ABI.
#pragma once

#include <string>
#include <vector>

#include "sipg_mg.h"

namespace sipg {

constexpr int kMaxOrder = 32;  // orders 1..16 and 32

struct Dir1D {
  // one direction of one level
  int p = 0, n = 0, ne = 0;
  double h = 0, mu = 0;
  std::vector<double> xi, w;       // GLL or GL rule (n)
  std::vector<double> D;           // n x n, D[i*n+j] = phi_j'(xi_i)
  std::vector<double> mass;        // (h/2) w
  std::vector<double> Ld;          // element diagonal block of L (n x n)
  std::vector<double> U;           // coupling block L_{e,e+1} (n x n)
  std::vector<double> TL, TR;      // traces phi_j(-1), phi_j(+1) (unit vectors for GLL)
  std::vector<double> DLs, DRs;    // (1/h) phi_j'(-1), (1/h) phi_j'(+1)
  // subdomain (levels >= 1)
  int no = 0, m = 0;
  std::vector<double> Ls, Ms;      // m x m, m
  std::vector<double> lam, S;      // m, m x m (S[a*m+j]: node a, pair j)
  std::vector<double> wsub;        // m
  // The same eigenpairs split by the reversal symmetry a -> m-1-a of the
  // subdomain: the m - m/2 even eigenvectors first, then the m/2 odd ones,
  // each group ascending; columns exactly even / odd.
  std::vector<double> lam_eo, S_eo;  // m, m x m
};

struct LevelHost {
  int p = 0, n = 0;
  Dir1D dir[3];
  std::vector<double> J;           // n x n_prev (levels >= 1)
};

struct CoarseHost {
  int N[3] = {0, 0, 0};            // 2 ne_d
  std::vector<double> S[3];        // N x N, S[i*N+j]
  std::vector<double> lam[3];      // N, zero mode set to exactly 0
  int zero[3] = {0, 0, 0};         // index of the zero mode
};

struct HierarchyHost {
  sipg_params prm;
  std::vector<int> orders;
  std::vector<LevelHost> lev;
  CoarseHost coarse;
};

// Validates parameters; returns an empty string if valid, else the reason.
std::string validate(const sipg_params &p);

// Builds all host tables; throws std::runtime_error on failure.
void build_hierarchy(const sipg_params &p, HierarchyHost &H);

std::vector<int> level_orders(int P);

// Building blocks (exposed for the host-only table queries).
void gll_rule(int p, std::vector<double> &xi, std::vector<double> &w);
// Gauss-Legendre: the p + 1 zeros of P_{p+1} and their weights
void gl_rule(int p, std::vector<double> &xi, std::vector<double> &w);
void derivative_matrix(const std::vector<double> &xi, std::vector<double> &D);
void interpolation_matrix(const std::vector<double> &from, const std::vector<double> &to,
                          std::vector<double> &J);
// Symmetric eigen-decomposition by cyclic Jacobi rotations: A (n x n,
// row-major, symmetric) -> ascending eigenvalues and orthonormal eigenvectors
// (column j of Q, Q[i*n+j]).
void jacobi_eigen(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &Q);

}  // namespace sipg
