// Host-side set-up numerics; see host_tables.h.
//
// The discretization follows Sec. 2 of the paper with the standard symmetric
// interior penalty form: on a face between element e (minus side, at its
// xi = +1) and e+1 (plus side, at its xi = -1) the 1D form contributes
// -{v'}[[u]] - [[v]]{u'} + mu [[v]][[u]]  with [[v]] = v^- - v^+ and {v'} the
// mean of the one-sided derivatives.  With the traces tm = phi(-1),
// tp = phi(+1) and end derivatives dm = phi'(-1), dp = phi'(+1) of the
// element's Lagrange basis, the element blocks of the 1D stiffness are
//   Ld = (2/h) D^T W D
//        - (1/h) (dp tp^T + tp dp^T) + mu tp tp^T            (right face)
//        + (1/h) (dm tm^T + tm dm^T) + mu tm tm^T            (left face)
//   U  = L_{e,e+1} = (1/h) dp tm^T - (1/h) tp dm^T - mu tp tm^T.
// For GLL nodes tm = e_0, tp = e_p and dm, dp are the first and last rows of
// the derivative matrix; for GL nodes (no node at the ends) all four are
// full vectors.
#include "host_tables.h"

#include <algorithm>
#include <cmath>
#include <sstream>
#include <stdexcept>

namespace sipg {

namespace {

// P_p(x) and P_p'(x) by the three-term recurrence and
// P'_{k+1} = P'_{k-1} + (2k+1) P_k.
void legendre(int p, double x, double &P, double &dP) {
  if (p == 0) { P = 1.0; dP = 0.0; return; }
  double pm = 1.0, pk = x, dm = 0.0, dk = 1.0;
  for (int k = 1; k < p; ++k) {
    double pn = ((2 * k + 1) * x * pk - k * pm) / (k + 1);
    double dn = dm + (2 * k + 1) * pk;
    pm = pk; pk = pn; dm = dk; dk = dn;
  }
  P = pk;
  dP = dk;
}

double overlap_fraction(const sipg_params &p, int d) {
  const double h[3] = {p.len[0] / p.ne[0], p.len[1] / p.ne[1], p.len[2] / p.ne[2]};
  switch (p.overlap_mode) {
    case SIPG_OVL_MIN: return 0.0;
    case SIPG_OVL_REL: return p.overlap;
    case SIPG_OVL_MAX: {
      double hmax = std::max(h[0], std::max(h[1], h[2]));
      return std::min(p.overlap * hmax, h[d]) / h[d];
    }
  }
  return 0.0;
}

// Overlap layers: neighbour nodes whose distance from the shared face,
// (1 + xi)/2 element widths, is at most frac (GLL) or below it (GL), with a
// 1e-12 tolerance (Table 1: the middle node at 0.5 dx counts for GLL, not
// for GL); at least `floor`.  The minimal overlap is one layer either way.
int count_layers(const sipg_params &prm, const std::vector<double> &xi, double frac) {
  if (prm.overlap_mode == SIPG_OVL_MIN) return 1;
  int c = 0;
  for (double x : xi) {
    const double d = (1.0 + x) / 2.0;
    if (prm.basis == SIPG_BASIS_GL ? d < frac - 1e-12 : d <= frac + 1e-12) ++c;
  }
  return std::max(c, prm.overlap_floor);
}

// Traces phi_j(x) and derivatives phi_j'(x) of the Lagrange basis on xi at a
// point x that is not a node: phi_j(x) = prod_{k != j} (x - x_k)/(x_j - x_k)
// and phi_j'(x) = phi_j(x) sum_{k != j} 1/(x - x_k).
void end_values(const std::vector<double> &xi, double x, std::vector<double> &phi, std::vector<double> &dphi) {
  const int n = (int)xi.size();
  phi.assign(n, 0.0);
  dphi.assign(n, 0.0);
  for (int j = 0; j < n; ++j) {
    double v = 1.0, s = 0.0;
    for (int k = 0; k < n; ++k) {
      if (k == j) continue;
      v *= (x - xi[k]) / (xi[j] - xi[k]);
      s += 1.0 / (x - xi[k]);
    }
    phi[j] = v;
    dphi[j] = v * s;
  }
}

// C = Dm^{-1/2} A Dm^{-1/2}, eigen-decomposed; S = Dm^{-1/2} Q so that
// A S = diag(Dm) S Lambda and S^T diag(Dm) S = I.
void generalized_eigen(int n, const std::vector<double> &A, const std::vector<double> &Dm,
                       std::vector<double> &lam, std::vector<double> &S) {
  std::vector<double> C(n * n);
  std::vector<double> s(n);
  for (int i = 0; i < n; ++i) s[i] = 1.0 / std::sqrt(Dm[i]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[i * n + j] = s[i] * A[i * n + j] * s[j];
  // exact symmetry for the rotation algorithm
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double v = 0.5 * (C[i * n + j] + C[j * n + i]);
      C[i * n + j] = C[j * n + i] = v;
    }
  std::vector<double> Q;
  jacobi_eigen(n, C, lam, Q);
  S.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) S[i * n + j] = s[i] * Q[i * n + j];
}

// Eigenpairs of the symmetric pair (A, diag(Dm)) of order m split by the
// reversal a -> m-1-a, under which both are invariant (uniform mesh,
// overlap layers alike on both sides, GLL nodes symmetric about 0).  With
// H = m/2, the even subspace has the orthonormal basis (e_a + e_{m-1-a})/sqrt2
// (a < H) plus e_H when m is odd, the odd subspace (e_a - e_{m-1-a})/sqrt2.
// The pair projected on each subspace is solved on its own, so every
// eigenvector is exactly even or odd.  Output: even pairs first, then odd.
void generalized_eigen_eo(int m, const std::vector<double> &A, const std::vector<double> &Dm,
                          std::vector<double> &lam, std::vector<double> &S) {
  const int H = m / 2, NE = m - H;
  const double r2 = std::sqrt(0.5);
  lam.assign(m, 0.0);
  S.assign((size_t)m * m, 0.0);
  for (int odd = 0; odd < 2; ++odd) {
    const int k = odd ? H : NE;
    // basis vector i of the subspace: entries (index, coefficient)
    auto basis = [&](int i, int &a0, double &c0, int &a1, double &c1) {
      if (i < H) {
        a0 = i;
        c0 = r2;
        a1 = m - 1 - i;
        c1 = odd ? -r2 : r2;
      } else {  // centre node of an odd m (even subspace only)
        a0 = a1 = H;
        c0 = 1.0;
        c1 = 0.0;
      }
    };
    std::vector<double> Ak((size_t)k * k), Dk(k);
    for (int i = 0; i < k; ++i) {
      int ai0, ai1;
      double ci0, ci1;
      basis(i, ai0, ci0, ai1, ci1);
      Dk[i] = ci0 * ci0 * Dm[ai0] + ci1 * ci1 * Dm[ai1];  // mean of the mirrored pair
      for (int j = 0; j < k; ++j) {
        int aj0, aj1;
        double cj0, cj1;
        basis(j, aj0, cj0, aj1, cj1);
        Ak[(size_t)i * k + j] = ci0 * cj0 * A[(size_t)ai0 * m + aj0] + ci0 * cj1 * A[(size_t)ai0 * m + aj1] +
                                ci1 * cj0 * A[(size_t)ai1 * m + aj0] + ci1 * cj1 * A[(size_t)ai1 * m + aj1];
      }
    }
    std::vector<double> lk, Sk;
    generalized_eigen(k, Ak, Dk, lk, Sk);
    const int col0 = odd ? NE : 0;
    for (int j = 0; j < k; ++j) {
      lam[col0 + j] = lk[j];
      for (int i = 0; i < k; ++i) {
        int a0, a1;
        double c0, c1;
        basis(i, a0, c0, a1, c1);
        S[(size_t)a0 * m + col0 + j] += c0 * Sk[(size_t)i * k + j];
        if (a1 != a0) S[(size_t)a1 * m + col0 + j] += c1 * Sk[(size_t)i * k + j];
      }
    }
  }
}

// Hat weights of the m = n + 2 N_O subdomain nodes (N_O may be 0 with GL
// nodes: weight 1 on the element): quintic step
// S5(t) = 10t^3 - 15t^4 + 6t^5 of t = (1 + delta - |xi_H|) / (2 delta),
// clipped to [0,1], where xi_H is xi - 2 / xi / xi + 2 in the left neighbour,
// the core and the right neighbour, and delta = min(1, 1 + xi_{N_O}) is the
// distance from the face to the first neighbour node outside the subdomain
// (1 when the whole neighbour is inside).
void hat_weights(const std::vector<double> &xi, int no, std::vector<double> &w) {
  const int n = (int)xi.size();
  const int m = n + 2 * no;
  const double delta = (no <= n - 1) ? std::min(1.0, 1.0 + xi[no]) : 1.0;
  w.resize(m);
  for (int a = 0; a < m; ++a) {
    double xh;
    if (a < no) xh = xi[n - no + a] - 2.0;
    else if (a < no + n) xh = xi[a - no];
    else xh = xi[a - no - n] + 2.0;
    double t = (1.0 + delta - std::fabs(xh)) / (2.0 * delta);
    t = std::min(1.0, std::max(0.0, t));
    w[a] = t * t * t * (10.0 + t * (-15.0 + 6.0 * t));
  }
}

void build_dir(const sipg_params &prm, int p, int d, bool smoothed, Dir1D &D1) {
  D1.p = p;
  D1.n = p + 1;
  D1.ne = prm.ne[d];
  D1.h = prm.len[d] / prm.ne[d];
  D1.mu = prm.penalty * p * (p + 1) / D1.h;
  const int n = D1.n;
  const double h = D1.h, mu = D1.mu;
  if (prm.basis == SIPG_BASIS_GL) gl_rule(p, D1.xi, D1.w);
  else gll_rule(p, D1.xi, D1.w);
  derivative_matrix(D1.xi, D1.D);
  const std::vector<double> &Dm = D1.D;
  D1.mass.resize(n);
  for (int i = 0; i < n; ++i) D1.mass[i] = 0.5 * h * D1.w[i];
  // traces and end derivatives
  std::vector<double> tm(n, 0.0), tp(n, 0.0), dm(n), dp(n);
  if (prm.basis == SIPG_BASIS_GL) {
    end_values(D1.xi, -1.0, tm, dm);
    end_values(D1.xi, 1.0, tp, dp);
  } else {
    tm[0] = 1.0;
    tp[n - 1] = 1.0;
    for (int i = 0; i < n; ++i) dm[i] = Dm[0 * n + i], dp[i] = Dm[(n - 1) * n + i];
  }
  D1.TL = tm;
  D1.TR = tp;
  D1.Ld.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += Dm[q * n + i] * D1.w[q] * Dm[q * n + j];
      D1.Ld[i * n + j] = (2.0 / h) * s
                         - (dp[i] * tp[j] + tp[i] * dp[j]) / h + mu * tp[i] * tp[j]   // right face
                         + (dm[i] * tm[j] + tm[i] * dm[j]) / h + mu * tm[i] * tm[j];  // left face
    }
  D1.U.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) D1.U[i * n + j] = (dp[i] * tm[j] - tp[i] * dm[j]) / h - mu * tp[i] * tm[j];
  D1.DLs.resize(n);
  D1.DRs.resize(n);
  for (int i = 0; i < n; ++i) {
    D1.DLs[i] = dm[i] / h;
    D1.DRs[i] = dp[i] / h;
  }
  if (!smoothed) return;
  const int no = std::min(n, count_layers(prm, D1.xi, overlap_fraction(prm, d)));
  D1.no = no;
  const int m = n + 2 * no;
  D1.m = m;
  // restricted pair: principal submatrix of the three-element block
  // [[Ld, U, 0], [U^T, Ld, U], [0, U^T, Ld]] on rows/cols [n - no, 2n + no)
  std::vector<double> B(9 * n * n, 0.0);
  auto Bat = [&](int r, int c) -> double & { return B[r * 3 * n + c]; };
  for (int blk = 0; blk < 3; ++blk)
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        Bat(blk * n + i, blk * n + j) = D1.Ld[i * n + j];
        if (blk < 2) {
          Bat(blk * n + i, (blk + 1) * n + j) = D1.U[i * n + j];
          Bat((blk + 1) * n + j, blk * n + i) = D1.U[i * n + j];
        }
      }
  D1.Ls.assign(m * m, 0.0);
  D1.Ms.resize(m);
  for (int a = 0; a < m; ++a) {
    D1.Ms[a] = D1.mass[(n - no + a) % n];
    for (int b = 0; b < m; ++b) D1.Ls[a * m + b] = Bat(n - no + a, n - no + b);
  }
  generalized_eigen(m, D1.Ls, D1.Ms, D1.lam, D1.S);
  generalized_eigen_eo(m, D1.Ls, D1.Ms, D1.lam_eo, D1.S_eo);
  hat_weights(D1.xi, no, D1.wsub);
}

}  // namespace

std::vector<int> level_orders(int P) {
  std::vector<int> o;
  int q = 1;
  while (q < P) { o.push_back(q); q *= 2; }
  o.push_back(P);
  return o;
}

void gll_rule(int p, std::vector<double> &xi, std::vector<double> &w) {
  const int n = p + 1;
  xi.assign(n, 0.0);
  w.assign(n, 0.0);
  xi[0] = -1.0;
  xi[p] = 1.0;
  const double pi = 3.14159265358979323846;
  for (int i = 1; i < p; ++i) {
    // Newton on P_p'(x) = 0 from the Chebyshev-Lobatto point
    double x = -std::cos(pi * i / p);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, x, P, dP);
      double d2P = (2.0 * x * dP - p * (p + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    xi[i] = x;
  }
  for (int i = 1; i < p; ++i) {  // exact symmetry
    if (i < p - i) {
      double a = 0.5 * (xi[p - i] - xi[i]);
      xi[i] = -a;
      xi[p - i] = a;
    } else if (i == p - i) {
      xi[i] = 0.0;
    }
  }
  for (int i = 0; i < n; ++i) {
    double P, dP;
    legendre(p, xi[i], P, dP);
    w[i] = 2.0 / (p * (p + 1.0) * P * P);
  }
}

void gl_rule(int p, std::vector<double> &xi, std::vector<double> &w) {
  const int n = p + 1;
  xi.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    // Newton on P_n(x) = 0 from the asymptotic guess of the i-th zero
    double x = -std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, x, P, dP);
      const double dx = P / dP;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    xi[i] = x;
  }
  for (int i = 0; i < n; ++i) {  // exact symmetry
    if (i < n - 1 - i) {
      const double a = 0.5 * (xi[n - 1 - i] - xi[i]);
      xi[i] = -a;
      xi[n - 1 - i] = a;
    } else if (i == n - 1 - i) {
      xi[i] = 0.0;
    }
  }
  for (int i = 0; i < n; ++i) {
    double P, dP;
    legendre(n, xi[i], P, dP);
    w[i] = 2.0 / ((1.0 - xi[i] * xi[i]) * dP * dP);
  }
}

void derivative_matrix(const std::vector<double> &xi, std::vector<double> &D) {
  // barycentric form: lambda_j = 1 / prod_{k != j} (x_j - x_k),
  // D_ij = (lambda_j / lambda_i) / (x_i - x_j), D_ii = -sum_{j != i} D_ij
  const int n = (int)xi.size();
  std::vector<double> lam(n, 1.0);
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != j) prod *= (xi[j] - xi[k]);
    lam[j] = 1.0 / prod;
  }
  D.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double v = (lam[j] / lam[i]) / (xi[i] - xi[j]);
      D[i * n + j] = v;
      diag -= v;
    }
    D[i * n + i] = diag;
  }
}

void interpolation_matrix(const std::vector<double> &from, const std::vector<double> &to,
                          std::vector<double> &J) {
  const int nf = (int)from.size(), nt = (int)to.size();
  std::vector<double> lam(nf);
  for (int j = 0; j < nf; ++j) {
    double prod = 1.0;
    for (int k = 0; k < nf; ++k)
      if (k != j) prod *= (from[j] - from[k]);
    lam[j] = 1.0 / prod;
  }
  J.assign(nt * nf, 0.0);
  for (int i = 0; i < nt; ++i) {
    int hit = -1;
    for (int j = 0; j < nf; ++j)
      if (to[i] == from[j]) hit = j;
    if (hit >= 0) { J[i * nf + hit] = 1.0; continue; }
    double den = 0.0;
    for (int j = 0; j < nf; ++j) den += lam[j] / (to[i] - from[j]);
    for (int j = 0; j < nf; ++j) J[i * nf + j] = (lam[j] / (to[i] - from[j])) / den;
  }
}

void jacobi_eigen(int n, std::vector<double> A, std::vector<double> &lam, std::vector<double> &Q) {
  Q.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[i * n + i] = 1.0;
  double frob = 0.0;
  for (double v : A) frob += v * v;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off <= 1e-32 * frob) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double app = A[p * n + p], aqq = A[q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  std::vector<int> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * n + a] < A[b * n + b]; });
  lam.resize(n);
  std::vector<double> Qs(n * n);
  for (int j = 0; j < n; ++j) {
    lam[j] = A[idx[j] * n + idx[j]];
    for (int i = 0; i < n; ++i) Qs[i * n + j] = Q[i * n + idx[j]];
  }
  Q.swap(Qs);
}

std::string validate(const sipg_params &p) {
  std::ostringstream os;
  for (int d = 0; d < 3; ++d) {
    if (p.ne[d] < 3) { os << "ne[" << d << "] = " << p.ne[d] << " < 3"; return os.str(); }
    if (p.ne[d] > 4096) { os << "ne[" << d << "] too large"; return os.str(); }
    if (!(p.len[d] > 0.0) || !std::isfinite(p.len[d])) {
      os << "len[" << d << "] must be positive and finite"; return os.str();
    }
  }
  if (p.P < 1 || (p.P > 16 && p.P != kMaxOrder)) {
    os << "order P = " << p.P << " not supported (1..16 or 32)";
    return os.str();
  }
  if (!(p.penalty > 0.5) || !std::isfinite(p.penalty)) {
    os << "penalty factor must exceed 1/2 (stability threshold)"; return os.str();
  }
  if (p.overlap_mode < 0 || p.overlap_mode > 2) return "unknown overlap mode";
  if (p.basis != SIPG_BASIS_GLL && p.basis != SIPG_BASIS_GL) return "basis must be SIPG_BASIS_GLL or SIPG_BASIS_GL";
  // GL traces couple a face to every node of the adjacent elements: with 3
  // elements the two overlap layers of a subdomain would also couple through
  // the periodic wrap, which the restricted 1D operator leaves out
  if (p.basis == SIPG_BASIS_GL)
    for (int d = 0; d < 3; ++d)
      if (p.ne[d] < 4) return "the GL basis needs ne >= 4 in every direction";
  if (p.overlap_floor < 0 || p.overlap_floor > 2) return "overlap_floor must be in 0..2";
  if (p.overlap_mode != SIPG_OVL_MIN && (!(p.overlap >= 0.0) || p.overlap > 1.0))
    return "overlap width omega must lie in [0, 1]";
  if (p.nsmooth_pre < 0 || p.nsmooth_post < 0 || p.nsmooth_pre + p.nsmooth_post < 1)
    return "need nsmooth_pre, nsmooth_post >= 0 with at least one smoothing step";
  if (p.smooth_growth < 1 || p.smooth_growth > 8) return "smooth_growth must be in 1..8";
  if (p.precond_bits != 64 && p.precond_bits != 32 && p.precond_bits != 16)
    return "precond_bits must be 64, 32 or 16";
  // the coarse solve moves level-0 lines (2 ne_d nodes) through chunks of
  // 4096 values in LDS, a z line twice
  for (int d = 0; d < 3; ++d)
    if (p.ne[d] > 1024) return "ne[d] must be at most 1024 (the level-0 lines of the coarse solve)";
  const int64_t E = (int64_t)p.ne[0] * p.ne[1] * p.ne[2];
  if (E * (int64_t)(p.P + 1) * (p.P + 1) * (p.P + 1) > (int64_t)1 << 31)
    return "problem too large (more than 2^31 unknowns)";
  return "";
}

void build_hierarchy(const sipg_params &prm, HierarchyHost &H) {
  std::string err = validate(prm);
  if (!err.empty()) throw std::invalid_argument(err);
  H.prm = prm;
  H.orders = level_orders(prm.P);
  const int L = (int)H.orders.size() - 1;
  H.lev.assign(L + 1, LevelHost());
  for (int l = 0; l <= L; ++l) {
    LevelHost &lv = H.lev[l];
    lv.p = H.orders[l];
    lv.n = lv.p + 1;
    for (int d = 0; d < 3; ++d) {
      build_dir(prm, lv.p, d, l > 0, lv.dir[d]);
      if (l > 0 && lv.dir[d].no == lv.n && prm.ne[d] < 4) {
        std::ostringstream os;
        os << "direction " << d << " takes whole neighbour elements on level " << l
           << " and needs ne >= 4";
        throw std::invalid_argument(os.str());
      }
    }
    if (l > 0) interpolation_matrix(H.lev[l - 1].dir[0].xi, lv.dir[0].xi, lv.J);
  }
  // level 0 global periodic pairs (P = 1, two nodes per element)
  for (int d = 0; d < 3; ++d) {
    const Dir1D &D0 = H.lev[0].dir[d];
    const int n = D0.n, ne = prm.ne[d], N = ne * n;
    std::vector<double> Lg(N * N, 0.0), Mg(N);
    for (int e = 0; e < ne; ++e) {
      const int e1 = (e + 1) % ne;
      for (int i = 0; i < n; ++i) {
        Mg[e * n + i] = D0.mass[i];
        for (int j = 0; j < n; ++j) {
          Lg[(e * n + i) * N + e * n + j] += D0.Ld[i * n + j];
          Lg[(e * n + i) * N + e1 * n + j] += D0.U[i * n + j];
          Lg[(e1 * n + j) * N + e * n + i] += D0.U[i * n + j];
        }
      }
    }
    CoarseHost &C = H.coarse;
    C.N[d] = N;
    generalized_eigen(N, Lg, Mg, C.lam[d], C.S[d]);
    int z = 0;
    for (int i = 1; i < N; ++i)
      if (std::fabs(C.lam[d][i]) < std::fabs(C.lam[d][z])) z = i;
    C.lam[d][z] = 0.0;
    C.zero[d] = z;
  }
}

}  // namespace sipg
