// Host-callable launchers of the gfx950 kernels.  Every launcher enqueues on
// the given stream, never synchronizes, and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace sipg {

enum ApplyMode { APPLY_PLAIN = 0, APPLY_RESID = 1, APPLY_RESTRICT = 2 };

// y = A u (optionally with per-block partial sums of u.y), r = f - A u, or
// f_c = J^T (f - A u) per element.  n = P_l + 1 (2..17).
template <typename T>
struct ApplyLaunch {
  Mesh mesh;
  int n;
  ApplyTabs<T> tabs;
  const T *u;
  const T *f;       // RESID, RESTRICT
  T *out;
  int mode;
  T *partial;       // PLAIN only: one partial dot product per block, or null
  const T *J;       // RESTRICT: n x nc interpolation matrix
  int nc;           // RESTRICT: coarse nodes per direction
  int epb = 0;      // elements per workgroup (0: the default choice)
  // PLAIN with T = double: a single-precision input vector in place of u
  // (read and promoted to double; n <= 17)
  const float *u32 = nullptr;
};
template <typename T>
hipError_t launch_apply(const ApplyLaunch<T> &a, hipStream_t st);

// Several applications of one order (n <= 17), one mode and one elements-
// per-workgroup choice in one launch (at most kMaxApplySegments): each
// computes exactly what its own launch_apply would, partial sums included.
constexpr int kMaxApplySegments = 8;
// elements per workgroup a launch with ApplyLaunch::epb = epb uses
int apply_launch_epb(int E, int n, int epb);
template <typename T>
hipError_t launch_apply_segments(const ApplyLaunch<T> *a, int n, hipStream_t st);

// Number of partial sums launch_apply / launch_apply_large write with partials
// (epb as in ApplyLaunch).
int apply_num_blocks(int E, int n, int epb = 0);
// Largest elements-per-workgroup of the compile-time operator kernel of order
// n - 1 (0 when the order uses the large-element path).
int apply_max_epb(int n);

// Orders whose elements do not fit in LDS (n = 33): axis-by-axis operator
// passes from global memory.  tmp holds E*(n^3 + n^2*nc) values (restriction
// and prolongation scratch).
bool apply_is_large(int n);
int apply_large_num_blocks(int E, int n);
template <typename T>
hipError_t launch_apply_large(const ApplyLaunch<T> &a, T *tmp, hipStream_t st);

// u_f += (J x J x J)(u_c - m) per element, where m = mean_scale * (sum of
// the n_partials values at mean_partials) when mean_partials is not null (the
// Euclidean mean of the level-0 solution, from the coarse solve's row sums).
template <typename T, typename TC>
struct ProlongLaunch {
  int E;
  int nf, nc;
  const T *J;
  const TC *uc;
  const double *mean_partials;
  int n_partials;
  double mean_scale;
  T *uf;
};
template <typename T, typename TC>
hipError_t launch_prolong(const ProlongLaunch<T, TC> &a, hipStream_t st);
template <typename T, typename TC>
hipError_t launch_prolong_large(const ProlongLaunch<T, TC> &a, T *tmp, hipStream_t st);
// Several prolongations of one order (n <= 17) in one launch (at most
// kMaxApplySegments), each computed as by its own launch_prolong.
template <typename T, typename TC>
hipError_t launch_prolong_segments(const ProlongLaunch<T, TC> *a, int n, hipStream_t st);

// One weighted additive Schwarz correction: C[s] = W_s A_ss^{-1} R_s r for
// every subdomain s (m_x*m_y*m_z values per subdomain, layout [s][c][b][a]),
// then u_out = u_in + sum_s R_s^T C[s] in a fixed order (u_in may be null,
// u_out may equal u_in).
// Tables of the FP16 matrix-core local solves (kernels_mfma.hip) of one
// level with cubic subdomains of m <= 16 nodes per direction; q = l / 16.
struct MfmaTabs {
  const _Float16 *fwd[3];  // lane l, item v: S[4q + v][l % 16] / f_d (zero beyond m)
  const _Float16 *bwd[3];  // lane l, item v: w[l % 16] S[l % 16][4q + v] / g_d
  const float *ilam;       // [tile][lane][4]: (1/lambda) / max(1/lambda), zero-padded
  float kout;              // f_x f_y f_z g_x g_y g_z max(1/lambda)
};
// f_d: largest absolute column sum of S_d; g_d: largest absolute row sum of W S_d
bool mfma_fdm_supported(int n, const int m[3]);
int mfma_fdm_tiles(int m);  // 16-line tiles of the m^2 lines of one direction
hipError_t launch_schwarz_mfma(const Mesh &mesh, int n, const int m[3], const MfmaTabs &tb, const float *r,
                               float *C, hipStream_t st);

template <typename T>
struct SchwarzLaunch {
  Mesh mesh;
  int n;
  SchwarzTabs<T> tabs;
  const T *r;
  T *C;             // scratch of E * m_x*m_y*m_z values
  const T *ilam;    // 1 / (lam_x[a] + lam_y[b] + lam_z[c]), layout [c][b][a]
  const T *u_in;
  T *u_out;
  const MfmaTabs *mfma = nullptr;  // FP32 levels: local solves in FP16 on the matrix cores
  int spb = 0;                     // subdomains per workgroup of the compile-time-shape kernel
                                   // (0: its default)
  int wide_planes = 0;             // subdomains wider than the LDS kernels: planes per wave
                                   // (matrix-core kernels) or per workgroup (vector plane
                                   // kernels); 0: automatic
};
// Largest subdomains-per-workgroup of the compile-time-shape local-solve
// kernel for (n, m) (0 when there is none).
int schwarz_fixed_max_spb(int n, const int m[3]);
// Local solves and assembly of up to kMaxApplySegments levels of the same
// subdomain shape (one per solve) in one launch each; every subdomain and
// node is computed as in launch_schwarz.  Only the compile-time-shape
// kernels: segments_supported says whether a level has one.
template <typename T>
bool schwarz_segments_supported(const SchwarzLaunch<T> &a);
template <typename T>
hipError_t launch_schwarz_segments(const SchwarzLaunch<T> *a, int n, hipStream_t st);
template <typename T>
hipError_t launch_schwarz(const SchwarzLaunch<T> &a, hipStream_t st);
// the two phases separately: local solves into C, then the assembly into u
template <typename T>
hipError_t launch_schwarz_local(const SchwarzLaunch<T> &a, hipStream_t st);
template <typename T>
hipError_t launch_schwarz_assemble(const SchwarzLaunch<T> &a, hipStream_t st);
// true if the subdomain tensor of this size is solved in LDS in one kernel
bool schwarz_fits_lds(const int m[3], size_t elem_bytes);
// subdomains wider than 64 nodes: plane-by-plane kernels
bool schwarz_is_wide(const int m[3]);
template <typename T>
hipError_t launch_schwarz_wide(const SchwarzLaunch<T> &a, hipStream_t st);
// the wide local solves on the matrix cores (kernels_wide_mfma.hip): for
// subdomains up to 64 nodes per direction with SchwarzTabs::frag set;
// hipErrorNotSupported (nothing launched) otherwise
bool wide_mfma_supported(const int m[3]);
int wide_mfma_frag_count(int m);  // values of one fragment-major table
template <typename T>
hipError_t launch_schwarz_wide_mfma(const SchwarzLaunch<T> &a, hipStream_t st);

// Level-0 pseudo-inverse by global fast diagonalization; see kernels_coarse.hip.
struct CoarseLaunch {
  int ne[3];
  int N[3];                 // 2 ne_d
  const double *S[3];       // N x N
  const double *colsum[3];  // column sums of S
  const double *lam[3];     // eigenvalues, zero mode exactly 0
  int zero[3];              // zero-mode index per direction
  double *t0;               // work array of N0 = N[0]*N[1]*N[2] doubles
  double *partial;          // coarse_num_partials() plane sums of f0
  double *partial_u;        // coarse_num_partials() plane sums of u0
  double *scalars;          // [0] mean of f0, [1] mean of u0
};
int coarse_num_partials(const CoarseLaunch &c);
template <typename TI>
hipError_t launch_coarse(const CoarseLaunch &a, const TI *f0, double *u0, bool subtract_mean,
                         hipStream_t st);

// ---- fixed scratch of the allocation-free Schwarz step (scratch_noalloc.hip)
// Bytes of the file-scope device array (per device, held until the process
// ends).
constexpr size_t kNoallocScratchBytes = (size_t)96 << 20;
// Looks up the array's address on `device` (once per device; makes the device
// current for the lookup and restores the previous one).
hipError_t noalloc_scratch_init(int device);
// The address found by noalloc_scratch_init (nullptr before it).
void *noalloc_scratch(int device);

// ---- vector kernels (kernels_vec.hip) -------------------------------------
constexpr int kDotBlocks = 1024;
// partial[b] = sum over block b of x[i]*y[i] (fixed partition, deterministic)
template <typename TX, typename TY>
hipError_t launch_dot_partials(const TX *x, const TY *y, int64_t n, double *partial, hipStream_t st);
// out[0] = scale * sum_{b<np} partial[b], reduced in a fixed order by one
// block; with pub_dst, pub_src[0..pub_n) (a scalar block holding out) is then
// copied to pub_dst (a device-mapped host mirror), so no separate copy is
// needed before the host reads it
hipError_t launch_finalize(const double *partial, int np, double scale, double *out, hipStream_t st,
                           const double *pub_src = nullptr, double *pub_dst = nullptr, int pub_n = 0);
// partial[b] = sum over block b of x[i], kDotBlocks blocks
template <typename T>
hipError_t launch_sum_partials(const T *x, int64_t n, double *partial, hipStream_t st);
// y[i] -= (*s)
template <typename T>
hipError_t launch_sub_scalar(T *y, int64_t n, const double *s, hipStream_t st);
// y[i] = x[i] - (*s)
template <typename T>
hipError_t launch_sub_scalar_copy(const T *x, T *y, int64_t n, const double *s, hipStream_t st);
template <typename TO, typename TI>
hipError_t launch_convert(const TI *x, TO *y, int64_t n, hipStream_t st);
template <typename T>
hipError_t launch_fill(T *x, int64_t n, T v, hipStream_t st);

// Flexible CG scalars live in device memory: see kernels_vec.hip.
enum FcgScalar { FS_RZ = 0, FS_PQ = 1, FS_RR = 2, FS_ZQ = 3, FS_RZNEW = 4, FS_ALPHA = 5, FS_BETA = 6,
                 FS_MEAN = 7,  // Euclidean mean removed from a right-hand side
                 FS_XMEAN = 8, // Euclidean mean removed from a solution
                 FS_COUNT = 9 };
// One flexible-CG iteration is split so that no vector is read twice where
// it can be avoided:
//   r -= alpha q, partial = r.r, r32 = (float) r when given   (alpha = s[RZ] / s[PQ])
hipError_t launch_fcg_r(double *r, const double *q, int64_t n, double *s, double *partial, float *r32,
                        hipStream_t st);
// The finalize of several partial-sum arrays (scale 1, optional publish) and
// the residual update of several flexible-CG states, each in one launch
// (at most kMaxApplySegments); every segment computes exactly what its own
// launch_finalize / launch_fcg_r would.
struct FinalizeSeg {
  const double *partial;
  int np;
  double *out;
  const double *pub_src;
  double *pub_dst;
  int pub_n;
};
struct FinalizeSegs {
  FinalizeSeg s[kMaxApplySegments];
  int n;
};
hipError_t launch_finalize_segments(const FinalizeSegs &segs, hipStream_t st);
struct FcgRSeg {
  double *r;
  const double *q;
  int64_t n;
  double *s;
  double *partial;
  float *r32;
};
struct FcgRSegs {
  FcgRSeg s[kMaxApplySegments];
  int n;
};
hipError_t launch_fcg_r_segments(const FcgRSegs &segs, hipStream_t st);
//   partial = z.q and r.z (z in the preconditioner's precision)
template <typename TZ>
hipError_t launch_fcg_dot2(const TZ *z, const double *q, const double *r, int64_t n, double *partial,
                           hipStream_t st);
//   s[ZQ], s[RZNEW] from those partials; beta = -alpha s[ZQ] / s[RZ]; s[RZ] = s[RZNEW]
hipError_t launch_fcg_finalize2(const double *partial, double *s, hipStream_t st);
//   x += alpha p (deferred from the residual update, when update_x); p = z + beta p
//   (p in double, or in single precision with a single-precision z)
template <typename TZ, typename TP>
hipError_t launch_fcg_xp(double *x, TP *p, const TZ *z, int64_t n, const double *s, bool update_x,
                         hipStream_t st);
//   x += alpha p (before a convergence check of the true residual)
template <typename TP>
hipError_t launch_fcg_x(double *x, const TP *p, int64_t n, const double *s, hipStream_t st);

// Fourier right-hand side: b = M f(nodes) (before mean removal)
struct RhsLaunch {
  Mesh mesh;
  int n;
  const double *xi;      // GLL nodes (n)
  const double *mass[3]; // element mass diagonals (n)
  double h[3], len[3];
  int nmodes;
  const int *k;          // device arrays: nmodes*3, nmodes*3, nmodes
  const double *phi;
  const double *amp;
};
hipError_t launch_rhs(const RhsLaunch &a, double *b, hipStream_t st);

}  // namespace sipg
