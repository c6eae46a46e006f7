// Weighted overlapping additive Schwarz correction (Sec. 3.1):
//   du = sum_s R_s^T W_s (Sz x Sy x Sx) [ (Sz^T x Sy^T x Sx^T) R_s r
//                                          / (lam_z + lam_y + lam_x) ]
// with W_s = Wz x Wy x Wx folded into WS_d = diag(w_d) S_d.
//
// Phase 1 computes, for every element-centred subdomain, its weighted local
// correction C[s] (m_x*m_y*m_z values, layout [c][b][a], x fastest) from the
// gathered residual.  Common shapes have a compile-time kernel (even-odd
// transforms, several subdomains per workgroup).  Otherwise, when the
// subdomain tensor fits LDS this is one workgroup per subdomain: gather,
// three forward contractions, scaling, three backward contractions, all in
// LDS with one thread per 1D line.  Larger subdomains (the enlarged overlap
// of anisotropic meshes) use the three plane kernels of kernels_large.hip.
//
// Phase 2 (assembly) adds to every node the corrections of the (up to 27)
// subdomains that contain it, in a fixed order, so the result is bitwise
// reproducible (no atomics).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

// base[o*st] = sum_a S[a*m + o] base[a*st]     (S^T applied to the line)
template <typename T, int MB>
__device__ __forceinline__ void line_fwd(T *base, int st, int m, const T *__restrict__ S) {
  T v[MB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
    if (a < m) v[a] = base[a * st];
  for (int o = 0; o < m; ++o) {
    T acc = 0;
#pragma unroll
    for (int a = 0; a < MB; ++a)
      if (a < m) acc += S[a * m + o] * v[a];
    base[o * st] = acc;
  }
}

// base[a*st] = sum_o WS[a*m + o] base[o*st]    (W S applied to the line)
template <typename T, int MB>
__device__ __forceinline__ void line_bwd(T *base, int st, int m, const T *__restrict__ WS) {
  T v[MB];
#pragma unroll
  for (int o = 0; o < MB; ++o)
    if (o < m) v[o] = base[o * st];
  for (int a = 0; a < m; ++a) {
    T acc = 0;
#pragma unroll
    for (int o = 0; o < MB; ++o)
      if (o < m) acc += WS[a * m + o] * v[o];
    base[a * st] = acc;
  }
}

// z line: forward with S, divide by (lam_xy + lam_z[o]), backward with WS.
template <typename T, int MB>
__device__ __forceinline__ void line_z(T *base, int st, int m, const T *__restrict__ S,
                                       const T *__restrict__ WS, const T *__restrict__ lamz, T lam_xy) {
  line_fwd<T, MB>(base, st, m, S);
  for (int o = 0; o < m; ++o) base[o * st] = base[o * st] / (lam_xy + lamz[o]);
  line_bwd<T, MB>(base, st, m, WS);
}

template <typename T>
__device__ __forceinline__ T gather_r(const Mesh &g, int n, const T *__restrict__ r, int ex, int ey, int ez,
                                      int gx, int gy, int gz) {
  // gx etc. are node positions relative to the first node of element (ex,ey,ez)
  const int dx = gx < 0 ? -1 : (gx >= n ? 1 : 0);
  const int dy = gy < 0 ? -1 : (gy >= n ? 1 : 0);
  const int dz = gz < 0 ? -1 : (gz >= n ? 1 : 0);
  const int e = elem_index(g, wrap(ex + dx, g.ne[0]), wrap(ey + dy, g.ne[1]), wrap(ez + dz, g.ne[2]));
  return r[(size_t)e * n * n * n + ((gz - dz * n) * n + (gy - dy * n)) * n + (gx - dx * n)];
}

// for (i = tid; i < tot; i += nth) put(i, get(i)), with the loads of kGB
// consecutive iterations issued before any of their values is used
constexpr int kGB = 8;
template <typename T, typename Get, typename Put>
__device__ __forceinline__ void batched_copy(int tot, int tid, int nth, Get get, Put put) {
  for (int i0 = tid; i0 < tot; i0 += kGB * nth) {
    T val[kGB];
#pragma unroll
    for (int u = 0; u < kGB; ++u) {
      const int i = i0 + u * nth;
      val[u] = i < tot ? get(i) : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kGB; ++u) {
      const int i = i0 + u * nth;
      if (i < tot) put(i, val[u]);
    }
  }
}

template <typename T, int MB>
__global__ void __launch_bounds__(512)
schwarz_lds_kernel(Mesh g, int n, SchwarzTabs<T> tb, const T *__restrict__ r, T *__restrict__ C) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *t = reinterpret_cast<T *>(smem_raw);
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const int RX = mx | 1;  // odd row stride: x lines of neighbouring threads hit different banks
  const int s = xcd_block(blockIdx.x, gridDim.x);
  const int ex = s % g.ne[0], rest = s / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int mxy = mx * my, mxyz = mxy * mz;
  batched_copy<T>(
      mxyz, tid, nth,
      [&](int idx) {
        const int a = idx % mx, bc = idx / mx, b = bc % my, c = bc / my;
        return gather_r(g, n, r, ex, ey, ez, a - tb.no[0], b - tb.no[1], c - tb.no[2]);
      },
      [&](int idx, T v) { t[(idx / mx) * RX + idx % mx] = v; });
  __syncthreads();
  for (int L = tid; L < my * mz; L += nth) line_fwd<T, MB>(t + L * RX, 1, mx, tb.S[0]);
  __syncthreads();
  for (int L = tid; L < mx * mz; L += nth) {
    const int a = L % mx, c = L / mx;
    line_fwd<T, MB>(t + c * my * RX + a, RX, my, tb.S[1]);
  }
  __syncthreads();
  for (int L = tid; L < mx * my; L += nth) {
    const int a = L % mx, b = L / mx;
    line_z<T, MB>(t + b * RX + a, my * RX, mz, tb.S[2], tb.WS[2], tb.lam[2], tb.lam[0][a] + tb.lam[1][b]);
  }
  __syncthreads();
  for (int L = tid; L < mx * mz; L += nth) {
    const int a = L % mx, c = L / mx;
    line_bwd<T, MB>(t + c * my * RX + a, RX, my, tb.WS[1]);
  }
  __syncthreads();
  for (int L = tid; L < my * mz; L += nth) line_bwd<T, MB>(t + L * RX, 1, mx, tb.WS[0]);
  __syncthreads();
  T *Cs = C + (size_t)s * mxyz;
  batched_copy<T>(
      mxyz, tid, nth, [&](int idx) { return t[(idx / mx) * RX + idx % mx]; },
      [&](int idx, T v) { Cs[idx] = v; });
}

// u_out = u_in + sum over the subdomains containing the node, fixed order
template <typename T>
__global__ void __launch_bounds__(256)
schwarz_assemble(Mesh g, int n, SchwarzTabs<T> tb, const T *__restrict__ C, const T *u_in, T *u_out) {
  const int n3 = n * n * n;
  const int64_t idx = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)g.E * n3) return;
  const int e = (int)(idx / n3), loc = (int)(idx - (int64_t)e * n3);
  const int i = loc % n, j = (loc / n) % n, k = loc / (n * n);
  const int ex = e % g.ne[0], rest = e / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const size_t mxyz = (size_t)mx * my * mz;
  // all candidate loads are issued before any is summed (a load consumed
  // inside its branch would wait before the next is issued)
  T v[27];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    const int c = k - dz * n + tb.no[2];
    const int sz = wrap(ez + dz, g.ne[2]);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const int b = j - dy * n + tb.no[1];
      const int sy = wrap(ey + dy, g.ne[1]);
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int a = i - dx * n + tb.no[0];
        const int q = (dz + 1) * 9 + (dy + 1) * 3 + dx + 1;
        v[q] = 0;
        if (c >= 0 && c < mz && b >= 0 && b < my && a >= 0 && a < mx) {
          const int sx = wrap(ex + dx, g.ne[0]);
          v[q] = C[(size_t)elem_index(g, sx, sy, sz) * mxyz + (c * my + b) * mx + a];
        }
      }
    }
  }
  const T base = u_in ? u_in[idx] : (T)0;
  T sum = 0;
#pragma unroll
  for (int q = 0; q < 27; ++q) sum += v[q];
  u_out[idx] = base + sum;
}

// ---- fixed-size fast path ----------------------------------------------
// Subdomain sizes known at compile time: all index arithmetic folds to
// constants, the line arrays live in registers and the (uniform) table
// entries are read through the scalar cache.  SPB subdomains share a
// workgroup so that the line phases fill whole wavefronts.  The 1D
// contractions use the even-odd form below; the diagonal scaling uses the
// precomputed 1 / (lam_x[a] + lam_y[b] + lam_z[c]) table in the same mode
// order.
template <int MX, int MY, int MZ>
struct FdmShape {
  static constexpr int RX = MX | 1;
  static constexpr int VOL = MX * MY * MZ;
  static constexpr int TILE = MZ * MY * RX;
  static constexpr int L1 = MY * MZ, L2 = MX * MZ, L3 = MX * MY;
  static constexpr int LINES = L1 > L2 ? (L1 > L3 ? L1 : L3) : (L2 > L3 ? L2 : L3);
  // subdomains per workgroup by default: small workgroups (about three
  // wavefronts) interleave best on a CU (measured against 2, 3 and 6 at
  // m = 13)
  static constexpr int SPB = LINES >= 192 ? 1 : 192 / LINES;
  // the most a launch may ask for (the autotuner tries 1 .. SPBMAX): up to 8
  // subdomains, 1024 threads and 64 KiB of FP64 tile.  A partly filled last
  // wavefront issues every instruction of a full one (144 lines of a 12^3
  // subdomain fill 2.25 wavefronts; four subdomains fill 9 exactly).
  static constexpr int SPB_LINES = 1024 / LINES > 8 ? 8 : 1024 / LINES;
  static constexpr int SPB_LDS = (64 * 1024) / (TILE * 8 + 27 * 4);
  static constexpr int SPBMAX0 = SPB_LINES < SPB_LDS ? SPB_LINES : SPB_LDS;
  static constexpr int SPBMAX = SPBMAX0 > SPB ? SPBMAX0 : SPB;
  static constexpr int MMAX = MX > MY ? (MX > MZ ? MX : MZ) : (MY > MZ ? MY : MZ);
  // lines per thread in every phase (more lines per thread share each table
  // entry but lower the occupancy, which costs more: measured slower)
  static constexpr int LPT = 1;
  static constexpr int NTH0 = ((SPBMAX * LINES + LPT - 1) / LPT + 63) / 64 * 64;
  static constexpr int NTH = NTH0 > 1024 ? 1024 : NTH0;
  // threads of a launch with spb subdomains per workgroup
  static int threads(int spb) {
    const int v = ((spb * LINES + LPT - 1) / LPT + 63) / 64 * 64;
    return v > 1024 ? 1024 : v;
  }
  // dynamic LDS bytes: the spb tiles, then the 27 neighbour indices per subdomain
  static size_t lds(int spb, size_t eb) { return (size_t)spb * TILE * eb + (size_t)spb * 27 * sizeof(int); }
};

// Even-odd 1D transforms.  The subdomain pair (L_s, M_s) and the hat weights
// are invariant under the reversal a -> m-1-a of the m subdomain nodes
// (uniform mesh, equal overlap on both sides, GLL nodes symmetric about 0),
// so the eigenvectors are taken exactly even (NE = m - H of them, H = m/2)
// or odd (H), even modes first in the spectral index.  A forward transform
// contracts the H sums and H differences of mirrored entries (plus the
// centre entry for odd m) with half tables; a backward transform forms the
// even part E_a and the odd part O_a of each mirrored pair.  Per line this is
// H NE + (m odd) NE + H^2 multiply-adds instead of m^2.  Table layout: see
// pack_even_odd on the host.  K lines are transformed together, so that every
// table entry (uniform, from the scalar cache) feeds K multiply-adds.
// F: fence (else the plain pointer; the FP64 23^3 kernel spilled more with
// the fences than without)
template <bool F, typename T>
__device__ __forceinline__ auto row_ptr(const T *p) {
  if constexpr (F) return row_fence(p);
  else return p;
}

template <int M>
struct Eo {
  static constexpr int H = M / 2, NE = M - H, ODD = M & 1;
  static constexpr int FE = 0, FC = FE + H * NE, FO = FC + ODD * NE;
  static constexpr int BE = FO + H * H, BC = BE + H * NE, BO = BC + ODD * NE;
};

template <typename T, int M, int K, bool F = true>
__device__ __forceinline__ void eo_fwd(const T (&v)[K][M], T (&y)[K][M], const T *__restrict__ tab) {
  using E = Eo<M>;
  T sm[K][E::H], df[K][E::H];
#pragma unroll
  for (int l = 0; l < K; ++l)
#pragma unroll
    for (int a = 0; a < E::H; ++a) {
      sm[l][a] = v[l][a] + v[l][M - 1 - a];
      df[l][a] = v[l][a] - v[l][M - 1 - a];
    }
#pragma unroll
  for (int l = 0; l < K; ++l)
#pragma unroll
    for (int j = 0; j < M; ++j) y[l][j] = 0;
  if constexpr (E::ODD) {
    const auto t = row_ptr<F>(tab);
#pragma unroll
    for (int j = 0; j < E::NE; ++j) {
      const T c = t[E::FC + j];
#pragma unroll
      for (int l = 0; l < K; ++l) y[l][j] = c * v[l][E::H];
    }
  }
#pragma unroll
  for (int a = 0; a < E::H; ++a) {
    const auto t = row_ptr<F>(tab);
#pragma unroll
    for (int j = 0; j < E::NE; ++j) {
      const T c = t[E::FE + a * E::NE + j];
#pragma unroll
      for (int l = 0; l < K; ++l) y[l][j] += c * sm[l][a];
    }
#pragma unroll
    for (int j = 0; j < E::H; ++j) {
      const T c = t[E::FO + a * E::H + j];
#pragma unroll
      for (int l = 0; l < K; ++l) y[l][E::NE + j] += c * df[l][a];
    }
  }
}

template <typename T, int M, int K, bool F = true>
__device__ __forceinline__ void eo_bwd(const T (&y)[K][M], T (&x)[K][M], const T *__restrict__ tab) {
  using E = Eo<M>;
#pragma unroll
  for (int a = 0; a < E::H; ++a) {
    const auto t = row_ptr<F>(tab);
    T ev[K], od[K];
#pragma unroll
    for (int l = 0; l < K; ++l) ev[l] = od[l] = 0;
#pragma unroll
    for (int j = 0; j < E::NE; ++j) {
      const T c = t[E::BE + a * E::NE + j];
#pragma unroll
      for (int l = 0; l < K; ++l) ev[l] += c * y[l][j];
    }
#pragma unroll
    for (int j = 0; j < E::H; ++j) {
      const T c = t[E::BO + a * E::H + j];
#pragma unroll
      for (int l = 0; l < K; ++l) od[l] += c * y[l][E::NE + j];
    }
#pragma unroll
    for (int l = 0; l < K; ++l) {
      x[l][a] = ev[l] + od[l];
      x[l][M - 1 - a] = ev[l] - od[l];
    }
  }
  if constexpr (E::ODD) {
    const auto t = row_ptr<F>(tab);
    T cs[K];
#pragma unroll
    for (int l = 0; l < K; ++l) cs[l] = 0;
#pragma unroll
    for (int j = 0; j < E::NE; ++j) {
      const T c = t[E::BC + j];
#pragma unroll
      for (int l = 0; l < K; ++l) cs[l] += c * y[l][j];
    }
#pragma unroll
    for (int l = 0; l < K; ++l) x[l][E::H] = cs[l];
  }
}

// spb: subdomains per workgroup (at most Sh::SPBMAX); the tiles live in
// dynamic LDS (Sh::lds(spb) bytes).  In every phase thread t owns lines t,
// t + blockDim.x, ... (Sh::LPT of them), reads them from the tile and writes
// them back in place; lines of one phase are disjoint.
template <typename T, int N, int MX, int MY, int MZ>
__device__ __forceinline__ void fdm_fixed_body(const Mesh &g, const SchwarzTabs<T> &tb, const T *__restrict__ r,
                                               T *__restrict__ C, int spb, int blk) {
  using Sh = FdmShape<MX, MY, MZ>;
  constexpr int RX = Sh::RX, VOL = Sh::VOL, TILE = Sh::TILE, K = Sh::LPT;
  constexpr int NOX = (MX - N) / 2, NOY = (MY - N) / 2, NOZ = (MZ - N) / 2;
  constexpr int N3 = N * N * N;
  constexpr bool FENCE = !(sizeof(T) == 8 && MX >= 23 && MY >= 23 && MZ >= 23);
  extern __shared__ __align__(16) unsigned char fdm_smem[];
  T *t = reinterpret_cast<T *>(fdm_smem);
  int *nb = reinterpret_cast<int *>(fdm_smem + (size_t)spb * TILE * sizeof(T));  // 27 elements around each core
  const int s0 = blk * spb;
  const int nsub = min(spb, g.E - s0);
  const int tid = threadIdx.x, nth = blockDim.x;

  for (int i = tid; i < nsub * 27; i += nth) {
    const int q = i / 27, k = i - q * 27;
    const int s = s0 + q;
    const int ex = s % g.ne[0], rest = s / g.ne[0];
    const int ey = rest % g.ne[1], ez = rest / g.ne[1];
    nb[i] = elem_index(g, wrap(ex + k % 3 - 1, g.ne[0]), wrap(ey + (k / 3) % 3 - 1, g.ne[1]),
                       wrap(ez + k / 9 - 1, g.ne[2]));
  }
  __syncthreads();
  // x forward: rows (q, c, b); the row of R_s r is three contiguous runs in
  // the left neighbour, the core element and the right neighbour
  {
    const int nl = nsub * Sh::L1;
    T v[K][MX], y[K][MX];
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = tid + l * nth;
#pragma unroll
      for (int a = 0; a < MX; ++a) v[l][a] = 0;
      if (li < nl) {
        const int q = li / Sh::L1, cb = li - q * Sh::L1;
        const int b = cb % MY, c = cb / MY;
        const int gy = b - NOY, gz = c - NOZ;
        const int dy = gy < 0 ? -1 : (gy >= N ? 1 : 0), dz = gz < 0 ? -1 : (gz >= N ? 1 : 0);
        const int j = gy - dy * N, k = gz - dz * N;
        const int *nbq = nb + q * 27 + (dz + 1) * 9 + (dy + 1) * 3;
        const int row = (k * N + j) * N;
        const T *rl = r + (size_t)nbq[0] * N3 + row + (N - NOX);
        const T *r0 = r + (size_t)nbq[1] * N3 + row;
        const T *rr = r + (size_t)nbq[2] * N3 + row;
#pragma unroll
        for (int a = 0; a < NOX; ++a) v[l][a] = rl[a];
#pragma unroll
        for (int a = 0; a < N; ++a) v[l][NOX + a] = r0[a];
#pragma unroll
        for (int a = 0; a < NOX; ++a) v[l][NOX + N + a] = rr[a];
      }
    }
    eo_fwd<T, MX, K, FENCE>(v, y, tb.EO[0]);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = tid + l * nth;
      if (li < nl) {
        const int q = li / Sh::L1, cb = li - q * Sh::L1;
        T *base = t + q * TILE + cb * RX;
#pragma unroll
        for (int o = 0; o < MX; ++o) base[o] = y[l][o];
      }
    }
  }
  __syncthreads();
  // y forward: lines (q, c, a)
  {
    const int nl = nsub * Sh::L2;
    T v[K][MY], y[K][MY];
#pragma unroll
    for (int l = 0; l < K; ++l) {
      // surplus lanes read the last line (their results are not stored)
      const int li = min(tid + l * nth, nl - 1);
      const int q = li / Sh::L2, ca = li - q * Sh::L2;
      const int c = ca / MX, a = ca - c * MX;
      const T *base = t + q * TILE + c * MY * RX + a;
#pragma unroll
      for (int b = 0; b < MY; ++b) v[l][b] = base[b * RX];
    }
    eo_fwd<T, MY, K, FENCE>(v, y, tb.EO[1]);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = tid + l * nth;
      if (li < nl) {
        const int q = li / Sh::L2, ca = li - q * Sh::L2;
        const int c = ca / MX, a = ca - c * MX;
        T *base = t + q * TILE + c * MY * RX + a;
#pragma unroll
        for (int b = 0; b < MY; ++b) base[b * RX] = y[l][b];
      }
    }
  }
  __syncthreads();
  // z forward, scaling, z backward: lines (q, b, a)
  {
    const int nl = nsub * Sh::L3;
    constexpr int st = MY * RX;
    T v[K][MZ], y[K][MZ];
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = min(tid + l * nth, nl - 1);
      const int q = li / Sh::L3, ba = li - q * Sh::L3;
      const int b = ba / MX, a = ba - b * MX;
      const T *base = t + q * TILE + b * RX + a;
#pragma unroll
      for (int c = 0; c < MZ; ++c) v[l][c] = base[c * st];
    }
    eo_fwd<T, MZ, K, FENCE>(v, y, tb.EO[2]);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = min(tid + l * nth, nl - 1);
      const int q = li / Sh::L3, ba = li - q * Sh::L3;
      const T *il = tb.ilam_eo + ba;
#pragma unroll
      for (int o = 0; o < MZ; ++o) y[l][o] *= il[o * MY * MX];
    }
    eo_bwd<T, MZ, K, FENCE>(y, v, tb.EO[2]);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = tid + l * nth;
      if (li < nl) {
        const int q = li / Sh::L3, ba = li - q * Sh::L3;
        const int b = ba / MX, a = ba - b * MX;
        T *base = t + q * TILE + b * RX + a;
#pragma unroll
        for (int c = 0; c < MZ; ++c) base[c * st] = v[l][c];
      }
    }
  }
  __syncthreads();
  // y backward
  {
    const int nl = nsub * Sh::L2;
    T y[K][MY], v[K][MY];
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = min(tid + l * nth, nl - 1);
      const int q = li / Sh::L2, ca = li - q * Sh::L2;
      const int c = ca / MX, a = ca - c * MX;
      const T *base = t + q * TILE + c * MY * RX + a;
#pragma unroll
      for (int b = 0; b < MY; ++b) y[l][b] = base[b * RX];
    }
    eo_bwd<T, MY, K, FENCE>(y, v, tb.EO[1]);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = tid + l * nth;
      if (li < nl) {
        const int q = li / Sh::L2, ca = li - q * Sh::L2;
        const int c = ca / MX, a = ca - c * MX;
        T *base = t + q * TILE + c * MY * RX + a;
#pragma unroll
        for (int b = 0; b < MY; ++b) base[b * RX] = v[l][b];
      }
    }
  }
  __syncthreads();
  // x backward: rows (q, c, b), in place
  {
    const int nl = nsub * Sh::L1;
    T y[K][MX], v[K][MX];
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = min(tid + l * nth, nl - 1);
      const int q = li / Sh::L1, cb = li - q * Sh::L1;
      const T *base = t + q * TILE + cb * RX;
#pragma unroll
      for (int o = 0; o < MX; ++o) y[l][o] = base[o];
    }
    eo_bwd<T, MX, K, FENCE>(y, v, tb.EO[0]);
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const int li = tid + l * nth;
      if (li < nl) {
        const int q = li / Sh::L1, cb = li - q * Sh::L1;
        T *base = t + q * TILE + cb * RX;
#pragma unroll
        for (int a = 0; a < MX; ++a) base[a] = v[l][a];
      }
    }
  }
  __syncthreads();
  // the corrections of the workgroup's subdomains are one contiguous run of
  // C: store it with consecutive lanes on consecutive addresses (a row per
  // lane would scatter every store over 64 cache lines)
  {
    T *out = C + (size_t)s0 * VOL;
    const int tot = nsub * VOL;
    constexpr int VW = 16 / (int)sizeof(T);  // values per 16-byte store
    if constexpr (RX != MX && MX % VW == 0) {
      // 16-byte stores (a subdomain's run starts 16-byte aligned, VOL being
      // a multiple of VW); the tile holds the run's rows of MX values RX
      // apart (TILE = MZ MY RX), so entry i sits at (i / MX) RX + i % MX:
      // one division per VW values instead of two per value
      typedef T V __attribute__((ext_vector_type(VW)));
      V *ov = reinterpret_cast<V *>(out);
      for (int j = tid; j < tot / VW; j += nth) {
        const int i = j * VW, row = i / MX, a = i - row * MX;
        const T *src = t + row * RX + a;
        V v;
#pragma unroll
        for (int u = 0; u < VW; ++u) v[u] = src[u];
        ov[j] = v;
      }
    } else {
      for (int i = tid; i < tot; i += nth) {
        if constexpr (RX == MX) {
          out[i] = t[i + (i / VOL) * (TILE - VOL)];
        } else {
          const int q = i / VOL, rem = i - q * VOL;
          const int row = rem / MX, a = rem - row * MX;
          out[i] = t[q * TILE + row * RX + a];
        }
      }
    }
  }
}

// One launch per level: workgroup blk (in the XCD-aware order) owns
// subdomains blk*spb .. blk*spb + spb - 1.
template <typename T, int N, int MX, int MY, int MZ>
__global__ void __launch_bounds__((FdmShape<MX, MY, MZ>::NTH))
schwarz_fdm_fixed(Mesh g, SchwarzTabs<T> tb, const T *__restrict__ r, T *__restrict__ C, int spb) {
  fdm_fixed_body<T, N, MX, MY, MZ>(g, tb, r, C, spb, xcd_block(blockIdx.x, gridDim.x));
}

// Several levels of the same subdomain shape (one per solve of a serving
// cohort) in one launch: segment k owns the consecutive workgroups
// blk0 .. blk0 + nblk - 1, numbered and mapped within the segment exactly as
// in its own launch, so every subdomain is computed as there.
template <typename T>
struct SchwarzSeg {
  Mesh g;
  SchwarzTabs<T> tb;
  const T *r;
  T *C;
  const T *u_in;
  T *u_out;
  int blk0, nblk;
};
template <typename T>
struct SchwarzSegs {
  SchwarzSeg<T> s[kMaxApplySegments];
  int n;
};

template <typename T>
__device__ __forceinline__ const SchwarzSeg<T> &seg_of(const SchwarzSegs<T> &S, int b) {
  int k = 0;
  while (k + 1 < S.n && b >= S.s[k + 1].blk0) ++k;
  return S.s[k];
}

template <typename T, int N, int MX, int MY, int MZ>
__global__ void __launch_bounds__((FdmShape<MX, MY, MZ>::NTH))
schwarz_fdm_fixed_seg(SchwarzSegs<T> S, int spb) {
  const SchwarzSeg<T> &a = seg_of(S, (int)blockIdx.x);
  fdm_fixed_body<T, N, MX, MY, MZ>(a.g, a.tb, a.r, a.C, spb, xcd_block((int)blockIdx.x - a.blk0, a.nblk));
}

// Candidate subdomains of a node along one direction: its own element's
// (offset 0) and, where the overlap reaches it, the left or right
// neighbour's.  With an overlap below half an element (2 NO < N) a node lies
// in at most two subdomains along the direction, else in up to three.  The
// candidates are kept as element-index steps (periodic wrap included), so
// the subdomain index is the node's element index plus three steps.
template <int N, int M>
struct AxisCands {
  static constexpr int NO = (M - N) / 2;
  static constexpr int K = 2 * NO < N ? 2 : 3;
  int step[K];  // element-index step to the candidate subdomain
  int a[K];     // local index of the node in that subdomain
  bool ok[K];
  // i: node index in the element; ec, ne: element coordinate and count along
  // the direction; st: element-index stride of the direction
  __device__ __forceinline__ AxisCands(int i, int ec, int ne, int st) {
    const int sm = ec > 0 ? -st : (ne - 1) * st;       // to the left neighbour
    const int sp = ec < ne - 1 ? st : -(ne - 1) * st;  // to the right neighbour
    step[0] = 0;
    a[0] = i + NO;
    ok[0] = true;
    if constexpr (K == 2) {
      const bool left = i < NO;
      step[1] = left ? sm : sp;
      a[1] = left ? i + N + NO : i - N + NO;
      ok[1] = left || i >= N - NO;
    } else {
      step[1] = sm;
      a[1] = i + N + NO;
      ok[1] = a[1] < M;
      step[2] = sp;
      a[2] = i - N + NO;
      ok[2] = a[2] >= 0;
    }
  }
};

// Assembly with compile-time sizes: one thread per node, each workgroup
// whole elements (EPB of them; for n >= 7 one, so the element, its
// coordinates and its neighbour steps are uniform and live in scalar
// registers) when an element has at most 1024 nodes, else 256 nodes per
// workgroup.  Every candidate load is issued before any is summed (invalid
// candidates load nothing and count zero), then the contributions are added
// in a fixed order.  Offsets are 32-bit: the launcher checks that the
// correction buffer has fewer than 2^31 entries.  (The index arithmetic is
// what bounds this kernel: per node it once took about 200 vector
// instructions, and FP32 ran no faster than FP64.)
template <int N>
struct AsmShape {
  static constexpr int N3 = N * N * N;
  static constexpr bool WHOLE = N3 <= 1024;
  static constexpr int EPB = N3 >= 256 ? 1 : 256 / N3;
  static constexpr int NTH = WHOLE ? (EPB * N3 + 63) / 64 * 64 : 256;
};

template <typename T, int N, int MX, int MY, int MZ>
__device__ __forceinline__ void assemble_fixed_body(const Mesh &g, const T *__restrict__ C, const T *u_in, T *u_out,
                                                    int blk) {
  using Sh = AsmShape<N>;
  constexpr int N3 = Sh::N3, VOL = MX * MY * MZ;
  const int tid = threadIdx.x;
  int e, loc;
  if constexpr (Sh::WHOLE) {
    const int le = tid / N3;
    loc = tid - le * N3;
    e = blk * Sh::EPB + le;
    if (le >= Sh::EPB || e >= g.E) return;
  } else {
    const int gi = blk * Sh::NTH + tid;
    if (gi >= g.E * N3) return;
    e = gi / N3;
    loc = gi - e * N3;
  }
  const int idx = e * N3 + loc;
  const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
  const int ex = e % g.ne[0], rest = e / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  const AxisCands<N, MX> cx(i, ex, g.ne[0], 1);
  const AxisCands<N, MY> cy(j, ey, g.ne[1], g.ne[0]);
  const AxisCands<N, MZ> cz(k, ez, g.ne[2], g.ne[0] * g.ne[1]);
  constexpr int KX = AxisCands<N, MX>::K, KY = AxisCands<N, MY>::K, KZ = AxisCands<N, MZ>::K;
  T v[KZ][KY][KX];
#pragma unroll
  for (int zc = 0; zc < KZ; ++zc)
#pragma unroll
    for (int yc = 0; yc < KY; ++yc)
#pragma unroll
      for (int xc = 0; xc < KX; ++xc) {
        v[zc][yc][xc] = 0;
        if (cz.ok[zc] && cy.ok[yc] && cx.ok[xc]) {
          const int sub = e + cz.step[zc] + cy.step[yc] + cx.step[xc];
          v[zc][yc][xc] = C[sub * VOL + (cz.a[zc] * MY + cy.a[yc]) * MX + cx.a[xc]];
        }
      }
  const T base = u_in ? u_in[idx] : (T)0;
  T sum = 0;
#pragma unroll
  for (int zc = 0; zc < KZ; ++zc)
#pragma unroll
    for (int yc = 0; yc < KY; ++yc)
#pragma unroll
      for (int xc = 0; xc < KX; ++xc) sum += v[zc][yc][xc];
  u_out[idx] = base + sum;
}

template <typename T, int N, int MX, int MY, int MZ>
__global__ void __launch_bounds__(AsmShape<N>::NTH)
schwarz_assemble_fixed(Mesh g, const T *__restrict__ C, const T *u_in, T *u_out) {
  assemble_fixed_body<T, N, MX, MY, MZ>(g, C, u_in, u_out, xcd_block(blockIdx.x, gridDim.x));
}

template <typename T, int N, int MX, int MY, int MZ>
__global__ void __launch_bounds__(AsmShape<N>::NTH)
schwarz_assemble_fixed_seg(SchwarzSegs<T> S) {
  const SchwarzSeg<T> &a = seg_of(S, (int)blockIdx.x);
  assemble_fixed_body<T, N, MX, MY, MZ>(a.g, a.C, a.u_in, a.u_out, xcd_block((int)blockIdx.x - a.blk0, a.nblk));
}

template <typename T, int N, int MX, int MY, int MZ>
hipError_t launch_assemble_fixed(const SchwarzLaunch<T> &a, hipStream_t st) {
  using Sh = AsmShape<N>;
  if ((int64_t)a.mesh.E * MX * MY * MZ >= (int64_t)1 << 31) return hipErrorInvalidValue;
  const int nblk = Sh::WHOLE ? (a.mesh.E + Sh::EPB - 1) / Sh::EPB
                             : (int)(((int64_t)a.mesh.E * Sh::N3 + Sh::NTH - 1) / Sh::NTH);
  schwarz_assemble_fixed<T, N, MX, MY, MZ><<<nblk, Sh::NTH, 0, st>>>(a.mesh, a.C, a.u_in, a.u_out);
  return hipGetLastError();
}

template <typename T, int N, int MX, int MY, int MZ>
hipError_t launch_fixed(const SchwarzLaunch<T> &a, hipStream_t st) {
  using Sh = FdmShape<MX, MY, MZ>;
  static_assert(Sh::SPB * Sh::TILE * sizeof(T) + Sh::SPB * 27 * sizeof(int) <= 160 * 1024,
                "subdomain tile exceeds LDS");
  const int spb = a.spb > 0 ? std::min(a.spb, Sh::SPBMAX) : Sh::SPB;
  const int nblk = (a.mesh.E + spb - 1) / spb;
  const int nth = Sh::threads(spb);
  const size_t shm = Sh::lds(spb, sizeof(T));
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)schwarz_fdm_fixed<T, N, MX, MY, MZ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  schwarz_fdm_fixed<T, N, MX, MY, MZ><<<nblk, nth, shm, st>>>(a.mesh, a.tabs, a.r, a.C, spb);
  return hipGetLastError();
}

// (n, m_x, m_y, m_z) shapes with a compiled fast path: the isotropic
// minimal and 8% overlaps of orders 2..16, the levels of the 16:1:1
// aspect-ratio mesh with the "max" overlap, and the "max" overlap levels of
// orders 2..8 at aspect ratios 2..8 (x the long direction).
#define SIPG_FDM_SHAPES(X)                                                              \
  X(3, 5, 5, 5) X(5, 7, 7, 7) X(8, 10, 10, 10) X(8, 12, 12, 12) X(9, 11, 11, 11)        \
  X(9, 13, 13, 13) X(17, 19, 19, 19) X(17, 23, 23, 23) X(3, 5, 9, 9) X(5, 7, 15, 15)     \
  X(9, 13, 27, 27) X(3, 5, 7, 7) X(5, 7, 9, 9) X(5, 7, 11, 11) X(9, 13, 15, 15)          \
  X(9, 13, 17, 17) X(9, 13, 19, 19)

template <typename T>
hipError_t launch_fixed_if_any(const SchwarzLaunch<T> &a, hipStream_t st, bool &done) {
  done = true;
  const int *m = a.tabs.m;
#define SIPG_TRY(NN, AX, AY, AZ) \
  if (a.n == NN && m[0] == AX && m[1] == AY && m[2] == AZ) return launch_fixed<T, NN, AX, AY, AZ>(a, st);
  SIPG_FDM_SHAPES(SIPG_TRY)
#undef SIPG_TRY
  done = false;
  return hipSuccess;
}

// Segmented launches: the same compile-time shape for every segment, the
// first segment's subdomains-per-workgroup for all (a subdomain's values do
// not depend on it).
template <typename T, int N, int MX, int MY, int MZ>
hipError_t launch_fixed_segments(const SchwarzLaunch<T> *a, int n, hipStream_t st) {
  using Sh = FdmShape<MX, MY, MZ>;
  const int spb = a[0].spb > 0 ? std::min(a[0].spb, Sh::SPBMAX) : Sh::SPB;
  SchwarzSegs<T> S{};
  S.n = n;
  int blk = 0;
  for (int k = 0; k < n; ++k) {
    const int nblk = (a[k].mesh.E + spb - 1) / spb;
    S.s[k] = SchwarzSeg<T>{a[k].mesh, a[k].tabs, a[k].r, a[k].C, a[k].u_in, a[k].u_out, blk, nblk};
    blk += nblk;
  }
  const size_t shm = Sh::lds(spb, sizeof(T));
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)schwarz_fdm_fixed_seg<T, N, MX, MY, MZ>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  schwarz_fdm_fixed_seg<T, N, MX, MY, MZ><<<blk, Sh::threads(spb), shm, st>>>(S, spb);
  return hipGetLastError();
}

template <typename T, int N, int MX, int MY, int MZ>
hipError_t launch_assemble_fixed_segments(const SchwarzLaunch<T> *a, int n, hipStream_t st) {
  using Sh = AsmShape<N>;
  SchwarzSegs<T> S{};
  S.n = n;
  int blk = 0;
  for (int k = 0; k < n; ++k) {
    if ((int64_t)a[k].mesh.E * MX * MY * MZ >= (int64_t)1 << 31) return hipErrorInvalidValue;
    const int nblk = Sh::WHOLE ? (a[k].mesh.E + Sh::EPB - 1) / Sh::EPB
                               : (int)(((int64_t)a[k].mesh.E * Sh::N3 + Sh::NTH - 1) / Sh::NTH);
    S.s[k] = SchwarzSeg<T>{a[k].mesh, a[k].tabs, a[k].r, a[k].C, a[k].u_in, a[k].u_out, blk, nblk};
    blk += nblk;
  }
  schwarz_assemble_fixed_seg<T, N, MX, MY, MZ><<<blk, Sh::NTH, 0, st>>>(S);
  return hipGetLastError();
}

bool fixed_shape(int n, const int m[3]) {
#define SIPG_IS(NN, AX, AY, AZ) \
  if (n == NN && m[0] == AX && m[1] == AY && m[2] == AZ) return true;
  SIPG_FDM_SHAPES(SIPG_IS)
#undef SIPG_IS
  return false;
}

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

int schwarz_fixed_max_spb(int n, const int m[3]) {
#define SIPG_MAXSPB(NN, AX, AY, AZ) \
  if (n == NN && m[0] == AX && m[1] == AY && m[2] == AZ) return FdmShape<AX, AY, AZ>::SPBMAX;
  SIPG_FDM_SHAPES(SIPG_MAXSPB)
#undef SIPG_MAXSPB
  return 0;
}

namespace {

size_t lds_bytes(const int m[3], size_t eb) { return (size_t)m[2] * m[1] * (m[0] | 1) * eb; }

constexpr size_t kLdsLimit = 80 * 1024;

template <typename T, int MB>
hipError_t launch_lds(const SchwarzLaunch<T> &a, hipStream_t st) {
  const int *m = a.tabs.m;
  const int lines = std::max(m[1] * m[2], std::max(m[0] * m[2], m[0] * m[1]));
  const int nth = std::min(512, std::max(64, round_up(lines, 64)));
  const size_t shm = lds_bytes(m, sizeof(T));
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)schwarz_lds_kernel<T, MB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  schwarz_lds_kernel<T, MB><<<a.mesh.E, nth, shm, st>>>(a.mesh, a.n, a.tabs, a.r, a.C);
  return hipGetLastError();
}

}  // namespace

bool schwarz_fits_lds(const int m[3], size_t eb) {
  return lds_bytes(m, eb) <= kLdsLimit && std::max(m[0], std::max(m[1], m[2])) <= 32;
}

template <typename T>
hipError_t launch_schwarz_local(const SchwarzLaunch<T> &a, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (a.mfma) return launch_schwarz_mfma(a.mesh, a.n, a.tabs.m, *a.mfma, a.r, a.C, st);
  }
  if (a.tabs.ilam_eo) {
    bool done = false;
    hipError_t e = launch_fixed_if_any<T>(a, st, done);
    if (done) return e;
  }
  const int *m = a.tabs.m;
  const int mmax = std::max(m[0], std::max(m[1], m[2]));
  if (schwarz_fits_lds(m, sizeof(T))) {
    if (mmax <= 8) return launch_lds<T, 8>(a, st);
    if (mmax <= 16) return launch_lds<T, 16>(a, st);
    if (mmax <= 24) return launch_lds<T, 24>(a, st);
    return launch_lds<T, 32>(a, st);
  }
  return launch_schwarz_wide<T>(a, st);
}

template <typename T>
hipError_t launch_schwarz_assemble(const SchwarzLaunch<T> &a, hipStream_t st) {
  {
    const int *m = a.tabs.m;
    // the compile-time kernels use 32-bit offsets into the corrections
    const bool small = (int64_t)a.mesh.E * m[0] * m[1] * m[2] < ((int64_t)1 << 31);
#define SIPG_TRY(NN, AX, AY, AZ)                                                  \
  if (small && a.n == NN && m[0] == AX && m[1] == AY && m[2] == AZ)             \
    return launch_assemble_fixed<T, NN, AX, AY, AZ>(a, st);
    SIPG_FDM_SHAPES(SIPG_TRY)
#undef SIPG_TRY
  }
  const int64_t tot = (int64_t)a.mesh.E * a.n * a.n * a.n;
  schwarz_assemble<T><<<(int)((tot + 255) / 256), 256, 0, st>>>(a.mesh, a.n, a.tabs, a.C, a.u_in, a.u_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_schwarz(const SchwarzLaunch<T> &a, hipStream_t st) {
  hipError_t e = launch_schwarz_local<T>(a, st);
  if (e != hipSuccess) return e;
  return launch_schwarz_assemble<T>(a, st);
}

template <typename T>
bool schwarz_segments_supported(const SchwarzLaunch<T> &a) {
  const int *m = a.tabs.m;
  return a.mfma == nullptr && a.tabs.ilam_eo != nullptr && fixed_shape(a.n, m) &&
         (int64_t)a.mesh.E * m[0] * m[1] * m[2] < ((int64_t)1 << 31);
}

template <typename T>
hipError_t launch_schwarz_segments(const SchwarzLaunch<T> *a, int n, hipStream_t st) {
  if (n < 1 || n > kMaxApplySegments) return hipErrorInvalidValue;
  for (int k = 0; k < n; ++k) {
    if (!schwarz_segments_supported<T>(a[k]) || a[k].n != a[0].n) return hipErrorInvalidValue;
    for (int d = 0; d < 3; ++d)
      if (a[k].tabs.m[d] != a[0].tabs.m[d]) return hipErrorInvalidValue;
  }
  const int *m = a[0].tabs.m;
  hipError_t e = hipErrorInvalidValue;
#define SIPG_TRY(NN, AX, AY, AZ)                                  \
  if (a[0].n == NN && m[0] == AX && m[1] == AY && m[2] == AZ) {   \
    e = launch_fixed_segments<T, NN, AX, AY, AZ>(a, n, st);       \
    if (e == hipSuccess) e = launch_assemble_fixed_segments<T, NN, AX, AY, AZ>(a, n, st); \
  }
  SIPG_FDM_SHAPES(SIPG_TRY)
#undef SIPG_TRY
  return e;
}

template hipError_t launch_schwarz<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz<float>(const SchwarzLaunch<float> &, hipStream_t);
template hipError_t launch_schwarz_local<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz_local<float>(const SchwarzLaunch<float> &, hipStream_t);
template hipError_t launch_schwarz_assemble<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz_assemble<float>(const SchwarzLaunch<float> &, hipStream_t);

template bool schwarz_segments_supported<double>(const SchwarzLaunch<double> &);
template bool schwarz_segments_supported<float>(const SchwarzLaunch<float> &);
template hipError_t launch_schwarz_segments<double>(const SchwarzLaunch<double> *, int, hipStream_t);
template hipError_t launch_schwarz_segments<float>(const SchwarzLaunch<float> *, int, hipStream_t);

}  // namespace sipg
