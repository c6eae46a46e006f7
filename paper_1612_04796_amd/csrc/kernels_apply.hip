// Element-by-element application of the SIPG operator of eq. (A),
//   A = Mz x My x Lx + Mz x Ly x Mx + Lz x My x Mx,
// by sum factorization, and the inter-level transfers of Sec. 3.2.
//
// Each workgroup owns EPB consecutive elements.  Thread t owns one x line,
// one y line and one z line of one element (the same index pair in the three
// orientations).  In a prologue every thread reads the six face-neighbour
// lines it needs and reduces each to the two numbers the face coupling uses
// (the neighbour value at the shared face and its one-sided derivative
// there), so all neighbour loads of the workgroup are in flight at once.  The
// element's own data is staged in LDS and each direction's n x n block of L_d
// (centro-symmetric) is applied in even-odd form with the line in registers
// (uniform table entries through the scalar cache).  XCD-aware block
// numbering keeps neighbour re-reads in L2.
//
// With DL = D[0][:]/h, DR = D[p][:]/h the coupling of line v of element e to
// its right neighbour line vr and left neighbour line vl is (GLL)
//   c[i] = DR[i] vr[0] - DL[i] vl[p]
//        - [i = p] (DL . vr + mu vr[0]) + [i = 0] (DR . vl - mu vl[p]).
// For the GL basis (GL = true) the face values are the traces
// vR = TL . vr, vL = TR . vl (TL = phi(-1), TR = phi(+1)), DL, DR the end
// derivatives over h, and the unit vectors e_p, e_0 above become TR, TL:
//   c[i] = (DR[i] - mu TR[i]) vR - TR[i] (DL . vr)
//        + (-DL[i] - mu TL[i]) vL + TL[i] (DR . vl).
//
// Levels are 1, 2, 4, ..., 2^k < P, P, so the coarse size below a level of n
// nodes is fixed by n: n_c = 2^floor(log2(n - 2)) + 1.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

enum { MODE_APPLY = 0, MODE_RESID = 1, MODE_RESTRICT = 2 };

constexpr int coarse_n(int n) {
  int q = 1;
  while (2 * q <= n - 2) q *= 2;
  return n >= 3 ? q + 1 : 0;
}

template <int N>
struct ApplyShape {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int EPB = (256 / N2) > 0 ? 256 / N2 : 1;
  static constexpr int LINES = EPB * N2;
  static constexpr int NTH0 = (LINES + 63) / 64 * 64;
  static constexpr int NTH = NTH0 > 1024 ? 1024 : NTH0;
  static constexpr size_t SHM = 2 * (size_t)EPB * N3;  // elements of T
};

// Face data of one line direction: neighbour value at the shared face (v) and
// its scaled one-sided normal derivative (g), right (+) and left (-) side.
template <typename T>
struct FaceData {
  T vR, gR, vL, gL;
};

// (lines stored in TI, computed in T)
template <typename T, int N, bool GL, typename TI>
__device__ __forceinline__ FaceData<T> face_data(const TI *__restrict__ lr, const TI *__restrict__ ll, int st,
                                                 const T *__restrict__ DL, const T *__restrict__ DR,
                                                 const T *__restrict__ TL, const T *__restrict__ TR) {
  FaceData<T> fd;
  T gR = 0, gL = 0;
  if constexpr (GL) {
    T vR = 0, vL = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T r = (T)lr[i * st], l = (T)ll[i * st];
      gR += DL[i] * r;
      gL += DR[i] * l;
      vR += TL[i] * r;
      vL += TR[i] * l;
    }
    fd.vR = vR;
    fd.vL = vL;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      gR += DL[i] * (T)lr[i * st];
      gL += DR[i] * (T)ll[i * st];
    }
    fd.vR = (T)lr[0];
    fd.vL = (T)ll[(N - 1) * st];
  }
  fd.gR = gR;
  fd.gL = gL;
  return fd;
}

// All N outputs of L_d applied to the line v, with the face coupling; the
// element block is applied in its even-odd form (about half the
// multiply-adds of the plain n x n product; Ld is centro-symmetric).
template <typename T, int N, bool GL>
__device__ __forceinline__ void line_op_all(const T (&v)[N], T (&out)[N], const T *__restrict__ eo,
                                            const T *__restrict__ DL, const T *__restrict__ DR, T mu,
                                            const FaceData<T> &fd, const T *__restrict__ TL,
                                            const T *__restrict__ TR) {
  constexpr int H = N / 2;
  const T *Ae = eo, *Ao = eo + H * H, *Ac = eo + 2 * H * H, *Acr = Ac + H;
  T sm[H], df[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    sm[j] = v[j] + v[N - 1 - j];
    df[j] = v[j] - v[N - 1 - j];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T ev = 0, od = 0;
#pragma unroll
    for (int j = 0; j < H; ++j) {
      ev += Ae[i * H + j] * sm[j];
      od += Ao[i * H + j] * df[j];
    }
    if constexpr (N & 1) ev += Ac[i] * v[H];
    out[i] = ev + od;
    out[N - 1 - i] = ev - od;
  }
  if constexpr (N & 1) {
    T c = Acr[H] * v[H];
#pragma unroll
    for (int j = 0; j < H; ++j) c += Acr[j] * sm[j];
    out[H] = c;
  }
  if constexpr (GL) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      out[i] += (DR[i] - mu * TR[i]) * fd.vR - TR[i] * fd.gR - (DL[i] + mu * TL[i]) * fd.vL + TL[i] * fd.gL;
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] += DR[i] * fd.vR - DL[i] * fd.vL;
    out[N - 1] -= fd.gR + mu * fd.vR;
    out[0] += fd.gL - mu * fd.vL;
  }
}

// Several operator applications of one order in one launch (the same-order
// work of several resident solves): segment k owns workgroups
// [blk0, blk0 + nblk) and runs them exactly as its own launch would (same
// elements per workgroup, workgroup numbering and partial sums).
template <typename T>
struct ApplySeg {
  Mesh g;
  ApplyTabs<T> tb;
  const T *u;
  const T *f;
  T *out;
  T *partial;
  const T *J;
  int blk0, nblk;
  bool nt, tiled;
  const float *u32;  // the input when the kernel reads single precision
};
template <typename T>
struct ApplySegs {
  ApplySeg<T> s[kMaxApplySegments];
  int n;
};

// EPB (elements per workgroup) is chosen at launch, at most ApplyShape<N>::EPB.
// SEG: the launch covers the segments in `segs` (every other operand except
// EPB is taken from the workgroup's segment).  TI: the precision u is stored
// in (promoted to T on load).
template <typename T, int N, int MODE, bool DOT, bool SEG, bool GL, typename TI = T>
__global__ void __launch_bounds__(ApplyShape<N>::NTH)
apply_kernel(Mesh g, ApplyTabs<T> tb, const TI *__restrict__ u, const T *__restrict__ f, T *__restrict__ out,
             T *__restrict__ partial, const T *__restrict__ J, int EPB, bool nt, bool tiled, ApplySegs<T> segs) {
  using Sh = ApplyShape<N>;
  int bid = blockIdx.x, nblocks = gridDim.x;
  if constexpr (SEG) {
    int k = 0;
    while (k + 1 < segs.n && bid >= segs.s[k + 1].blk0) ++k;
    const ApplySeg<T> &a = segs.s[k];
    g = a.g;
    tb = a.tb;
    if constexpr (std::is_same<TI, T>::value) u = a.u;
    else u = a.u32;
    f = a.f;
    out = a.out;
    partial = a.partial;
    J = a.J;
    nt = a.nt;
    tiled = a.tiled;
    bid -= a.blk0;
    nblocks = a.nblk;
  }
  constexpr int N2 = Sh::N2, N3 = Sh::N3;
  constexpr int NC = coarse_n(N);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *su = reinterpret_cast<T *>(smem_raw);
  T *sy = su + EPB * N3;
  __shared__ T red[16];
  const int blk = xcd_block(bid, nblocks);
  const int e0 = group_first_element(g, blk, EPB, tiled);
  const int nloc = min(EPB, g.E - e0);
  const int t = threadIdx.x;
  const bool active = t < nloc * N2;
  const int le = t / N2, pq = t - le * N2;
  const int p = pq / N, q = pq - p * N;  // x line (k=p, j=q); y line (k=p, i=q); z line (j=p, i=q)

  // All global loads of the prologue are issued before any is consumed: the
  // element's own values (N per thread suffice, as blockDim.x >= nloc N^2),
  // the load vector of the z line, then the face lines.
  T st[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int idx = t + j * (int)blockDim.x;
    st[j] = idx < nloc * N3 ? (T)u[(size_t)e0 * N3 + idx] : (T)0;
  }
  T fl[N];
  if (MODE != MODE_APPLY && active) {
#pragma unroll
    for (int k = 0; k < N; ++k) fl[k] = f[(size_t)(e0 + le) * N3 + pq + k * N2];
  }
  FaceData<T> fx{}, fy{}, fz{};
  // mass-matrix factors of the three line directions, loaded with the rest
  // of the prologue (a load inside a phase would stall it after its barrier)
  const T scx = tb.M[2][p] * tb.M[1][q], scy = tb.M[2][p] * tb.M[0][q], scz = tb.M[1][p] * tb.M[0][q];
  if (active) {
    const int e = e0 + le;
    const int ex = e % g.ne[0], rest = e / g.ne[0];
    const int ey = rest % g.ne[1], ez = rest / g.ne[1];
    const TI *uxr = u + (size_t)elem_index(g, wrap(ex + 1, g.ne[0]), ey, ez) * N3 + pq * N;
    const TI *uxl = u + (size_t)elem_index(g, wrap(ex - 1, g.ne[0]), ey, ez) * N3 + pq * N;
    const TI *uyr = u + (size_t)elem_index(g, ex, wrap(ey + 1, g.ne[1]), ez) * N3 + p * N2 + q;
    const TI *uyl = u + (size_t)elem_index(g, ex, wrap(ey - 1, g.ne[1]), ez) * N3 + p * N2 + q;
    const TI *uzr = u + (size_t)elem_index(g, ex, ey, wrap(ez + 1, g.ne[2])) * N3 + pq;
    const TI *uzl = u + (size_t)elem_index(g, ex, ey, wrap(ez - 1, g.ne[2])) * N3 + pq;
    fx = face_data<T, N, GL, TI>(uxr, uxl, 1, tb.DL[0], tb.DR[0], tb.TL[0], tb.TR[0]);
    fy = face_data<T, N, GL, TI>(uyr, uyl, N, tb.DL[1], tb.DR[1], tb.TL[1], tb.TR[1]);
    fz = face_data<T, N, GL, TI>(uzr, uzl, N2, tb.DL[2], tb.DR[2], tb.TL[2], tb.TR[2]);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const int idx = t + j * (int)blockDim.x;
    if (idx < nloc * N3) su[idx] = st[j];
  }
  __syncthreads();

  if (active) {  // x: line (k=p, j=q), contiguous
    T *sl = su + le * N3 + pq * N;
    T *yl = sy + le * N3 + pq * N;
    T v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = sl[i];
    const T sc = scx;
    T o[N];
    line_op_all<T, N, GL>(v, o, tb.LdEO[0], tb.DL[0], tb.DR[0], tb.mu[0], fx, tb.TL[0], tb.TR[0]);
#pragma unroll
    for (int i = 0; i < N; ++i) yl[i] = sc * o[i];
  }
  __syncthreads();
  if (active) {  // y: line (k=p, i=q), stride N
    T *sl = su + le * N3 + p * N2 + q;
    T *yl = sy + le * N3 + p * N2 + q;
    T v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = sl[j * N];
    const T sc = scy;
    T o[N];
    line_op_all<T, N, GL>(v, o, tb.LdEO[1], tb.DL[1], tb.DR[1], tb.mu[1], fy, tb.TL[1], tb.TR[1]);
#pragma unroll
    for (int j = 0; j < N; ++j) yl[j * N] += sc * o[j];
  }
  __syncthreads();
  T dot = 0;
  if (active) {  // z: line (j=p, i=q), stride N^2; completes the operator
    T *sl = su + le * N3 + pq;
    T *yl = sy + le * N3 + pq;
    T v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = sl[k * N2];
    const T sc = scz;
    const size_t gbase = (size_t)(e0 + le) * N3 + pq;
    T o[N];
    line_op_all<T, N, GL>(v, o, tb.LdEO[2], tb.DL[2], tb.DR[2], tb.mu[2], fz, tb.TL[2], tb.TR[2]);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const T y = yl[k * N2] + sc * o[k];
      if (MODE == MODE_APPLY) {
        store_out(out + gbase + k * N2, y, nt);
        if (DOT) dot += v[k] * y;
      } else if (MODE == MODE_RESID) {
        const T r = fl[k] - y;
        store_out(out + gbase + k * N2, r, nt);
        if (DOT) dot += r * r;
      } else {
        yl[k * N2] = fl[k] - y;
      }
    }
  }
  if (DOT) {
    const T s = block_reduce_sum(dot, red);
    if (t == 0) partial[blk] = s;
  }
  if constexpr (MODE == MODE_RESTRICT) {
    // f_c = (J^T x J^T x J^T) r per element; J is N x NC
    __syncthreads();
    if (active) {  // x: sy[le][k][j][i] -> su[le][k][j][a]
      T v[N];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = sy[le * N3 + pq * N + i];
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const auto Jr = row_fence(J);
        T acc = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) acc += Jr[i * NC + a] * v[i];
        su[le * N3 + pq * NC + a] = acc;
      }
    }
    __syncthreads();
    // y: su[le][k][j][a] -> sy[le][k][b][a]; lines (le, k, a)
    for (int L = t; L < nloc * N * NC; L += blockDim.x) {
      const int l2 = L / (N * NC), ka = L - l2 * N * NC;
      const int k = ka / NC, a = ka - k * NC;
      T v[N];
#pragma unroll
      for (int j = 0; j < N; ++j) v[j] = su[l2 * N3 + (k * N + j) * NC + a];
#pragma unroll
      for (int b = 0; b < NC; ++b) {
        const auto Jr = row_fence(J);
        T acc = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) acc += Jr[j * NC + b] * v[j];
        sy[l2 * N3 + (k * NC + b) * NC + a] = acc;
      }
    }
    __syncthreads();
    // z: sy[le][k][b][a] -> out[e][c][b][a]; lines (le, b, a)
    constexpr int NC2 = NC * NC, NC3 = NC2 * NC;
    for (int L = t; L < nloc * NC2; L += blockDim.x) {
      const int l2 = L / NC2, ba = L - l2 * NC2;
      T v[N];
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] = sy[l2 * N3 + k * NC2 + ba];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const auto Jr = row_fence(J);
        T acc = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) acc += Jr[k * NC + c] * v[k];
        out[(size_t)(e0 + l2) * NC3 + c * NC2 + ba] = acc;
      }
    }
  }
}

// u_f += (J x J x J)(u_c - mean), element by element; J is NF x NC.
template <typename T, typename TC, int NF>
__device__ __forceinline__ void prolong_body(int E, const T *__restrict__ J, const TC *__restrict__ uc,
                                             const double *__restrict__ mean_partials, int n_partials,
                                             double mean_scale, T *__restrict__ uf, int blk) {
  using Sh = ApplyShape<NF>;
  constexpr int NC = coarse_n(NF);
  constexpr int NF2 = NF * NF, NF3 = NF2 * NF, NC2 = NC * NC, NC3 = NC2 * NC, EPB = Sh::EPB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *s0 = reinterpret_cast<T *>(smem_raw);  // EPB * NC3  : coarse element
  T *s1 = s0 + EPB * NC3;                   // EPB * NC2 * NF : after x
  T *s2 = s1 + EPB * NC2 * NF;              // EPB * NC * NF2 : after y
  const int e0 = blk * EPB;
  const int nloc = min(EPB, E - e0);
  const int t = threadIdx.x;
  __shared__ double red[16];
  __shared__ double mean_sh;
  if (mean_partials) {  // every workgroup reduces the same partials in the same order
    double ms = 0.0;
    for (int i = t; i < n_partials; i += Sh::NTH) ms += mean_partials[i];
    ms = block_reduce_sum(ms, red);
    if (t == 0) mean_sh = ms * mean_scale;
    __syncthreads();
  }
  const double m = mean_partials ? mean_sh : 0.0;
  for (int idx = t; idx < nloc * NC3; idx += Sh::NTH)
    s0[idx] = (T)((double)uc[(size_t)e0 * NC3 + idx] - m);
  __syncthreads();
  for (int L = t; L < nloc * NC2; L += Sh::NTH) {  // x: lines (le, c, b)
    const int le = L / NC2, cb = L - le * NC2;
    T v[NC];
#pragma unroll
    for (int a = 0; a < NC; ++a) v[a] = s0[le * NC3 + cb * NC + a];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < NC; ++a) acc += J[i * NC + a] * v[a];
      s1[le * NC2 * NF + cb * NF + i] = acc;
    }
  }
  __syncthreads();
  for (int L = t; L < nloc * NC * NF; L += Sh::NTH) {  // y: lines (le, c, i)
    const int le = L / (NC * NF), ci = L - le * NC * NF;
    const int c = ci / NF, i = ci - c * NF;
    T v[NC];
#pragma unroll
    for (int b = 0; b < NC; ++b) v[b] = s1[le * NC2 * NF + (c * NC + b) * NF + i];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < NC; ++b) acc += J[j * NC + b] * v[b];
      s2[le * NC * NF2 + (c * NF + j) * NF + i] = acc;
    }
  }
  __syncthreads();
  for (int L = t; L < nloc * NF2; L += Sh::NTH) {  // z: lines (le, j, i)
    const int le = L / NF2, ji = L - le * NF2;
    T v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = s2[le * NC * NF2 + c * NF2 + ji];
    T *o = uf + (size_t)(e0 + le) * NF3 + ji;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc += J[k * NC + c] * v[c];
      o[k * NF2] += acc;
    }
  }
}

template <typename T, typename TC, int NF>
__global__ void __launch_bounds__(ApplyShape<NF>::NTH)
prolong_kernel(int E, const T *__restrict__ J, const TC *__restrict__ uc, const double *__restrict__ mean_partials,
               int n_partials, double mean_scale, T *__restrict__ uf) {
  prolong_body<T, TC, NF>(E, J, uc, mean_partials, n_partials, mean_scale, uf, xcd_block(blockIdx.x, gridDim.x));
}

// Prolongations of one order from several solves in one launch (segments
// as in ApplySegs: each numbered and mapped as in its own launch)
template <typename T, typename TC>
struct ProlongSeg {
  ProlongLaunch<T, TC> a;
  int blk0, nblk;
};
template <typename T, typename TC>
struct ProlongSegs {
  ProlongSeg<T, TC> s[kMaxApplySegments];
  int n;
};

template <typename T, typename TC, int NF>
__global__ void __launch_bounds__(ApplyShape<NF>::NTH) prolong_seg_kernel(ProlongSegs<T, TC> S) {
  int k = 0;
  const int b = blockIdx.x;
  while (k + 1 < S.n && b >= S.s[k + 1].blk0) ++k;
  const ProlongSeg<T, TC> &g = S.s[k];
  prolong_body<T, TC, NF>(g.a.E, g.a.J, g.a.uc, g.a.mean_partials, g.a.n_partials, g.a.mean_scale, g.a.uf,
                          xcd_block(b - g.blk0, g.nblk));
}

template <typename K>
hipError_t allow_lds(K kernel, size_t shm) {
  if (shm <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

// elements per workgroup: the full packing when the level fills the chip,
// one wavefront per workgroup otherwise
int apply_epb(int E, int n) {
  const int full = std::max(1, 256 / (n * n));
  if ((E + full - 1) / full >= 512) return full;
  return std::max(1, std::min(full, 64 / (n * n)));
}

int launch_epb(int E, int n, int epb) {
  return epb > 0 ? std::min(epb, std::max(1, 256 / (n * n))) : apply_epb(E, n);
}

// outputs beyond the last-level cache: non-temporal stores
template <typename T, int N>
bool out_streams(const Mesh &g) {
  return (int64_t)g.E * N * N * N * (int64_t)sizeof(T) > kStreamOutBytes;
}
// xy planes beyond half an L2: column-tile visiting order
template <typename T, int N>
bool tiled_order(const Mesh &g) {
  return (int64_t)g.ne[0] * g.ne[1] * N * N * N * (int64_t)sizeof(T) >= (2 << 20);
}

// a single-precision input only for y = A u in double
template <typename T, int MODE>
constexpr bool single_input_ok() {
  return MODE == MODE_APPLY && std::is_same<T, double>::value;
}

template <typename T, int N, int MODE, bool DOT, bool GL>
hipError_t launch_mode_b(const ApplyLaunch<T> &a, hipStream_t st) {
  using Sh = ApplyShape<N>;
  const int epb = launch_epb(a.mesh.E, N, a.epb);
  const int nblk = (a.mesh.E + epb - 1) / epb;
  const int nth = std::min(Sh::NTH, (epb * N * N + 63) / 64 * 64);
  const size_t shm = 2 * (size_t)epb * N * N * N * sizeof(T);
  const bool nt = out_streams<T, N>(a.mesh), tiled = tiled_order<T, N>(a.mesh);
  if (a.u32) {
    if constexpr (single_input_ok<T, MODE>()) {
      hipError_t e = allow_lds(apply_kernel<T, N, MODE, DOT, false, GL, float>, shm);
      if (e != hipSuccess) return e;
      apply_kernel<T, N, MODE, DOT, false, GL, float><<<nblk, nth, shm, st>>>(
          a.mesh, a.tabs, a.u32, a.f, a.out, a.partial, a.J, epb, nt, tiled, ApplySegs<T>{});
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  hipError_t e = allow_lds(apply_kernel<T, N, MODE, DOT, false, GL>, shm);
  if (e != hipSuccess) return e;
  apply_kernel<T, N, MODE, DOT, false, GL><<<nblk, nth, shm, st>>>(a.mesh, a.tabs, a.u, a.f, a.out, a.partial, a.J,
                                                                   epb, nt, tiled, ApplySegs<T>{});
  return hipGetLastError();
}

template <typename T, int N, int MODE, bool DOT>
hipError_t launch_mode(const ApplyLaunch<T> &a, hipStream_t st) {
  return a.tabs.gl ? launch_mode_b<T, N, MODE, DOT, true>(a, st) : launch_mode_b<T, N, MODE, DOT, false>(a, st);
}

template <typename T, int N>
hipError_t launch_apply_n(const ApplyLaunch<T> &a, hipStream_t st) {
  switch (a.mode) {
    case APPLY_PLAIN:
      return a.partial ? launch_mode<T, N, MODE_APPLY, true>(a, st) : launch_mode<T, N, MODE_APPLY, false>(a, st);
    case APPLY_RESID:
      return a.partial ? launch_mode<T, N, MODE_RESID, true>(a, st) : launch_mode<T, N, MODE_RESID, false>(a, st);
    case APPLY_RESTRICT:
      if constexpr (N >= 3) {
        if (a.nc != coarse_n(N)) return hipErrorInvalidValue;
        return launch_mode<T, N, MODE_RESTRICT, false>(a, st);
      }
      return hipErrorInvalidValue;
  }
  return hipErrorInvalidValue;
}

template <typename T, typename TC, int NF>
hipError_t launch_prolong_segments_n(const ProlongLaunch<T, TC> *a, int n, hipStream_t st) {
  if constexpr (NF >= 3) {
    using Sh = ApplyShape<NF>;
    constexpr int NC = coarse_n(NF);
    ProlongSegs<T, TC> S{};
    S.n = n;
    int blk = 0;
    for (int k = 0; k < n; ++k) {
      if (a[k].nf != NF || a[k].nc != NC) return hipErrorInvalidValue;
      const int nblk = (a[k].E + Sh::EPB - 1) / Sh::EPB;
      S.s[k] = ProlongSeg<T, TC>{a[k], blk, nblk};
      blk += nblk;
    }
    const size_t shm = (size_t)Sh::EPB * (NC * NC * NC + NC * NC * NF + NC * NF * NF) * sizeof(T);
    hipError_t e = allow_lds(prolong_seg_kernel<T, TC, NF>, shm);
    if (e != hipSuccess) return e;
    prolong_seg_kernel<T, TC, NF><<<blk, Sh::NTH, shm, st>>>(S);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <typename T, typename TC, int NF>
hipError_t launch_prolong_n(const ProlongLaunch<T, TC> &a, hipStream_t st) {
  if constexpr (NF >= 3) {
    using Sh = ApplyShape<NF>;
    constexpr int NC = coarse_n(NF);
    if (a.nc != NC) return hipErrorInvalidValue;
    const int nblk = (a.E + Sh::EPB - 1) / Sh::EPB;
    const size_t shm = (size_t)Sh::EPB * (NC * NC * NC + NC * NC * NF + NC * NF * NF) * sizeof(T);
    hipError_t e = allow_lds(prolong_kernel<T, TC, NF>, shm);
    if (e != hipSuccess) return e;
    prolong_kernel<T, TC, NF><<<nblk, Sh::NTH, shm, st>>>(a.E, a.J, a.uc, a.mean_partials, a.n_partials,
                                                          a.mean_scale, a.uf);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

}  // namespace

int apply_num_blocks(int E, int n, int epb) {
  if (apply_is_large(n)) return apply_large_num_blocks(E, n);
  const int b = launch_epb(E, n, epb);
  return (E + b - 1) / b;
}

int apply_max_epb(int n) { return apply_is_large(n) ? 0 : std::max(1, 256 / (n * n)); }

#define SIPG_ORDER_CASES(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17)

template <typename T, int N>
hipError_t launch_segments_n(const ApplyLaunch<T> *a, int n, hipStream_t st) {
  using Sh = ApplyShape<N>;
  const bool dot = a[0].partial != nullptr;
  const int epb = launch_epb(a[0].mesh.E, N, a[0].epb);
  const int mode = a[0].mode;
  if (mode == APPLY_RESTRICT && (N < 3 || dot)) return hipErrorInvalidValue;
  ApplySegs<T> S{};
  S.n = n;
  int blk = 0;
  const bool gl = a[0].tabs.gl != 0;
  const bool in32 = a[0].u32 != nullptr;
  if (in32 && mode != APPLY_PLAIN) return hipErrorInvalidValue;
  for (int k = 0; k < n; ++k) {
    if (a[k].n != N || a[k].mode != mode || (a[k].partial != nullptr) != dot ||
        launch_epb(a[k].mesh.E, N, a[k].epb) != epb || (a[k].tabs.gl != 0) != gl ||
        (a[k].u32 != nullptr) != in32 || (mode == APPLY_RESTRICT && a[k].nc != coarse_n(N)))
      return hipErrorInvalidValue;
    const int nblk = (a[k].mesh.E + epb - 1) / epb;
    S.s[k] = ApplySeg<T>{a[k].mesh, a[k].tabs, a[k].u, a[k].f, a[k].out, a[k].partial, a[k].J,
                         blk, nblk, out_streams<T, N>(a[k].mesh), tiled_order<T, N>(a[k].mesh), a[k].u32};
    blk += nblk;
  }
  const int nth = std::min(Sh::NTH, (epb * N * N + 63) / 64 * 64);
  const size_t shm = 2 * (size_t)epb * N * N * N * sizeof(T);
  const ApplyLaunch<T> &a0 = a[0];
  auto go_in = [&](auto kernel, auto u0) {
    hipError_t e = allow_lds(kernel, shm);
    if (e != hipSuccess) return e;
    kernel<<<blk, nth, shm, st>>>(a0.mesh, a0.tabs, u0, a0.f, a0.out, a0.partial, a0.J, epb, false, false, S);
    return hipGetLastError();
  };
  auto go = [&](auto kernel) { return go_in(kernel, a0.u); };
  if (in32) {
    if constexpr (single_input_ok<T, MODE_APPLY>()) {
      if (dot) return gl ? go_in(apply_kernel<T, N, MODE_APPLY, true, true, true, float>, a0.u32)
                         : go_in(apply_kernel<T, N, MODE_APPLY, true, true, false, float>, a0.u32);
      return gl ? go_in(apply_kernel<T, N, MODE_APPLY, false, true, true, float>, a0.u32)
                : go_in(apply_kernel<T, N, MODE_APPLY, false, true, false, float>, a0.u32);
    }
    return hipErrorInvalidValue;
  }
  if (mode == APPLY_RESTRICT) {
    if constexpr (N >= 3)
      return gl ? go(apply_kernel<T, N, MODE_RESTRICT, false, true, true>)
                : go(apply_kernel<T, N, MODE_RESTRICT, false, true, false>);
    return hipErrorInvalidValue;
  }
  if (mode == APPLY_RESID) {
    if (dot) return gl ? go(apply_kernel<T, N, MODE_RESID, true, true, true>)
                       : go(apply_kernel<T, N, MODE_RESID, true, true, false>);
    return gl ? go(apply_kernel<T, N, MODE_RESID, false, true, true>)
              : go(apply_kernel<T, N, MODE_RESID, false, true, false>);
  }
  if (dot) return gl ? go(apply_kernel<T, N, MODE_APPLY, true, true, true>)
                     : go(apply_kernel<T, N, MODE_APPLY, true, true, false>);
  return gl ? go(apply_kernel<T, N, MODE_APPLY, false, true, true>)
            : go(apply_kernel<T, N, MODE_APPLY, false, true, false>);
}

int apply_launch_epb(int E, int n, int epb) { return launch_epb(E, n, epb); }

template <typename T>
hipError_t launch_apply_segments(const ApplyLaunch<T> *a, int n, hipStream_t st) {
  if (n < 1 || n > kMaxApplySegments || apply_is_large(a[0].n)) return hipErrorInvalidValue;
  switch (a[0].n) {
#define CASE(NN) \
  case NN: return launch_segments_n<T, NN>(a, n, st);
    SIPG_ORDER_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_apply(const ApplyLaunch<T> &a, hipStream_t st) {
  switch (a.n) {
#define CASE(NN) \
  case NN: return launch_apply_n<T, NN>(a, st);
    SIPG_ORDER_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, typename TC>
hipError_t launch_prolong(const ProlongLaunch<T, TC> &a, hipStream_t st) {
  switch (a.nf) {
#define CASE(NN) \
  case NN: return launch_prolong_n<T, TC, NN>(a, st);
    SIPG_ORDER_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, typename TC>
hipError_t launch_prolong_segments(const ProlongLaunch<T, TC> *a, int n, hipStream_t st) {
  if (n < 1 || n > kMaxApplySegments) return hipErrorInvalidValue;
  switch (a[0].nf) {
#define CASE(NN) \
  case NN: return launch_prolong_segments_n<T, TC, NN>(a, n, st);
    SIPG_ORDER_CASES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_prolong_segments<double, double>(const ProlongLaunch<double, double> *, int, hipStream_t);
template hipError_t launch_prolong_segments<float, float>(const ProlongLaunch<float, float> *, int, hipStream_t);
template hipError_t launch_prolong_segments<float, double>(const ProlongLaunch<float, double> *, int, hipStream_t);
template hipError_t launch_apply<double>(const ApplyLaunch<double> &, hipStream_t);
template hipError_t launch_apply<float>(const ApplyLaunch<float> &, hipStream_t);
template hipError_t launch_apply_segments<double>(const ApplyLaunch<double> *, int, hipStream_t);
template hipError_t launch_apply_segments<float>(const ApplyLaunch<float> *, int, hipStream_t);
template hipError_t launch_prolong<double, double>(const ProlongLaunch<double, double> &, hipStream_t);
template hipError_t launch_prolong<float, float>(const ProlongLaunch<float, float> &, hipStream_t);
template hipError_t launch_prolong<float, double>(const ProlongLaunch<float, double> &, hipStream_t);

}  // namespace sipg
