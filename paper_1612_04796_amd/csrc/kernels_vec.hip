// Vector kernels: deterministic two-stage reductions (fixed partition into
// kDotBlocks blocks, fixed tree inside a block, one finalizing block), the
// flexible-CG updates with their scalars kept in device memory, precision
// conversions, and the Fourier right-hand side.
#include <hip/hip_runtime.h>

#include <math.h>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

__device__ __forceinline__ void chunk_of(int64_t n, int64_t &lo, int64_t &hi) {
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  lo = chunk * blockIdx.x;
  hi = lo + chunk < n ? lo + chunk : n;
}

// the same partition for block b of nb
__device__ __forceinline__ void chunk_of(int64_t n, int b, int nb, int64_t &lo, int64_t &hi) {
  const int64_t chunk = (n + nb - 1) / nb;
  lo = chunk * b;
  hi = lo + chunk < n ? lo + chunk : n;
}

// Streaming loops issue the loads of kUnroll iterations before using any,
// and accumulate in a fixed order (deterministic).
constexpr int kUnroll = 4;

template <typename TX, typename TY>
__global__ void __launch_bounds__(256)
dot_partials(const TX *__restrict__ x, const TY *__restrict__ y, int64_t n, double *__restrict__ partial) {
  __shared__ double red[16];
  int64_t lo, hi;
  chunk_of(n, lo, hi);
  double s = 0.0;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kUnroll * blockDim.x) {
    double a[kUnroll], b[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * blockDim.x;
      a[u] = i < hi ? (double)x[i] : 0.0;
      b[u] = i < hi ? (double)y[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) s += a[u] * b[u];
  }
  s = block_reduce_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(256)
sum_partials_kernel(const T *__restrict__ x, int64_t n, double *__restrict__ partial) {
  __shared__ double red[16];
  int64_t lo, hi;
  chunk_of(n, lo, hi);
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += (double)x[i];
  s = block_reduce_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// SEG: block k finalizes segment k of `segs` (the other operands unused)
template <bool SEG>
__global__ void __launch_bounds__(1024)
finalize_kernel(const double *__restrict__ partial, int np, double scale, double *out, const double *pub_src,
                double *pub_dst, int pub_n, FinalizeSegs segs) {
  __shared__ double red[16];
  if constexpr (SEG) {
    const FinalizeSeg &a = segs.s[blockIdx.x];
    partial = a.partial;
    np = a.np;
    scale = 1.0;
    out = a.out;
    pub_src = a.pub_src;
    pub_dst = a.pub_dst;
    pub_n = a.pub_dst ? a.pub_n : 0;
  }
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  s = block_reduce_sum(s, red);
  if (threadIdx.x == 0) {
    out[0] = scale * s;
    // publish: copy the scalar block (which holds out) to the host mirror
    for (int i = 0; i < pub_n; ++i) pub_dst[i] = pub_src[i];
  }
}

// y = x - s[0]; y may equal x
template <typename T>
__global__ void __launch_bounds__(256) sub_scalar(const T *x, T *y, int64_t n, const double *__restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)((double)x[i] - s[0]);
}

template <typename TO, typename TI>
__global__ void __launch_bounds__(256) convert_kernel(const TI *__restrict__ x, TO *__restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (TO)x[i];
}

template <typename T>
__global__ void __launch_bounds__(256) fill_kernel(T *__restrict__ x, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void __launch_bounds__(1024) fcg_finalize2_kernel(const double *__restrict__ partial, double *s) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < kDotBlocks; i += blockDim.x) {
    a += partial[i];
    b += partial[kDotBlocks + i];
  }
  a = block_reduce_sum(a, red);
  __syncthreads();
  b = block_reduce_sum(b, red);
  if (threadIdx.x == 0) {
    // a = z_new . q, b = r_new . z_new
    s[FS_ZQ] = a;
    s[FS_RZNEW] = b;
    s[FS_BETA] = -s[FS_ALPHA] * a / s[FS_RZ];
    s[FS_RZ] = b;
  }
}

// alpha = s[RZ] / s[PQ]; r -= alpha q; partial = r.r; r32 = (float) r when
// given (the input of a single-precision preconditioner)
// SEG: blocks [k kDotBlocks, (k + 1) kDotBlocks) run segment k of `segs`
template <bool SEG>
__global__ void __launch_bounds__(256)
fcg_r_kernel(double *__restrict__ r, const double *__restrict__ q, int64_t n, double *s,
             double *__restrict__ partial, float *__restrict__ r32, FcgRSegs segs) {
  __shared__ double red[16];
  int bid = blockIdx.x;
  if constexpr (SEG) {
    const FcgRSeg &a = segs.s[bid / kDotBlocks];
    bid -= (bid / kDotBlocks) * kDotBlocks;
    r = a.r;
    q = a.q;
    n = a.n;
    s = a.s;
    partial = a.partial;
    r32 = a.r32;
  }
  const double alpha = s[FS_RZ] / s[FS_PQ];
  int64_t lo, hi;
  if constexpr (SEG) chunk_of(n, bid, kDotBlocks, lo, hi);
  else chunk_of(n, lo, hi);
  double acc = 0.0;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kUnroll * blockDim.x) {
    double rv[kUnroll], qv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * blockDim.x;
      rv[u] = i < hi ? r[i] : 0.0;
      qv[u] = i < hi ? q[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * blockDim.x;
      const double ri = rv[u] - alpha * qv[u];
      acc += ri * ri;
      if (i < hi) {
        r[i] = ri;
        if (r32) r32[i] = (float)ri;
      }
    }
  }
  acc = block_reduce_sum(acc, red);
  if (threadIdx.x == 0) {
    partial[bid] = acc;
    if (bid == 0) s[FS_ALPHA] = alpha;
  }
}

// partial[b] = z.q, partial[kDotBlocks + b] = r.z over block b
template <typename TZ>
__global__ void __launch_bounds__(256)
fcg_dot2_kernel(const TZ *__restrict__ z, const double *__restrict__ q, const double *__restrict__ r, int64_t n,
                double *__restrict__ partial) {
  __shared__ double red[16];
  int64_t lo, hi;
  chunk_of(n, lo, hi);
  double a = 0.0, b = 0.0;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kUnroll * blockDim.x) {
    double zv[kUnroll], qv[kUnroll], rv[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = i0 + u * blockDim.x;
      zv[u] = i < hi ? (double)z[i] : 0.0;
      qv[u] = i < hi ? q[i] : 0.0;
      rv[u] = i < hi ? r[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      a += zv[u] * qv[u];
      b += rv[u] * zv[u];
    }
  }
  a = block_reduce_sum(a, red);
  __syncthreads();
  b = block_reduce_sum(b, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = a;
    partial[gridDim.x + blockIdx.x] = b;
  }
}

// x += alpha p (when update_x); p = z + beta p, formed in double and stored
// in p's precision
template <typename TZ, typename TP>
__global__ void __launch_bounds__(256)
fcg_xp_kernel(double *__restrict__ x, TP *__restrict__ p, const TZ *__restrict__ z, int64_t n,
              const double *__restrict__ s, int update_x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double pi = (double)p[i];
  if (update_x) x[i] += s[FS_ALPHA] * pi;
  p[i] = (TP)((double)z[i] + s[FS_BETA] * pi);
}

// x += alpha p
template <typename TP>
__global__ void __launch_bounds__(256)
fcg_x_kernel(double *__restrict__ x, const TP *__restrict__ p, int64_t n, const double *__restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += s[FS_ALPHA] * (double)p[i];
}

__global__ void __launch_bounds__(256) rhs_kernel(RhsLaunch a, double *__restrict__ b) {
  const int n = a.n, n3 = n * n * n;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)a.mesh.E * n3) return;
  const int e = (int)(idx / n3), loc = (int)(idx - (int64_t)e * n3);
  const int i = loc % n, j = (loc / n) % n, k = loc / (n * n);
  const int ex = e % a.mesh.ne[0], rest = e / a.mesh.ne[0];
  const int ey = rest % a.mesh.ne[1], ez = rest / a.mesh.ne[1];
  const double x[3] = {ex * a.h[0] + (1.0 + a.xi[i]) * a.h[0] * 0.5,
                       ey * a.h[1] + (1.0 + a.xi[j]) * a.h[1] * 0.5,
                       ez * a.h[2] + (1.0 + a.xi[k]) * a.h[2] * 0.5};
  const double twopi = 6.283185307179586476925286766559;
  double f = 0.0;
  for (int q = 0; q < a.nmodes; ++q) {
    double prod = a.amp[q];
    for (int d = 0; d < 3; ++d) prod *= sin(twopi * a.k[3 * q + d] * x[d] / a.len[d] + a.phi[3 * q + d]);
    f += prod;
  }
  b[idx] = a.mass[2][k] * a.mass[1][j] * a.mass[0][i] * f;
}

inline int nblocks(int64_t n) { return (int)((n + 255) / 256); }

}  // namespace

template <typename TX, typename TY>
hipError_t launch_dot_partials(const TX *x, const TY *y, int64_t n, double *partial, hipStream_t st) {
  dot_partials<TX, TY><<<kDotBlocks, 256, 0, st>>>(x, y, n, partial);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sum_partials(const T *x, int64_t n, double *partial, hipStream_t st) {
  sum_partials_kernel<T><<<kDotBlocks, 256, 0, st>>>(x, n, partial);
  return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, int np, double scale, double *out, hipStream_t st,
                           const double *pub_src, double *pub_dst, int pub_n) {
  finalize_kernel<false><<<1, 1024, 0, st>>>(partial, np, scale, out, pub_src, pub_dst, pub_dst ? pub_n : 0,
                                             FinalizeSegs{});
  return hipGetLastError();
}

hipError_t launch_finalize_segments(const FinalizeSegs &segs, hipStream_t st) {
  if (segs.n < 1 || segs.n > kMaxApplySegments) return hipErrorInvalidValue;
  finalize_kernel<true><<<segs.n, 1024, 0, st>>>(nullptr, 0, 1.0, nullptr, nullptr, nullptr, 0, segs);
  return hipGetLastError();
}

hipError_t launch_fcg_r_segments(const FcgRSegs &segs, hipStream_t st) {
  if (segs.n < 1 || segs.n > kMaxApplySegments) return hipErrorInvalidValue;
  fcg_r_kernel<true><<<segs.n * kDotBlocks, 256, 0, st>>>(nullptr, nullptr, 0, nullptr, nullptr, nullptr, segs);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sub_scalar(T *y, int64_t n, const double *s, hipStream_t st) {
  if (n == 0) return hipSuccess;
  sub_scalar<T><<<nblocks(n), 256, 0, st>>>(y, y, n, s);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sub_scalar_copy(const T *x, T *y, int64_t n, const double *s, hipStream_t st) {
  if (n == 0) return hipSuccess;
  sub_scalar<T><<<nblocks(n), 256, 0, st>>>(x, y, n, s);
  return hipGetLastError();
}

template <typename TO, typename TI>
hipError_t launch_convert(const TI *x, TO *y, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  convert_kernel<TO, TI><<<nblocks(n), 256, 0, st>>>(x, y, n);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *x, int64_t n, T v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  fill_kernel<T><<<nblocks(n), 256, 0, st>>>(x, n, v);
  return hipGetLastError();
}

hipError_t launch_fcg_r(double *r, const double *q, int64_t n, double *s, double *partial, float *r32,
                        hipStream_t st) {
  fcg_r_kernel<false><<<kDotBlocks, 256, 0, st>>>(r, q, n, s, partial, r32, FcgRSegs{});
  return hipGetLastError();
}

hipError_t launch_fcg_finalize2(const double *partial, double *s, hipStream_t st) {
  fcg_finalize2_kernel<<<1, 1024, 0, st>>>(partial, s);
  return hipGetLastError();
}

template <typename TZ>
hipError_t launch_fcg_dot2(const TZ *z, const double *q, const double *r, int64_t n, double *partial,
                           hipStream_t st) {
  fcg_dot2_kernel<TZ><<<kDotBlocks, 256, 0, st>>>(z, q, r, n, partial);
  return hipGetLastError();
}

template <typename TZ, typename TP>
hipError_t launch_fcg_xp(double *x, TP *p, const TZ *z, int64_t n, const double *s, bool update_x,
                         hipStream_t st) {
  fcg_xp_kernel<TZ, TP><<<nblocks(n), 256, 0, st>>>(x, p, z, n, s, update_x ? 1 : 0);
  return hipGetLastError();
}

template <typename TP>
hipError_t launch_fcg_x(double *x, const TP *p, int64_t n, const double *s, hipStream_t st) {
  fcg_x_kernel<TP><<<nblocks(n), 256, 0, st>>>(x, p, n, s);
  return hipGetLastError();
}

hipError_t launch_rhs(const RhsLaunch &a, double *b, hipStream_t st) {
  const int64_t n = (int64_t)a.mesh.E * a.n * a.n * a.n;
  rhs_kernel<<<nblocks(n), 256, 0, st>>>(a, b);
  return hipGetLastError();
}

template hipError_t launch_dot_partials<double, double>(const double *, const double *, int64_t, double *,
                                                        hipStream_t);
template hipError_t launch_dot_partials<double, float>(const double *, const float *, int64_t, double *,
                                                       hipStream_t);
template hipError_t launch_fcg_dot2<double>(const double *, const double *, const double *, int64_t, double *,
                                            hipStream_t);
template hipError_t launch_fcg_dot2<float>(const float *, const double *, const double *, int64_t, double *,
                                           hipStream_t);
template hipError_t launch_fcg_xp<double, double>(double *, double *, const double *, int64_t, const double *,
                                                  bool, hipStream_t);
template hipError_t launch_fcg_xp<float, double>(double *, double *, const float *, int64_t, const double *, bool,
                                                 hipStream_t);
template hipError_t launch_fcg_xp<float, float>(double *, float *, const float *, int64_t, const double *, bool,
                                                hipStream_t);
template hipError_t launch_fcg_x<double>(double *, const double *, int64_t, const double *, hipStream_t);
template hipError_t launch_fcg_x<float>(double *, const float *, int64_t, const double *, hipStream_t);
template hipError_t launch_sub_scalar<double>(double *, int64_t, const double *, hipStream_t);
template hipError_t launch_sub_scalar_copy<double>(const double *, double *, int64_t, const double *, hipStream_t);
template hipError_t launch_sub_scalar<float>(float *, int64_t, const double *, hipStream_t);
template hipError_t launch_sum_partials<double>(const double *, int64_t, double *, hipStream_t);
template hipError_t launch_sum_partials<float>(const float *, int64_t, double *, hipStream_t);
template hipError_t launch_fill<double>(double *, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float *, int64_t, float, hipStream_t);
template hipError_t launch_convert<double, double>(const double *, double *, int64_t, hipStream_t);
template hipError_t launch_convert<float, float>(const float *, float *, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const double *, float *, int64_t, hipStream_t);
template hipError_t launch_convert<double, float>(const float *, double *, int64_t, hipStream_t);

}  // namespace sipg
