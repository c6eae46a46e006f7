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

template <typename T>
__global__ void __launch_bounds__(256)
dot_partials(const T *__restrict__ x, const T *__restrict__ y, int64_t n, double *__restrict__ partial) {
  __shared__ double red[16];
  int64_t lo, hi;
  chunk_of(n, lo, hi);
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += (double)x[i] * (double)y[i];
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

template <typename T>
__global__ void __launch_bounds__(256)
dot2_partials(const T *__restrict__ x, const T *__restrict__ y, const T *__restrict__ z,
              const T *__restrict__ w, int64_t n, double *__restrict__ partial) {
  __shared__ double red[16];
  int64_t lo, hi;
  chunk_of(n, lo, hi);
  double s = 0.0, t = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    s += (double)x[i] * (double)y[i];
    t += (double)z[i] * (double)w[i];
  }
  s = block_reduce_sum(s, red);
  __syncthreads();
  t = block_reduce_sum(t, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    partial[gridDim.x + blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(1024)
finalize_kernel(const double *__restrict__ partial, int np, double scale, double *__restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  s = block_reduce_sum(s, red);
  if (threadIdx.x == 0) out[0] = scale * s;
}

template <typename T>
__global__ void __launch_bounds__(256) sub_scalar(T *__restrict__ y, int64_t n, const double *__restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)((double)y[i] - s[0]);
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

__global__ void __launch_bounds__(256)
fcg_xr_kernel(double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
              const double *__restrict__ q, int64_t n, double *s, double *__restrict__ partial) {
  __shared__ double red[16];
  const double alpha = s[FS_RZ] / s[FS_PQ];
  int64_t lo, hi;
  chunk_of(n, lo, hi);
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  acc = block_reduce_sum(acc, red);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = acc;
    if (blockIdx.x == 0) s[FS_ALPHA] = alpha;
  }
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

__global__ void __launch_bounds__(256)
fcg_p_kernel(double *__restrict__ p, const double *__restrict__ z, int64_t n, const double *__restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + s[FS_BETA] * p[i];
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

template <typename T>
hipError_t launch_dot_partials(const T *x, const T *y, int64_t n, double *partial, hipStream_t st) {
  dot_partials<T><<<kDotBlocks, 256, 0, st>>>(x, y, n, partial);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sum_partials(const T *x, int64_t n, double *partial, hipStream_t st) {
  sum_partials_kernel<T><<<kDotBlocks, 256, 0, st>>>(x, n, partial);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dot2_partials(const T *x, const T *y, const T *z, const T *w, int64_t n,
                                double *partial, hipStream_t st) {
  dot2_partials<T><<<kDotBlocks, 256, 0, st>>>(x, y, z, w, n, partial);
  return hipGetLastError();
}

hipError_t launch_finalize(const double *partial, int np, double scale, double *out, hipStream_t st) {
  finalize_kernel<<<1, 1024, 0, st>>>(partial, np, scale, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sub_scalar(T *y, int64_t n, const double *s, hipStream_t st) {
  if (n == 0) return hipSuccess;
  sub_scalar<T><<<nblocks(n), 256, 0, st>>>(y, n, s);
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

hipError_t launch_fcg_xr(double *x, double *r, const double *p, const double *q, int64_t n, double *s,
                         double *partial, hipStream_t st) {
  fcg_xr_kernel<<<kDotBlocks, 256, 0, st>>>(x, r, p, q, n, s, partial);
  return hipGetLastError();
}

hipError_t launch_fcg_finalize2(const double *partial, double *s, hipStream_t st) {
  fcg_finalize2_kernel<<<1, 1024, 0, st>>>(partial, s);
  return hipGetLastError();
}

hipError_t launch_fcg_p(double *p, const double *z, int64_t n, double *s, hipStream_t st) {
  fcg_p_kernel<<<nblocks(n), 256, 0, st>>>(p, z, n, s);
  return hipGetLastError();
}

hipError_t launch_rhs(const RhsLaunch &a, double *b, hipStream_t st) {
  const int64_t n = (int64_t)a.mesh.E * a.n * a.n * a.n;
  rhs_kernel<<<nblocks(n), 256, 0, st>>>(a, b);
  return hipGetLastError();
}

template hipError_t launch_dot_partials<double>(const double *, const double *, int64_t, double *, hipStream_t);
template hipError_t launch_dot_partials<float>(const float *, const float *, int64_t, double *, hipStream_t);
template hipError_t launch_dot2_partials<double>(const double *, const double *, const double *,
                                                 const double *, int64_t, double *, hipStream_t);
template hipError_t launch_sub_scalar<double>(double *, int64_t, const double *, hipStream_t);
template hipError_t launch_sub_scalar<float>(float *, int64_t, const double *, hipStream_t);
template hipError_t launch_sum_partials<double>(const double *, int64_t, double *, hipStream_t);
template hipError_t launch_sum_partials<float>(const float *, int64_t, double *, hipStream_t);
template hipError_t launch_fill<double>(double *, int64_t, double, hipStream_t);
template hipError_t launch_fill<float>(float *, int64_t, float, hipStream_t);
template hipError_t launch_convert<double, double>(const double *, double *, int64_t, hipStream_t);
template hipError_t launch_convert<float, double>(const double *, float *, int64_t, hipStream_t);
template hipError_t launch_convert<double, float>(const float *, double *, int64_t, hipStream_t);

}  // namespace sipg
