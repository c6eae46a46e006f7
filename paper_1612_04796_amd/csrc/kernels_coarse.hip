// Level-0 coarse solve u_0 = A_0^+ f_0 (Algorithm 1, coarse grid solution).
//
// On the periodic Cartesian mesh A_0 is itself a Kronecker sum of the global
// 1D pairs (L_d, M_d) of order 1 (2 ne_d nodes per direction), so its
// minimum-norm pseudo-inverse is a global fast diagonalization:
//   f <- f - mean(f)                      (projection onto range(A_0))
//   u  = (Sz x Sy x Sx) Lambda^+ (Sz^T x Sy^T x Sx^T) f,   u <- u - mean(u)
// with Lambda^+ zero on the single zero mode.  The mean of f is removed after
// the forward transform, using the column sums cs_d of S_d:
//   (S^T x S^T x S^T)(f - m 1) = (S^T x S^T x S^T) f - m cs_z x cs_y x cs_x.
// The contractions run one axis per kernel over global arrays in
// lexicographic order (z, y, x); the level-0 vector is small (8 E values), so
// these kernels are latency-bound.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

struct Dims {
  int N[3];
  int ne[3];
};

// element-major index of lexicographic node (gx, gy, gz) at order 1
__device__ __forceinline__ int64_t elem_major_p1(const Dims &d, int gx, int gy, int gz) {
  const int e = ((gz >> 1) * d.ne[1] + (gy >> 1)) * d.ne[0] + (gx >> 1);
  return (int64_t)e * 8 + ((gz & 1) * 2 + (gy & 1)) * 2 + (gx & 1);
}

// out = contraction of `in` along AXIS with A (N_axis x N_axis):
//   FWD: out[..o..] = sum_c A[c*Na + o] in[..c..]
//   BWD: out[..o..] = sum_c A[o*Na + c] in[..c..]
// IN_ELEM / OUT_ELEM select element-major order for the input / output.
template <typename TI, int AXIS, bool FWD, bool IN_ELEM, bool OUT_ELEM>
__global__ void __launch_bounds__(256)
coarse_axis(Dims d, const double *__restrict__ A, const TI *__restrict__ in, double *__restrict__ out) {
  const int64_t N0 = (int64_t)d.N[0] * d.N[1] * d.N[2];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N0) return;
  int x = (int)(t % d.N[0]);
  int y = (int)((t / d.N[0]) % d.N[1]);
  int z = (int)(t / ((int64_t)d.N[0] * d.N[1]));
  const int Na = d.N[AXIS];
  const int o = AXIS == 0 ? x : (AXIS == 1 ? y : z);
  double acc = 0.0;
  for (int c = 0; c < Na; ++c) {
    const int xx = AXIS == 0 ? c : x, yy = AXIS == 1 ? c : y, zz = AXIS == 2 ? c : z;
    const int64_t ii = IN_ELEM ? elem_major_p1(d, xx, yy, zz)
                               : ((int64_t)zz * d.N[1] + yy) * d.N[0] + xx;
    const double a = FWD ? A[c * Na + o] : A[o * Na + c];
    acc += a * (double)in[ii];
  }
  out[OUT_ELEM ? elem_major_p1(d, x, y, z) : t] = acc;
}

// z forward transform, then the mean correction and Lambda^+ scaling
__global__ void __launch_bounds__(256)
coarse_z_scale(Dims d, CoarseLaunch c, const double *__restrict__ in, double *__restrict__ out) {
  const int64_t N0 = (int64_t)d.N[0] * d.N[1] * d.N[2];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N0) return;
  const int x = (int)(t % d.N[0]);
  const int y = (int)((t / d.N[0]) % d.N[1]);
  const int z = (int)(t / ((int64_t)d.N[0] * d.N[1]));
  const int Nz = d.N[2];
  const double *Sz = c.S[2];
  double acc = 0.0;
  for (int k = 0; k < Nz; ++k) acc += Sz[k * Nz + z] * in[((int64_t)k * d.N[1] + y) * d.N[0] + x];
  const double mean = c.scalars[0];
  acc -= mean * c.colsum[2][z] * c.colsum[1][y] * c.colsum[0][x];
  const bool zero = (x == c.zero[0] && y == c.zero[1] && z == c.zero[2]);
  out[t] = zero ? 0.0 : acc / (c.lam[0][x] + c.lam[1][y] + c.lam[2][z]);
}

template <typename T>
__global__ void __launch_bounds__(256)
sum_partials(const T *__restrict__ x, int64_t n, double *__restrict__ partial) {
  __shared__ double red[16];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = chunk * blockIdx.x;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += (double)x[i];
  s = block_reduce_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

}  // namespace

template <typename TI>
hipError_t launch_coarse(const CoarseLaunch &c, const TI *f0, double *u0, bool subtract_mean,
                         hipStream_t st) {
  Dims d;
  for (int i = 0; i < 3; ++i) {
    d.N[i] = c.N[i];
    d.ne[i] = c.ne[i];
  }
  const int64_t N0 = (int64_t)d.N[0] * d.N[1] * d.N[2];
  const int nb = (int)((N0 + 255) / 256);
  hipError_t e;
  sum_partials<TI><<<kCoarsePartials, 256, 0, st>>>(f0, N0, c.partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_finalize(c.partial, kCoarsePartials, 1.0 / (double)N0, c.scalars + 0, st)) != hipSuccess)
    return e;
  coarse_axis<TI, 0, true, true, false><<<nb, 256, 0, st>>>(d, c.S[0], f0, c.t0);
  coarse_axis<double, 1, true, false, false><<<nb, 256, 0, st>>>(d, c.S[1], c.t0, c.t1);
  coarse_z_scale<<<nb, 256, 0, st>>>(d, c, c.t1, c.t0);
  coarse_axis<double, 2, false, false, false><<<nb, 256, 0, st>>>(d, c.S[2], c.t0, c.t1);
  coarse_axis<double, 1, false, false, false><<<nb, 256, 0, st>>>(d, c.S[1], c.t1, c.t0);
  coarse_axis<double, 0, false, false, true><<<nb, 256, 0, st>>>(d, c.S[0], c.t0, u0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  sum_partials<double><<<kCoarsePartials, 256, 0, st>>>(u0, N0, c.partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_finalize(c.partial, kCoarsePartials, 1.0 / (double)N0, c.scalars + 1, st)) != hipSuccess)
    return e;
  if (subtract_mean) return launch_sub_scalar<double>(u0, N0, c.scalars + 1, st);
  return hipSuccess;
}

template hipError_t launch_coarse<double>(const CoarseLaunch &, const double *, double *, bool, hipStream_t);
template hipError_t launch_coarse<float>(const CoarseLaunch &, const float *, double *, bool, hipStream_t);

}  // namespace sipg
