// Weighted overlapping additive Schwarz correction (Sec. 3.1):
//   du = sum_s R_s^T W_s (Sz x Sy x Sx) [ (Sz^T x Sy^T x Sx^T) R_s r
//                                          / (lam_z + lam_y + lam_x) ]
// with W_s = Wz x Wy x Wx folded into WS_d = diag(w_d) S_d.
//
// Phase 1 computes, for every element-centred subdomain, its weighted local
// correction C[s] (m_x*m_y*m_z values, layout [c][b][a], x fastest) from the
// gathered residual.  When the subdomain tensor fits LDS this is one
// workgroup per subdomain: gather, three forward contractions, scaling, three
// backward contractions, all in LDS with one thread per 1D line.  Larger
// subdomains (the enlarged overlap of anisotropic meshes) use three kernels:
// (x,y) forward per z-slab in LDS, z forward/scale/backward per line in
// global memory, (y,x) backward per z-slab in LDS.
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
  for (int idx = tid; idx < mxyz; idx += nth) {
    const int a = idx % mx, bc = idx / mx, b = bc % my, c = bc / my;
    t[bc * RX + a] = gather_r(g, n, r, ex, ey, ez, a - tb.no[0], b - tb.no[1], c - tb.no[2]);
  }
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
  for (int idx = tid; idx < mxyz; idx += nth) {
    const int a = idx % mx, bc = idx / mx;
    Cs[idx] = t[bc * RX + a];
  }
}

// slab phase 1: block (s, c): gather the z-slab c of subdomain s, x and y forward
template <typename T, int MB>
__global__ void __launch_bounds__(256)
schwarz_slab1(Mesh g, int n, SchwarzTabs<T> tb, const T *__restrict__ r, T *__restrict__ W) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *t = reinterpret_cast<T *>(smem_raw);
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const int RX = mx | 1;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int s = blk / mz, c = blk - s * mz;
  const int ex = s % g.ne[0], rest = s / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int mxy = mx * my;
  for (int idx = tid; idx < mxy; idx += nth) {
    const int a = idx % mx, b = idx / mx;
    t[b * RX + a] = gather_r(g, n, r, ex, ey, ez, a - tb.no[0], b - tb.no[1], c - tb.no[2]);
  }
  __syncthreads();
  for (int L = tid; L < my; L += nth) line_fwd<T, MB>(t + L * RX, 1, mx, tb.S[0]);
  __syncthreads();
  for (int L = tid; L < mx; L += nth) line_fwd<T, MB>(t + L, RX, my, tb.S[1]);
  __syncthreads();
  T *Ws = W + ((size_t)s * mz + c) * mxy;
  for (int idx = tid; idx < mxy; idx += nth) Ws[idx] = t[(idx / mx) * RX + idx % mx];
}

// slab phase 2: one thread per z line (s, b, a) in global memory
template <typename T, int MB>
__global__ void __launch_bounds__(256)
schwarz_slab2(int E, SchwarzTabs<T> tb, T *__restrict__ W) {
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const int mxy = mx * my;
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= (int64_t)E * mxy) return;
  const int s = (int)(t / mxy), ab = (int)(t - (int64_t)s * mxy);
  const int a = ab % mx, b = ab / mx;
  line_z<T, MB>(W + (size_t)s * mxy * mz + ab, mxy, mz, tb.S[2], tb.WS[2], tb.lam[2],
                tb.lam[0][a] + tb.lam[1][b]);
}

// slab phase 3: block (s, c): y and x backward on the z-slab, in place
template <typename T, int MB>
__global__ void __launch_bounds__(256)
schwarz_slab3(int E, SchwarzTabs<T> tb, T *__restrict__ W) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *t = reinterpret_cast<T *>(smem_raw);
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const int RX = mx | 1;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int s = blk / mz, c = blk - s * mz;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int mxy = mx * my;
  T *Ws = W + ((size_t)s * mz + c) * mxy;
  for (int idx = tid; idx < mxy; idx += nth) t[(idx / mx) * RX + idx % mx] = Ws[idx];
  __syncthreads();
  for (int L = tid; L < mx; L += nth) line_bwd<T, MB>(t + L, RX, my, tb.WS[1]);
  __syncthreads();
  for (int L = tid; L < my; L += nth) line_bwd<T, MB>(t + L * RX, 1, mx, tb.WS[0]);
  __syncthreads();
  for (int idx = tid; idx < mxy; idx += nth) Ws[idx] = t[(idx / mx) * RX + idx % mx];
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
  T sum = 0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int c = k - dz * n + tb.no[2];
    if (c < 0 || c >= mz) continue;
    const int sz = wrap(ez + dz, g.ne[2]);
    for (int dy = -1; dy <= 1; ++dy) {
      const int b = j - dy * n + tb.no[1];
      if (b < 0 || b >= my) continue;
      const int sy = wrap(ey + dy, g.ne[1]);
      for (int dx = -1; dx <= 1; ++dx) {
        const int a = i - dx * n + tb.no[0];
        if (a < 0 || a >= mx) continue;
        const int sx = wrap(ex + dx, g.ne[0]);
        sum += C[(size_t)elem_index(g, sx, sy, sz) * mxyz + (c * my + b) * mx + a];
      }
    }
  }
  u_out[idx] = (u_in ? u_in[idx] : (T)0) + sum;
}

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

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

template <typename T, int MB>
hipError_t launch_slab(const SchwarzLaunch<T> &a, hipStream_t st) {
  const int *m = a.tabs.m;
  const size_t shm = (size_t)m[1] * (m[0] | 1) * sizeof(T);
  const int nslab = a.mesh.E * m[2];
  schwarz_slab1<T, MB><<<nslab, 256, shm, st>>>(a.mesh, a.n, a.tabs, a.r, a.C);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t nl = (int64_t)a.mesh.E * m[0] * m[1];
  schwarz_slab2<T, MB><<<(int)((nl + 255) / 256), 256, 0, st>>>(a.mesh.E, a.tabs, a.C);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  schwarz_slab3<T, MB><<<nslab, 256, shm, st>>>(a.mesh.E, a.tabs, a.C);
  return hipGetLastError();
}

}  // namespace

bool schwarz_fits_lds(const int m[3], size_t eb) {
  return lds_bytes(m, eb) <= kLdsLimit && std::max(m[0], std::max(m[1], m[2])) <= 32;
}

template <typename T>
hipError_t launch_schwarz_local(const SchwarzLaunch<T> &a, hipStream_t st) {
  const int *m = a.tabs.m;
  const int mmax = std::max(m[0], std::max(m[1], m[2]));
  if (schwarz_fits_lds(m, sizeof(T))) {
    if (mmax <= 8) return launch_lds<T, 8>(a, st);
    if (mmax <= 16) return launch_lds<T, 16>(a, st);
    if (mmax <= 24) return launch_lds<T, 24>(a, st);
    return launch_lds<T, 32>(a, st);
  }
  if (mmax <= 32) return launch_slab<T, 32>(a, st);
  if (mmax <= 64) return launch_slab<T, 64>(a, st);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_schwarz_assemble(const SchwarzLaunch<T> &a, hipStream_t st) {
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

template hipError_t launch_schwarz<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz<float>(const SchwarzLaunch<float> &, hipStream_t);
template hipError_t launch_schwarz_local<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz_local<float>(const SchwarzLaunch<float> &, hipStream_t);
template hipError_t launch_schwarz_assemble<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz_assemble<float>(const SchwarzLaunch<float> &, hipStream_t);

}  // namespace sipg
