// Kernels for elements too large to stage in LDS (order P = 32, n = 33:
// one FP64 element is 287 KB) and for Schwarz subdomains wider than 64 nodes.
//
// Operator: three passes over the level, one per direction, each with one
// thread per 1D line.  The line and the two face-neighbour lines are read from
// global memory; the x pass writes the partial result, the y pass adds to it,
// the z pass completes it (plain apply, residual with optional r.r partials).
//
// Transfers: element-local contraction along one axis of an element tensor of
// shape (s_z, s_y, s_x), one thread per output entry; three calls give
// (J x J x J) or its transpose.
//
// Schwarz for wide subdomains: the same three phases as the slab path, but on
// 2D planes held in LDS and with one thread per output entry, processed in
// batches of rows or columns so that every update is in place without a second
// buffer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

template <typename T, int N, int DIR, int MODE, bool DOT>
__global__ void __launch_bounds__(256)
apply_axis(Mesh g, ApplyTabs<T> tb, const T *__restrict__ u, const T *__restrict__ f, T *out, T *partial) {
  constexpr int N2 = N * N, N3 = N2 * N;
  __shared__ T red[16];
  const int64_t gid = (int64_t)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  const bool active = gid < (int64_t)g.E * N2;
  T dot = 0;
  if (active) {
    const int e = (int)(gid / N2), pq = (int)(gid - (int64_t)e * N2);
    const int p = pq / N, q = pq - p * N;
    const int ex = e % g.ne[0], rest = e / g.ne[0];
    const int ey = rest % g.ne[1], ez = rest / g.ne[1];
    // line base offset and stride inside an element, neighbour elements
    int base, st, eR, eL;
    if (DIR == 0) {
      base = pq * N; st = 1;
      eR = elem_index(g, wrap(ex + 1, g.ne[0]), ey, ez);
      eL = elem_index(g, wrap(ex - 1, g.ne[0]), ey, ez);
    } else if (DIR == 1) {
      base = p * N2 + q; st = N;
      eR = elem_index(g, ex, wrap(ey + 1, g.ne[1]), ez);
      eL = elem_index(g, ex, wrap(ey - 1, g.ne[1]), ez);
    } else {
      base = pq; st = N2;
      eR = elem_index(g, ex, ey, wrap(ez + 1, g.ne[2]));
      eL = elem_index(g, ex, ey, wrap(ez - 1, g.ne[2]));
    }
    const T *__restrict__ Ld = tb.Ld[DIR];
    const T *__restrict__ DL = tb.DL[DIR];
    const T *__restrict__ DR = tb.DR[DIR];
    const T mu = tb.mu[DIR];
    const T *lr = u + (size_t)eR * N3 + base;
    const T *ll = u + (size_t)eL * N3 + base;
    const T *lv = u + (size_t)e * N3 + base;
    const T *__restrict__ TL = tb.TL[DIR];
    const T *__restrict__ TR = tb.TR[DIR];
    const bool gl = tb.gl != 0;
    T v[N];
    T gR = 0, gL = 0, vR = 0, vL = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v[i] = lv[i * st];
      const T r = lr[i * st], l = ll[i * st];
      gR += DL[i] * r;
      gL += DR[i] * l;
      if (gl) {
        vR += TL[i] * r;
        vL += TR[i] * l;
      }
    }
    if (!gl) vR = lr[0], vL = ll[(N - 1) * st];
    // mass factors of the two other directions
    T sc;
    if (DIR == 0) sc = tb.M[2][p] * tb.M[1][q];
    else if (DIR == 1) sc = tb.M[2][p] * tb.M[0][q];
    else sc = tb.M[1][p] * tb.M[0][q];
    T *o = out + (size_t)e * N3 + base;
    const T *fl = f ? f + (size_t)e * N3 + base : nullptr;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = DR[i] * vR - DL[i] * vL;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += Ld[i * N + k] * v[k];
      if (gl) {  // the face terms of the GL basis reach every node of the line
        acc += -TR[i] * (gR + mu * vR) + TL[i] * (gL - mu * vL);
      } else {
        if (i == N - 1) acc -= gR + mu * vR;
        if (i == 0) acc += gL - mu * vL;
      }
      acc *= sc;
      if (DIR == 0) {
        o[i * st] = acc;
      } else if (DIR == 1) {
        o[i * st] += acc;
      } else {
        const T y = o[i * st] + acc;
        if (MODE == 0) {
          o[i * st] = y;
          if (DOT) dot += v[i] * y;
        } else {
          const T r = fl[i * st] - y;
          o[i * st] = r;
          if (DOT) dot += r * r;
        }
      }
    }
  }
  if (DOT) {
    const T s = block_reduce_sum(dot, red);
    if (threadIdx.x == 0) partial[xcd_block(blockIdx.x, gridDim.x)] = s;
  }
}

// out = contraction of each element tensor along `axis`:
//   TRANS = false: out[..o..] = sum_i A[o * nin + i] in[..i..]      (A is nout x nin)
//   TRANS = true : out[..o..] = sum_i A[i * nout + o] in[..i..]     (A is nin x nout)
// in has per-element shape (sz, sy, sx) with the contracted extent nin;
// ADD accumulates into out.
template <typename T, typename TI, bool TRANS, bool ADD>
__global__ void __launch_bounds__(256)
elem_axis(int E, int sx, int sy, int sz, int axis, int nout, const T *__restrict__ A, const TI *__restrict__ in,
          T *out) {
  const int nin = axis == 0 ? sx : (axis == 1 ? sy : sz);
  const int ox = axis == 0 ? nout : sx, oy = axis == 1 ? nout : sy, oz = axis == 2 ? nout : sz;
  const int64_t ovol = (int64_t)ox * oy * oz, ivol = (int64_t)sx * sy * sz;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)E * ovol) return;
  const int e = (int)(gid / ovol);
  const int r = (int)(gid - (int64_t)e * ovol);
  const int x = r % ox, y = (r / ox) % oy, z = r / (ox * oy);
  const int o = axis == 0 ? x : (axis == 1 ? y : z);
  const int istride = axis == 0 ? 1 : (axis == 1 ? sx : sx * sy);
  const int ibase = axis == 0 ? (z * sy + y) * sx : (axis == 1 ? z * sy * sx + x : y * sx + x);
  const TI *src = in + (size_t)e * ivol + ibase;
  T acc = 0;
  for (int i = 0; i < nin; ++i) acc += (TRANS ? A[i * nout + o] : A[o * nin + i]) * (T)src[i * istride];
  if (ADD) out[gid] += acc;
  else out[gid] = acc;
}

// ---- Schwarz on wide subdomains: planes in LDS, one thread per output ----
// In-place contraction of the rows (ROWS = true: rows are contiguous runs of
// length m, `count` of them with pitch `pitch`) or the columns (ROWS = false:
// column j has entries P[k * pitch + j], k < m) of a plane in LDS, processed
// in batches so that every output of a batch is computed before the batch is
// written back: out[o] = sum_a At[a*ld + o] in[a] (S for a forward, (W S)^T
// for a backward contraction).  Each thread computes four consecutive outputs
// of a line, so one read of an input entry feeds four multiply-adds; with the
// table in LDS its rows are padded to ld = m rounded up to 4 (zeros), and the
// four table entries of a step are one aligned vector read.
template <typename T, bool ROWS, bool PADDED>
__device__ void plane_contract(T *P, int pitch, int count, int m, const T *__restrict__ At, int ld) {
  const int nth = blockDim.x, tid = threadIdx.x;
  const int mq = (m + 3) / 4;                // output quads per line
  const int per_batch = max(1, nth / mq);    // lines per batch
  for (int l0 = 0; l0 < count; l0 += per_batch) {
    const int nl = min(per_batch, count - l0);
    T acc[4] = {0, 0, 0, 0};
    const bool act = tid < nl * mq;
    const int line = l0 + tid / mq, o0 = 4 * (tid % mq);
    if (act) {
#pragma unroll 4
      for (int a = 0; a < m; ++a) {
        const T x = ROWS ? P[line * pitch + a] : P[a * pitch + line];
        const T *ar = At + a * ld + o0;
        if constexpr (PADDED) ar = static_cast<const T *>(__builtin_assume_aligned(ar, 4 * sizeof(T)));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (PADDED || o0 + r < m) acc[r] += ar[r] * x;
        }
      }
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + r;
        if (o < m) {
          if (ROWS) P[line * pitch + o] = acc[r];
          else P[o * pitch + line] = acc[r];
        }
      }
    }
    __syncthreads();
  }
}

inline __host__ __device__ int pad4(int m) { return (m + 3) / 4 * 4; }

// The m x m table a wide kernel contracts with: copied into LDS after the
// plane with its rows padded to pad4(m) (TL), or read from global memory.
template <typename T, bool TL>
__device__ __forceinline__ const T *stage_table(T *lds, const T *__restrict__ g, int m) {
  if constexpr (TL) {
    const int ld = pad4(m);
    for (int i = threadIdx.x; i < m * ld; i += blockDim.x) {
      const int a = i / ld, o = i - a * ld;
      lds[i] = o < m ? g[a * m + o] : (T)0;
    }
    return lds;
  } else {
    return g;
  }
}

template <typename T, bool TL, bool ROWS>
__device__ __forceinline__ void contract(T *P, int pitch, int count, int m, const T *At) {
  if constexpr (TL) plane_contract<T, ROWS, true>(P, pitch, count, m, At, pad4(m));
  else plane_contract<T, ROWS, false>(P, pitch, count, m, At, m);
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

template <typename T>
__device__ __forceinline__ T gather_node(const Mesh &g, int n, const T *__restrict__ r, int ex, int ey, int ez,
                                         int gx, int gy, int gz) {
  const int dx = gx < 0 ? -1 : (gx >= n ? 1 : 0);
  const int dy = gy < 0 ? -1 : (gy >= n ? 1 : 0);
  const int dz = gz < 0 ? -1 : (gz >= n ? 1 : 0);
  const int e = elem_index(g, wrap(ex + dx, g.ne[0]), wrap(ey + dy, g.ne[1]), wrap(ez + dz, g.ne[2]));
  return r[(size_t)e * n * n * n + ((gz - dz * n) * n + (gy - dy * n)) * n + (gx - dx * n)];
}

// phase 1: block (s, c): gather the z-slab, x and y forward
template <typename T, bool TL>
__global__ void __launch_bounds__(512)
wide_slab1(Mesh g, int n, SchwarzTabs<T> tb, const T *__restrict__ r, T *__restrict__ W, int ppb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *P = reinterpret_cast<T *>(smem_raw);
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const T *Ax = stage_table<T, TL>(P + pad4(mx * my), tb.S[0], mx);
  const T *Ay = stage_table<T, TL>(P + pad4(mx * my) + mx * pad4(mx), tb.S[1], my);
  const int nchunk = (mz + ppb - 1) / ppb;
  const int blk = blockIdx.x;
  const int s = blk / nchunk, c0 = (blk - s * nchunk) * ppb, c1 = min(mz, c0 + ppb);
  const int ex = s % g.ne[0], rest = s / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  for (int c = c0; c < c1; ++c) {
    if (c > c0) __syncthreads();  // the previous plane has been stored
    batched_copy<T>(
        mx * my, threadIdx.x, blockDim.x,
        [&](int idx) {
          const int a = idx % mx, b = idx / mx;
          return gather_node(g, n, r, ex, ey, ez, a - tb.no[0], b - tb.no[1], c - tb.no[2]);
        },
        [&](int idx, T v) { P[idx] = v; });
    __syncthreads();
    contract<T, TL, true>(P, mx, my, mx, Ax);
    contract<T, TL, false>(P, mx, mx, my, Ay);
    T *Ws = W + ((size_t)s * mz + c) * mx * my;
    batched_copy<T>(
        mx * my, threadIdx.x, blockDim.x, [&](int idx) { return P[idx]; }, [&](int idx, T v) { Ws[idx] = v; });
  }
}

// phase 2: block (s, b): the xz plane, z forward, scaling, z backward
template <typename T, bool TL>
__global__ void __launch_bounds__(512)
wide_slab2(int E, SchwarzTabs<T> tb, const T *__restrict__ ilam, T *__restrict__ W, int ppb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *P = reinterpret_cast<T *>(smem_raw);
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const T *Af = stage_table<T, TL>(P + pad4(mx * mz), tb.S[2], mz);
  const T *Ab = stage_table<T, TL>(P + pad4(mx * mz) + mz * pad4(mz), tb.WST[2], mz);
  const int nchunk = (my + ppb - 1) / ppb;
  const int blk = blockIdx.x;
  const int s = blk / nchunk, b0 = (blk - s * nchunk) * ppb, b1 = min(my, b0 + ppb);
  T *Ws = W + (size_t)s * mx * my * mz;
  for (int b = b0; b < b1; ++b) {
    if (b > b0) __syncthreads();  // the previous plane has been stored
    batched_copy<T>(
        mx * mz, threadIdx.x, blockDim.x,
        [&](int idx) { return Ws[((size_t)(idx / mx) * my + b) * mx + idx % mx]; },
        [&](int idx, T v) { P[idx] = v; });
    __syncthreads();
    contract<T, TL, false>(P, mx, mx, mz, Af);
    batched_copy<T>(
        mx * mz, threadIdx.x, blockDim.x,
        [&](int idx) { return ilam[((size_t)(idx / mx) * my + b) * mx + idx % mx]; },
        [&](int idx, T v) { P[idx] *= v; });
    __syncthreads();
    contract<T, TL, false>(P, mx, mx, mz, Ab);
    batched_copy<T>(
        mx * mz, threadIdx.x, blockDim.x, [&](int idx) { return P[idx]; },
        [&](int idx, T v) { Ws[((size_t)(idx / mx) * my + b) * mx + idx % mx] = v; });
  }
}

// phase 3: block (s, c): y and x backward
template <typename T, bool TL>
__global__ void __launch_bounds__(512) wide_slab3(int E, SchwarzTabs<T> tb, T *__restrict__ W, int ppb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *P = reinterpret_cast<T *>(smem_raw);
  const int mx = tb.m[0], my = tb.m[1], mz = tb.m[2];
  const T *Ay = stage_table<T, TL>(P + pad4(mx * my), tb.WST[1], my);
  const T *Ax = stage_table<T, TL>(P + pad4(mx * my) + my * pad4(my), tb.WST[0], mx);
  const int nchunk = (mz + ppb - 1) / ppb;
  const int blk = blockIdx.x;
  const int s = blk / nchunk, c0 = (blk - s * nchunk) * ppb, c1 = min(mz, c0 + ppb);
  for (int c = c0; c < c1; ++c) {
    if (c > c0) __syncthreads();  // the previous plane has been stored
    T *Ws = W + ((size_t)s * mz + c) * mx * my;
    batched_copy<T>(
        mx * my, threadIdx.x, blockDim.x, [&](int idx) { return Ws[idx]; }, [&](int idx, T v) { P[idx] = v; });
    __syncthreads();
    contract<T, TL, false>(P, mx, mx, my, Ay);
    contract<T, TL, true>(P, mx, my, mx, Ax);
    batched_copy<T>(
        mx * my, threadIdx.x, blockDim.x, [&](int idx) { return P[idx]; }, [&](int idx, T v) { Ws[idx] = v; });
  }
}

inline int nblk(int64_t n) { return (int)((n + 255) / 256); }

template <typename K>
hipError_t allow_lds(K kernel, size_t shm) {
  if (shm <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename T, int N>
hipError_t apply_large_n(const ApplyLaunch<T> &a, T *tmp, hipStream_t st) {
  const int64_t lines = (int64_t)a.mesh.E * N * N;
  const int nb = nblk(lines);
  T *y = (a.mode == APPLY_RESTRICT) ? tmp : a.out;
  apply_axis<T, N, 0, 0, false><<<nb, 256, 0, st>>>(a.mesh, a.tabs, a.u, nullptr, y, nullptr);
  apply_axis<T, N, 1, 0, false><<<nb, 256, 0, st>>>(a.mesh, a.tabs, a.u, nullptr, y, nullptr);
  if (a.mode == APPLY_PLAIN) {
    if (a.partial) apply_axis<T, N, 2, 0, true><<<nb, 256, 0, st>>>(a.mesh, a.tabs, a.u, nullptr, y, a.partial);
    else apply_axis<T, N, 2, 0, false><<<nb, 256, 0, st>>>(a.mesh, a.tabs, a.u, nullptr, y, nullptr);
    return hipGetLastError();
  }
  if (a.partial && a.mode == APPLY_RESID)
    apply_axis<T, N, 2, 1, true><<<nb, 256, 0, st>>>(a.mesh, a.tabs, a.u, a.f, y, a.partial);
  else
    apply_axis<T, N, 2, 1, false><<<nb, 256, 0, st>>>(a.mesh, a.tabs, a.u, a.f, y, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.mode == APPLY_RESID) return e;
  // restriction of the residual in tmp: J^T along x, y, z (J is N x nc)
  const int nc = a.nc, E = a.mesh.E;
  T *t1 = tmp + (size_t)E * N * N * N;  // second half of the scratch
  elem_axis<T, T, true, false><<<nblk((int64_t)E * N * N * nc), 256, 0, st>>>(E, N, N, N, 0, nc, a.J, tmp, t1);
  elem_axis<T, T, true, false><<<nblk((int64_t)E * N * nc * nc), 256, 0, st>>>(E, nc, N, N, 1, nc, a.J, t1, tmp);
  elem_axis<T, T, true, false><<<nblk((int64_t)E * nc * nc * nc), 256, 0, st>>>(E, nc, nc, N, 2, nc, a.J, tmp, a.out);
  return hipGetLastError();
}

}  // namespace

bool apply_is_large(int n) { return n > 17; }

template <typename T>
hipError_t launch_apply_large(const ApplyLaunch<T> &a, T *tmp, hipStream_t st) {
  if (a.n == 33) return apply_large_n<T, 33>(a, tmp, st);
  return hipErrorInvalidValue;
}

int apply_large_num_blocks(int E, int n) { return (int)(((int64_t)E * n * n + 255) / 256); }

template <typename T, typename TC>
hipError_t launch_prolong_large(const ProlongLaunch<T, TC> &a, T *tmp, hipStream_t st) {
  // u_f += (J x J x J) u_c with J nf x nc, through two scratch tensors
  const int E = a.E, nf = a.nf, nc = a.nc;
  T *t1 = tmp, *t2 = tmp + (size_t)E * nc * nc * nf;
  elem_axis<T, TC, false, false><<<nblk((int64_t)E * nc * nc * nf), 256, 0, st>>>(E, nc, nc, nc, 0, nf, a.J, a.uc, t1);
  elem_axis<T, T, false, false><<<nblk((int64_t)E * nc * nf * nf), 256, 0, st>>>(E, nf, nc, nc, 1, nf, a.J, t1, t2);
  elem_axis<T, T, false, true><<<nblk((int64_t)E * nf * nf * nf), 256, 0, st>>>(E, nf, nf, nc, 2, nf, a.J, t2, a.uf);
  return hipGetLastError();
}

bool schwarz_is_wide(const int m[3]) { return std::max(m[0], std::max(m[1], m[2])) > 64; }

template <typename T, bool TL>
hipError_t launch_wide_tl(const SchwarzLaunch<T> &a, size_t s13, size_t s2, hipStream_t st) {
  hipError_t e;
  if ((e = allow_lds(wide_slab1<T, TL>, s13)) != hipSuccess) return e;
  if ((e = allow_lds(wide_slab2<T, TL>, s2)) != hipSuccess) return e;
  if ((e = allow_lds(wide_slab3<T, TL>, s13)) != hipSuccess) return e;
  const int *m = a.tabs.m;
  // planes per workgroup (the tables are staged once per workgroup): as
  // many as keep at least 8192 workgroups, at most 4 (measured on the
  // 23 x 51 x 51 subdomains: 1 plane 15.9 ms, 3 planes 15.3 ms, 6-16 planes
  // slower)
  auto ppb_for = [&](int planes) { return std::max(1, std::min(4, a.mesh.E * planes / 8192)); };
  const int pz = a.wide_planes > 0 ? a.wide_planes : ppb_for(m[2]);
  const int py = a.wide_planes > 0 ? a.wide_planes : ppb_for(m[1]);
  wide_slab1<T, TL><<<a.mesh.E * ((m[2] + pz - 1) / pz), 512, s13, st>>>(a.mesh, a.n, a.tabs, a.r, a.C, pz);
  wide_slab2<T, TL><<<a.mesh.E * ((m[1] + py - 1) / py), 512, s2, st>>>(a.mesh.E, a.tabs, a.ilam, a.C, py);
  wide_slab3<T, TL><<<a.mesh.E * ((m[2] + pz - 1) / pz), 512, s13, st>>>(a.mesh.E, a.tabs, a.C, pz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_schwarz_wide(const SchwarzLaunch<T> &a, hipStream_t st) {
  {
    const hipError_t e = launch_schwarz_wide_mfma<T>(a, st);
    if (e != hipErrorNotSupported) return e;
  }
  const int *m = a.tabs.m;
  const size_t e = sizeof(T);
  const size_t p13 = (size_t)m[0] * m[1] * e, p2 = (size_t)m[0] * m[2] * e;
  if (std::max(p13, p2) > 150 * 1024) return hipErrorInvalidValue;
  // with the padded tables: x and y (phases 1 and 3), z forward and
  // backward (phase 2); the plane offset of the tables stays 16-byte aligned
  const size_t t13 = ((size_t)pad4(m[0] * m[1]) + (size_t)m[0] * pad4(m[0]) + (size_t)m[1] * pad4(m[1])) * e;
  const size_t t2 = ((size_t)pad4(m[0] * m[2]) + 2 * (size_t)m[2] * pad4(m[2])) * e;
  if (std::max(t13, t2) <= 150 * 1024) return launch_wide_tl<T, true>(a, t13, t2, st);
  return launch_wide_tl<T, false>(a, p13, p2, st);
}

template hipError_t launch_apply_large<double>(const ApplyLaunch<double> &, double *, hipStream_t);
template hipError_t launch_apply_large<float>(const ApplyLaunch<float> &, float *, hipStream_t);
template hipError_t launch_prolong_large<double, double>(const ProlongLaunch<double, double> &, double *,
                                                         hipStream_t);
template hipError_t launch_prolong_large<float, float>(const ProlongLaunch<float, float> &, float *, hipStream_t);
template hipError_t launch_prolong_large<float, double>(const ProlongLaunch<float, double> &, float *,
                                                        hipStream_t);
template hipError_t launch_schwarz_wide<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz_wide<float>(const SchwarzLaunch<float> &, hipStream_t);

}  // namespace sipg
