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
//
// Three kernels on 2D planes held in LDS, with the 1D eigenvector tables in
// LDS too when they fit (lexicographic (z, y, x) order); when the planes are
// few, each plane is shared by several workgroups (split kernels below):
//   1. per z plane: x and y forward from the element-major f_0; plane sums
//   2. per y plane: z forward, mean correction, Lambda^+, z backward
//   3. per z plane: y and x backward into the element-major u_0; plane sums
// The mean of u_0 is then either removed by two small kernels or, inside the
// V-cycle, by the prolongation, which reduces the plane sums itself.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

struct Dims {
  int N[3];
  int ne[3];
};

__device__ __forceinline__ int64_t elem_major_p1(const Dims &d, int gx, int gy, int gz) {
  const int e = ((gz >> 1) * d.ne[1] + (gy >> 1)) * d.ne[0] + (gx >> 1);
  return (int64_t)e * 8 + ((gz & 1) * 2 + (gy & 1)) * 2 + (gx & 1);
}

// In-place contraction of a 2D tile P[r * pitch + q] in LDS along one of its
// axes, with a 2D workgroup (blockDim.x >= pitch, so threadIdx.x is the q
// index).  ALONG_Q contracts the rows (over q, n = pitch), else the columns
// (over r, n = number of rows).  All inputs are read before any output is
// written (two barriers).
//   FWD: out[o] = sum_a A[a*n + o] in[a];  else out[o] = sum_a A[o*n + a] in[a]
template <bool ALONG_Q, bool FWD>
__device__ void tile_contract(double *P, double *W, int pitch, int rows, const double *A) {
  const int q = threadIdx.x;
  const int n = ALONG_Q ? pitch : rows;
  if (q < pitch) {
    for (int r = threadIdx.y; r < rows; r += blockDim.y) {
      // ALONG_Q: output (r, o = q) from row r; else output (o = r, q) from column q
      const int o = ALONG_Q ? q : r;
      double acc = 0.0;
#pragma unroll 8
      for (int a = 0; a < n; ++a) {
        const double x = ALONG_Q ? P[r * pitch + a] : P[a * pitch + q];
        acc += (FWD ? A[a * n + o] : A[o * n + a]) * x;
      }
      W[r * pitch + q] = acc;
    }
  }
  __syncthreads();
  if (q < pitch)
    for (int r = threadIdx.y; r < rows; r += blockDim.y) P[r * pitch + q] = W[r * pitch + q];
  __syncthreads();
}

// for (i = i0; i < tot; i += step) put(i, get(i)), the loads of four
// consecutive iterations issued before any of their values is stored
template <typename Get, typename Put>
__device__ __forceinline__ void copy4(int i0, int tot, int step, Get get, Put put) {
  for (int b = i0; b < tot; b += 4 * step) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = b + k * step;
      v[k] = i < tot ? get(i) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int i = b + k * step;
      if (i < tot) put(i, v[k]);
    }
  }
}

__device__ __forceinline__ int flat_tid() { return threadIdx.y * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int flat_nth() { return blockDim.x * blockDim.y; }

// block_reduce_sum over a 2D workgroup (flat thread order)
__device__ double block_sum_2d(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int t = flat_tid(), w = t >> 6, nw = (flat_nth() + 63) >> 6;
  if ((t & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int i = 0; i < nw; ++i) s += red[i];
  return s;  // valid in thread 0
}

// 1. one workgroup per z plane: the (y, x) plane of f_0 (and Sx, Sy) in LDS;
//    x and y forward; the plane sum of f_0 -> partial[z]
template <typename TI, bool TL>
__global__ void __launch_bounds__(1024)
coarse_plane_xy_fwd(Dims d, CoarseLaunch c, const TI *__restrict__ f0, double *__restrict__ t) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int Nx = d.N[0], Ny = d.N[1];
  double *P = reinterpret_cast<double *>(smem_raw);
  double *W = P + Nx * Ny;
  const double *Sx = c.S[0], *Sy = c.S[1];
  const int tid = flat_tid(), nth = flat_nth();
  if (TL) {
    double *sx = W + Nx * Ny, *sy = sx + Nx * Nx;
    copy4(tid, Nx * Nx, nth, [&](int i) { return c.S[0][i]; }, [&](int i, double v) { sx[i] = v; });
    copy4(tid, Ny * Ny, nth, [&](int i) { return c.S[1][i]; }, [&](int i, double v) { sy[i] = v; });
    Sx = sx;
    Sy = sy;
  }
  const int z = blockIdx.x;
  double s = 0.0;
  if (threadIdx.x < Nx)
    copy4(threadIdx.y, Ny, blockDim.y, [&](int y) { return (double)f0[elem_major_p1(d, threadIdx.x, y, z)]; },
          [&](int y, double v) {
            P[y * Nx + threadIdx.x] = v;
            s += v;
          });
  s = block_sum_2d(s, red);
  if (tid == 0) c.partial[z] = s;
  __syncthreads();
  tile_contract<true, true>(P, W, Nx, Ny, Sx);
  tile_contract<false, true>(P, W, Nx, Ny, Sy);
  double *tz = t + (size_t)z * Nx * Ny;
  for (int i = tid; i < Nx * Ny; i += nth) tz[i] = P[i];
}

// 2. one workgroup per y plane: the (z, x) plane (and Sz) in LDS; z forward,
//    mean correction (mean from the plane sums), Lambda^+, z backward
template <bool TL>
__global__ void __launch_bounds__(1024) coarse_plane_z(Dims d, CoarseLaunch c, double *__restrict__ t) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  __shared__ double mean_sh;
  const int Nx = d.N[0], Ny = d.N[1], Nz = d.N[2];
  double *P = reinterpret_cast<double *>(smem_raw);
  double *W = P + Nx * Nz;
  const double *Sz = c.S[2];
  const int tid = flat_tid(), nth = flat_nth();
  if (TL) {
    double *sz = W + Nx * Nz;
    copy4(tid, Nz * Nz, nth, [&](int i) { return c.S[2][i]; }, [&](int i, double v) { sz[i] = v; });
    Sz = sz;
  }
  const int y = blockIdx.x;
  if (threadIdx.x < Nx)
    copy4(threadIdx.y, Nz, blockDim.y, [&](int z) { return t[((size_t)z * Ny + y) * Nx + threadIdx.x]; },
          [&](int z, double v) { P[z * Nx + threadIdx.x] = v; });
  double s = 0.0;
  for (int i = tid; i < Nz; i += nth) s += c.partial[i];
  // the 1D eigenvalues and column sums the scaling needs, loaded before the
  // reductions and contractions (their latency hides behind them)
  const int x = threadIdx.x;
  const bool lane = x < Nx;
  const double cxy = lane ? c.colsum[0][x] * c.colsum[1][y] : 0.0;
  const double lxy = lane ? c.lam[0][x] + c.lam[1][y] : 1.0;
  double cz[4], lz[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int o = threadIdx.y + k * blockDim.y;
    cz[k] = o < Nz ? c.colsum[2][o] : 0.0;
    lz[k] = o < Nz ? c.lam[2][o] : 0.0;
  }
  s = block_sum_2d(s, red);
  if (tid == 0) mean_sh = s / ((double)Nx * Ny * Nz);
  __syncthreads();
  tile_contract<false, true>(P, W, Nx, Nz, Sz);
  const double mean = mean_sh;
  auto scale = [&](int o, double czo, double lzo) {
    const double v = P[o * Nx + x] - mean * czo * cxy;
    const bool zero = (x == c.zero[0] && y == c.zero[1] && o == c.zero[2]);
    P[o * Nx + x] = zero ? 0.0 : v / (lxy + lzo);
  };
  if (lane) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int o = threadIdx.y + k * blockDim.y;
      if (o < Nz) scale(o, cz[k], lz[k]);
    }
    for (int o = threadIdx.y + 4 * blockDim.y; o < Nz; o += blockDim.y) scale(o, c.colsum[2][o], c.lam[2][o]);
  }
  __syncthreads();
  tile_contract<false, false>(P, W, Nx, Nz, Sz);
  if (threadIdx.x < Nx)
    for (int z = threadIdx.y; z < Nz; z += blockDim.y) t[((size_t)z * Ny + y) * Nx + threadIdx.x] = P[z * Nx + threadIdx.x];
}

// 3. one workgroup per z plane: y and x backward into the element-major u_0;
//    the plane sum of u_0 -> partial_u[z]
template <bool TL>
__global__ void __launch_bounds__(1024)
coarse_plane_xy_bwd(Dims d, CoarseLaunch c, const double *__restrict__ t, double *__restrict__ u0) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int Nx = d.N[0], Ny = d.N[1];
  double *P = reinterpret_cast<double *>(smem_raw);
  double *W = P + Nx * Ny;
  const double *Sx = c.S[0], *Sy = c.S[1];
  const int tid = flat_tid(), nth = flat_nth();
  if (TL) {
    // Sx is stored transposed so that the x backward reads it along
    // consecutive addresses (no LDS bank conflicts)
    double *sxt = W + Nx * Ny, *sy = sxt + Nx * Nx;
    copy4(tid, Nx * Nx, nth, [&](int i) { return c.S[0][i]; },
          [&](int i, double v) { sxt[(i % Nx) * Nx + i / Nx] = v; });
    copy4(tid, Ny * Ny, nth, [&](int i) { return c.S[1][i]; }, [&](int i, double v) { sy[i] = v; });
    Sx = sxt;
    Sy = sy;
  }
  const int z = blockIdx.x;
  const double *tz = t + (size_t)z * Nx * Ny;
  copy4(tid, Nx * Ny, nth, [&](int i) { return tz[i]; }, [&](int i, double v) { P[i] = v; });
  __syncthreads();
  tile_contract<false, false>(P, W, Nx, Ny, Sy);
  if (TL) tile_contract<true, true>(P, W, Nx, Ny, Sx);  // (Sx^T)^T = Sx
  else tile_contract<true, false>(P, W, Nx, Ny, Sx);
  double s = 0.0;
  if (threadIdx.x < Nx)
    for (int y = threadIdx.y; y < Ny; y += blockDim.y) {
      const double v = P[y * Nx + threadIdx.x];
      u0[elem_major_p1(d, threadIdx.x, y, z)] = v;
      s += v;
    }
  s = block_sum_2d(s, red);
  if (tid == 0) c.partial_u[z] = s;
}

// ---- split plane kernels: np workgroups share a plane ------------------------
// With one workgroup per plane only 2 ne_d workgroups run (32 or 64 at the
// 16^3 and 32^3 meshes) and most CUs idle.  Here each plane is shared by np
// workgroups: the forward xy pass splits the plane's output columns (every
// part reads the whole input plane, contracts x for its columns only, then y
// on them), the z pass splits the columns of its (z, x) plane, the backward
// xy pass splits the output rows (y backward for its rows, then x).  Tables
// (and transposed copies where a contraction runs along a table row) are
// staged in LDS; LDS row pitches are odd so that rows read by one wavefront
// fall on different banks.  1024 threads per workgroup, outputs flat over
// the threads.

template <typename TI>
__global__ void __launch_bounds__(1024)
coarse_split_xy_fwd(Dims d, CoarseLaunch c, const TI *__restrict__ f0, double *__restrict__ t, int np) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int Nx = d.N[0], Ny = d.N[1], px = Nx + 1;
  const int z = blockIdx.x, part = blockIdx.y;
  const int cw = (Nx + np - 1) / np, x0 = part * cw, nx = min(cw, Nx - x0), pw = cw + 1;
  double *P = reinterpret_cast<double *>(smem_raw);  // Ny x px: input plane
  double *W = P + Ny * px;                            // Ny x pw: after x
  double *sx = W + Ny * pw, *sy = sx + Nx * Nx;
  const int tid = threadIdx.x, nth = blockDim.x;
  copy4(tid, Nx * Nx, nth, [&](int i) { return c.S[0][i]; }, [&](int i, double v) { sx[i] = v; });
  copy4(tid, Ny * Ny, nth, [&](int i) { return c.S[1][i]; }, [&](int i, double v) { sy[i] = v; });
  double s = 0.0;
  copy4(tid, Nx * Ny, nth,
        [&](int i) {
          const int y = i / Nx;
          return (double)f0[elem_major_p1(d, i - y * Nx, y, z)];
        },
        [&](int i, double v) {
          const int y = i / Nx;
          P[y * px + i - y * Nx] = v;
          s += v;
        });
  s = block_sum_2d(s, red);
  if (tid == 0 && part == 0) c.partial[z] = s;
  __syncthreads();
  for (int i = tid; i < Ny * nx; i += nth) {  // x forward on columns x0 .. x0 + nx
    const int y = i / nx, j = i - y * nx;
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < Nx; ++a) acc += sx[a * Nx + x0 + j] * P[y * px + a];
    W[y * pw + j] = acc;
  }
  __syncthreads();
  for (int i = tid; i < Ny * nx; i += nth) {  // y forward
    const int yo = i / nx, j = i - yo * nx;
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < Ny; ++a) acc += sy[a * Ny + yo] * W[a * pw + j];
    t[((size_t)z * Ny + yo) * Nx + x0 + j] = acc;
  }
}

__global__ void __launch_bounds__(1024) coarse_split_z(Dims d, CoarseLaunch c, double *__restrict__ t, int np) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  __shared__ double mean_sh;
  const int Nx = d.N[0], Ny = d.N[1], Nz = d.N[2];
  const int y = blockIdx.x, part = blockIdx.y;
  const int cw = (Nx + np - 1) / np, x0 = part * cw, nx = min(cw, Nx - x0), pw = cw + 1;
  double *P = reinterpret_cast<double *>(smem_raw);  // Nz x pw
  double *W = P + Nz * pw;                            // Nz x pw
  double *sz = W + Nz * pw, *szt = sz + Nz * Nz;     // Sz and its transpose
  const int tid = threadIdx.x, nth = blockDim.x;
  copy4(tid, Nz * Nz, nth, [&](int i) { return c.S[2][i]; }, [&](int i, double v) {
    sz[i] = v;
    szt[(i % Nz) * Nz + i / Nz] = v;
  });
  copy4(tid, Nz * nx, nth, [&](int i) {
    const int zz = i / nx;
    return t[((size_t)zz * Ny + y) * Nx + x0 + i - zz * nx];
  }, [&](int i, double v) {
    const int zz = i / nx;
    P[zz * pw + i - zz * nx] = v;
  });
  double s = 0.0;
  for (int i = tid; i < Nz; i += nth) s += c.partial[i];
  s = block_sum_2d(s, red);
  if (tid == 0) mean_sh = s / ((double)Nx * Ny * Nz);
  __syncthreads();
  const double mean = mean_sh;
  const double cy = c.colsum[1][y], ly = c.lam[1][y];
  for (int i = tid; i < Nz * nx; i += nth) {  // z forward, mean correction, Lambda^+
    const int o = i / nx, j = i - o * nx, x = x0 + j;
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < Nz; ++a) acc += sz[a * Nz + o] * P[a * pw + j];
    const double cxy = c.colsum[0][x] * cy, lxy = c.lam[0][x] + ly;
    const double v = acc - mean * c.colsum[2][o] * cxy;
    const bool zero = (x == c.zero[0] && y == c.zero[1] && o == c.zero[2]);
    W[o * pw + j] = zero ? 0.0 : v / (lxy + c.lam[2][o]);
  }
  __syncthreads();
  for (int i = tid; i < Nz * nx; i += nth) {  // z backward
    const int o = i / nx, j = i - o * nx;
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < Nz; ++a) acc += szt[a * Nz + o] * W[a * pw + j];
    t[((size_t)o * Ny + y) * Nx + x0 + j] = acc;
  }
}

__global__ void __launch_bounds__(1024)
coarse_split_xy_bwd(Dims d, CoarseLaunch c, const double *__restrict__ t, double *__restrict__ u0, int np) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double red[16];
  const int Nx = d.N[0], Ny = d.N[1], px = Nx + 1;
  const int z = blockIdx.x, part = blockIdx.y;
  const int rh = (Ny + np - 1) / np, y0 = part * rh, ny = min(rh, Ny - y0);
  double *P = reinterpret_cast<double *>(smem_raw);  // Ny x px: input plane
  double *W = P + Ny * px;                            // rh x px: after y
  double *sxt = W + rh * px, *syt = sxt + Nx * Nx;   // transposed Sx and Sy
  const int tid = threadIdx.x, nth = blockDim.x;
  copy4(tid, Nx * Nx, nth, [&](int i) { return c.S[0][i]; },
        [&](int i, double v) { sxt[(i % Nx) * Nx + i / Nx] = v; });
  copy4(tid, Ny * Ny, nth, [&](int i) { return c.S[1][i]; },
        [&](int i, double v) { syt[(i % Ny) * Ny + i / Ny] = v; });
  const double *tz = t + (size_t)z * Nx * Ny;
  copy4(tid, Nx * Ny, nth, [&](int i) { return tz[i]; }, [&](int i, double v) {
    const int y = i / Nx;
    P[y * px + i - y * Nx] = v;
  });
  __syncthreads();
  for (int i = tid; i < ny * Nx; i += nth) {  // y backward on rows y0 .. y0 + ny
    const int r = i / Nx, xq = i - r * Nx;
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < Ny; ++a) acc += syt[a * Ny + y0 + r] * P[a * px + xq];
    W[r * px + xq] = acc;
  }
  __syncthreads();
  double s = 0.0;
  for (int i = tid; i < ny * Nx; i += nth) {  // x backward
    const int r = i / Nx, x = i - r * Nx;
    double acc = 0.0;
#pragma unroll 8
    for (int a = 0; a < Nx; ++a) acc += sxt[a * Nx + x] * W[r * px + a];
    u0[elem_major_p1(d, x, y0 + r, z)] = acc;
    s += acc;
  }
  s = block_sum_2d(s, red);
  if (tid == 0) c.partial_u[z * np + part] = s;
}

// ---- level-0 grids whose planes exceed the LDS --------------------------------
// One workgroup per plane, five passes through global memory: x forward, y
// forward, z forward + mean correction + Lambda^+ + z backward, y backward,
// x backward.  A pass moves its plane's lines through LDS in chunks (all
// loads of a chunk before any output is written, so the y passes can work in
// place) and reads the 1D tables from global memory (they stay in the
// caches).  Same arithmetic as the plane kernels, in another summation order.
constexpr int kBigThreads = 256;
constexpr int kBigChunk = 4096;  // line values per chunk in LDS

// Contraction of the cl lines of length n in buf: out(l, o, v) receives
// output o of line l; FWD: sum_a A[a*n + o] x[a], else sum_a A[o*n + a] x[a].
// For n <= blockDim.x, thread t computes output o = t % n of lines
// t / n + G r (G = blockDim.x / n line groups; a wavefront shares its line,
// so the line entries are LDS broadcasts) for up to 8 lines at once, each
// table entry loaded once for all of them.
template <bool FWD, typename Out>
__device__ void big_contract(const double *buf, int cl, int n, const double *__restrict__ A, Out out) {
  constexpr int RB = 8;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (n <= nth) {
    const int G = nth / n, o = tid % n, lg = tid / n;
    if (lg >= G) return;
    for (int l0 = lg; l0 < cl; l0 += G * RB) {
      double acc[RB];
#pragma unroll
      for (int r = 0; r < RB; ++r) acc[r] = 0.0;
      for (int a = 0; a < n; ++a) {
        const double av = FWD ? A[a * n + o] : A[o * n + a];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
          const int l = l0 + r * G;
          if (l < cl) acc[r] += av * buf[l * n + a];
        }
      }
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const int l = l0 + r * G;
        if (l < cl) out(l, o, acc[r]);
      }
    }
  } else {
    for (int i = tid; i < cl * n; i += nth) {
      const int l = i / n, o = i - l * n;
      const double *x = buf + l * n;
      double acc = 0.0;
      for (int a = 0; a < n; ++a) acc += (FWD ? A[a * n + o] : A[o * n + a]) * x[a];
      out(l, o, acc);
    }
  }
}

// nl lines of length n: get(l, a) is entry a of line l, put(l, o, v) stores
// output o; lines lb .. le - 1 of a plane (the workgroup's part)
template <bool FWD, typename Get, typename Put>
__device__ void big_lines(double *buf, int lb, int le, int n, const double *__restrict__ A, Get get, Put put) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int L = max(1, kBigChunk / n);
  for (int l0 = lb; l0 < le; l0 += L) {
    const int cl = min(L, le - l0);
    for (int i = tid; i < cl * n; i += nth) {
      const int l = i / n;
      buf[i] = get(l0 + l, i - l * n);
    }
    __syncthreads();
    big_contract<FWD>(buf, cl, n, A, [&](int l, int o, double v) { put(l0 + l, o, v); });
    __syncthreads();
  }
}

// the part of a plane's nl lines that workgroup (blockIdx.x, blockIdx.y) owns
__device__ __forceinline__ int part_begin(int nl) { return (int)((int64_t)nl * blockIdx.y / gridDim.y); }
__device__ __forceinline__ int part_end(int nl) { return (int)((int64_t)nl * (blockIdx.y + 1) / gridDim.y); }

__device__ double big_block_sum(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int t = threadIdx.x, w = t >> 6, nw = (blockDim.x + 63) >> 6;
  if ((t & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;  // valid in thread 0
}

// x forward per z plane from the element-major f_0; plane sum -> partial[z]
template <typename TI>
__global__ void __launch_bounds__(kBigThreads)
coarse_big_x_fwd(Dims d, CoarseLaunch c, const TI *__restrict__ f0, double *__restrict__ t) {
  __shared__ double buf[kBigChunk];
  __shared__ double red[kBigThreads / 64];
  const int Nx = d.N[0], Ny = d.N[1], z = blockIdx.x;
  double s = 0.0;
  big_lines<true>(
      buf, part_begin(Ny), part_end(Ny), Nx, c.S[0],
      [&](int y, int x) {
        const double v = (double)f0[elem_major_p1(d, x, y, z)];
        s += v;
        return v;
      },
      [&](int y, int o, double v) { t[((size_t)z * Ny + y) * Nx + o] = v; });
  s = big_block_sum(s, red);
  if (threadIdx.x == 0) c.partial[z * gridDim.y + blockIdx.y] = s;
}

// y forward (FWD) or backward per z plane, in place
template <bool FWD>
__global__ void __launch_bounds__(kBigThreads) coarse_big_y(Dims d, const double *__restrict__ Sy, double *t) {
  __shared__ double buf[kBigChunk];
  const int Nx = d.N[0], Ny = d.N[1], z = blockIdx.x;
  double *tz = t + (size_t)z * Ny * Nx;
  big_lines<FWD>(
      buf, part_begin(Nx), part_end(Nx), Ny, Sy, [&](int x, int y) { return tz[(size_t)y * Nx + x]; },
      [&](int x, int o, double v) { tz[(size_t)o * Nx + x] = v; });
}

// per y plane: z forward, mean correction, Lambda^+, z backward, in place
__global__ void __launch_bounds__(kBigThreads) coarse_big_z(Dims d, CoarseLaunch c, double *t, int np) {
  __shared__ double buf[kBigChunk];
  __shared__ double red[kBigThreads / 64];
  __shared__ double mean_sh;
  const int Nx = d.N[0], Ny = d.N[1], Nz = d.N[2], y = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < Nz * np; i += blockDim.x) s += c.partial[i];
  s = big_block_sum(s, red);
  if (tid == 0) mean_sh = s / ((double)Nx * Ny * Nz);
  __syncthreads();
  const double mean = mean_sh;
  const size_t zs = (size_t)Ny * Nx;
  double *ty = t + (size_t)y * Nx;
  // forward into the LDS chunk, then scale and transform back through the
  // caller's lines: two chunk passes per line set
  const int L = max(1, kBigChunk / (2 * Nz));
  double *fw = buf + L * Nz;
  const int xe = part_end(Nx);
  for (int x0 = part_begin(Nx); x0 < xe; x0 += L) {
    const int cl = min(L, xe - x0);
    for (int i = tid; i < cl * Nz; i += blockDim.x) {
      const int l = i / Nz, z = i - l * Nz;
      buf[i] = ty[z * zs + x0 + l];
    }
    __syncthreads();
    big_contract<true>(buf, cl, Nz, c.S[2], [&](int l, int o, double acc) {
      const int x = x0 + l;
      const double v = acc - mean * c.colsum[2][o] * c.colsum[0][x] * c.colsum[1][y];
      const bool zero = (x == c.zero[0] && y == c.zero[1] && o == c.zero[2]);
      fw[l * Nz + o] = zero ? 0.0 : v / (c.lam[0][x] + c.lam[1][y] + c.lam[2][o]);
    });
    __syncthreads();
    big_contract<false>(fw, cl, Nz, c.S[2], [&](int l, int o, double acc) { ty[o * zs + x0 + l] = acc; });
    __syncthreads();
  }
}

// x backward per z plane into the element-major u_0; plane sum -> partial_u[z]
__global__ void __launch_bounds__(kBigThreads)
coarse_big_x_bwd(Dims d, CoarseLaunch c, const double *__restrict__ t, double *__restrict__ u0) {
  __shared__ double buf[kBigChunk];
  __shared__ double red[kBigThreads / 64];
  const int Nx = d.N[0], Ny = d.N[1], z = blockIdx.x;
  double s = 0.0;
  big_lines<false>(
      buf, part_begin(Ny), part_end(Ny), Nx, c.S[0], [&](int y, int x) { return t[((size_t)z * Ny + y) * Nx + x]; },
      [&](int y, int o, double v) {
        u0[elem_major_p1(d, o, y, z)] = v;
        s += v;
      });
  s = big_block_sum(s, red);
  if (threadIdx.x == 0) c.partial_u[z * gridDim.y + blockIdx.y] = s;
}

// LDS bytes of the plane kernels: two planes, plus the 1D tables when they fit
constexpr size_t kCoarseLds = 150 * 1024;
size_t plane_bytes(const Dims &d, int a, int b) { return 2 * (size_t)d.N[a] * d.N[b] * sizeof(double); }
size_t tab_bytes(const Dims &d, int a, int b) {
  return ((size_t)d.N[a] * d.N[a] + (a == b ? 0 : (size_t)d.N[b] * d.N[b])) * sizeof(double);
}

}  // namespace

// Workgroups per plane of the split kernels: doubled while the plane passes
// have fewer than 256 workgroups and each part keeps at least 4 columns
// (rows); 1 (one workgroup per plane) when their LDS would not fit.
// Workgroups per plane of the line passes (level-0 planes beyond the LDS).
constexpr int kBigParts = 8;

static bool coarse_planes_fit(const CoarseLaunch &c) {
  Dims d;
  for (int i = 0; i < 3; ++i) d.N[i] = c.N[i], d.ne[i] = c.ne[i];
  return plane_bytes(d, 0, 1) <= kCoarseLds && plane_bytes(d, 0, 2) <= kCoarseLds;
}

int coarse_parts(const CoarseLaunch &c) {
  if (!coarse_planes_fit(c)) return kBigParts;
  const int N0 = c.N[0], N1 = c.N[1], N2 = c.N[2];
  int np = 1;
  while (np < 8 && std::min(N1, N2) * np * 2 <= 256 && N0 / (2 * np) >= 4 && N1 / (2 * np) >= 4) np *= 2;
  if (np == 1) return 1;
  const size_t cw = (N0 + np - 1) / np, rh = (N1 + np - 1) / np;
  const size_t tabs = (size_t)N0 * N0 + (size_t)N1 * N1;
  const size_t fwd = (size_t)N1 * (N0 + 1) + N1 * (cw + 1) + tabs;
  const size_t zk = 2 * (size_t)N2 * (cw + 1) + 2 * (size_t)N2 * N2;
  const size_t bwd = (size_t)N1 * (N0 + 1) + rh * (N0 + 1) + tabs;
  if (std::max(fwd, std::max(zk, bwd)) * sizeof(double) > kCoarseLds) return 1;
  return np;
}

int coarse_num_partials(const CoarseLaunch &c) { return c.N[2] * coarse_parts(c); }

template <typename K>
static hipError_t allow_lds(K kernel, size_t shm) {
  if (shm <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <typename TI>
hipError_t launch_big(const Dims &d, const CoarseLaunch &c, const TI *f0, double *u0, hipStream_t st) {
  // a z line and its transform must fit one chunk (a part may own no lines:
  // its plane sum is then 0)
  if (2 * d.N[2] > kBigChunk || d.N[0] > kBigChunk || d.N[1] > kBigChunk) return hipErrorInvalidValue;
  const int np = kBigParts;
  coarse_big_x_fwd<TI><<<dim3(d.N[2], np), kBigThreads, 0, st>>>(d, c, f0, c.t0);
  coarse_big_y<true><<<dim3(d.N[2], np), kBigThreads, 0, st>>>(d, c.S[1], c.t0);
  coarse_big_z<<<dim3(d.N[1], np), kBigThreads, 0, st>>>(d, c, c.t0, np);
  coarse_big_y<false><<<dim3(d.N[2], np), kBigThreads, 0, st>>>(d, c.S[1], c.t0);
  coarse_big_x_bwd<<<dim3(d.N[2], np), kBigThreads, 0, st>>>(d, c, c.t0, u0);
  return hipGetLastError();
}

// one workgroup per plane
template <typename TI>
hipError_t launch_planes(const Dims &d, const CoarseLaunch &c, const TI *f0, double *u0, hipStream_t st) {
  size_t sxy = plane_bytes(d, 0, 1), sz = plane_bytes(d, 0, 2);
  if (sxy > kCoarseLds || sz > kCoarseLds) return hipErrorInvalidValue;
  const bool lds_xy = sxy + tab_bytes(d, 0, 1) <= kCoarseLds;
  const bool lds_z = sz + tab_bytes(d, 2, 2) <= kCoarseLds;
  if (lds_xy) sxy += tab_bytes(d, 0, 1);
  if (lds_z) sz += tab_bytes(d, 2, 2);
  hipError_t e;
  // 2D workgroups: x index in threadIdx.x, rows strided over threadIdx.y
  const int bx = (d.N[0] + 63) / 64 * 64;
  const dim3 blk(bx, std::max(1, std::min(1024 / bx, std::max(d.N[1], d.N[2]))));
  if (lds_xy) {
    if ((e = allow_lds(coarse_plane_xy_fwd<TI, true>, sxy)) != hipSuccess) return e;
    if ((e = allow_lds(coarse_plane_xy_bwd<true>, sxy)) != hipSuccess) return e;
  } else {
    if ((e = allow_lds(coarse_plane_xy_fwd<TI, false>, sxy)) != hipSuccess) return e;
    if ((e = allow_lds(coarse_plane_xy_bwd<false>, sxy)) != hipSuccess) return e;
  }
  if ((e = allow_lds(lds_z ? coarse_plane_z<true> : coarse_plane_z<false>, sz)) != hipSuccess) return e;
  if (lds_xy) coarse_plane_xy_fwd<TI, true><<<d.N[2], blk, sxy, st>>>(d, c, f0, c.t0);
  else coarse_plane_xy_fwd<TI, false><<<d.N[2], blk, sxy, st>>>(d, c, f0, c.t0);
  if (lds_z) coarse_plane_z<true><<<d.N[1], blk, sz, st>>>(d, c, c.t0);
  else coarse_plane_z<false><<<d.N[1], blk, sz, st>>>(d, c, c.t0);
  if (lds_xy) coarse_plane_xy_bwd<true><<<d.N[2], blk, sxy, st>>>(d, c, c.t0, u0);
  else coarse_plane_xy_bwd<false><<<d.N[2], blk, sxy, st>>>(d, c, c.t0, u0);
  return hipGetLastError();
}

template <typename TI>
hipError_t launch_coarse(const CoarseLaunch &c, const TI *f0, double *u0, bool subtract_mean, hipStream_t st) {
  Dims d;
  for (int i = 0; i < 3; ++i) {
    d.N[i] = c.N[i];
    d.ne[i] = c.ne[i];
  }
  const int64_t N0 = (int64_t)d.N[0] * d.N[1] * d.N[2];
  hipError_t e;
  const int np = coarse_parts(c);
  if (!coarse_planes_fit(c)) {
    if ((e = launch_big<TI>(d, c, f0, u0, st)) != hipSuccess) return e;
  } else if (np > 1) {
    const int Nx = d.N[0], Ny = d.N[1], Nz = d.N[2];
    const size_t cw = (Nx + np - 1) / np, rh = (Ny + np - 1) / np;
    const size_t tabs = (size_t)Nx * Nx + (size_t)Ny * Ny;
    const size_t s1 = ((size_t)Ny * (Nx + 1) + Ny * (cw + 1) + tabs) * sizeof(double);
    const size_t s2 = (2 * (size_t)Nz * (cw + 1) + 2 * (size_t)Nz * Nz) * sizeof(double);
    const size_t s3 = ((size_t)Ny * (Nx + 1) + rh * (Nx + 1) + tabs) * sizeof(double);
    if ((e = allow_lds(coarse_split_xy_fwd<TI>, s1)) != hipSuccess) return e;
    if ((e = allow_lds(coarse_split_z, s2)) != hipSuccess) return e;
    if ((e = allow_lds(coarse_split_xy_bwd, s3)) != hipSuccess) return e;
    coarse_split_xy_fwd<TI><<<dim3(Nz, np), 1024, s1, st>>>(d, c, f0, c.t0, np);
    coarse_split_z<<<dim3(Ny, np), 1024, s2, st>>>(d, c, c.t0, np);
    coarse_split_xy_bwd<<<dim3(Nz, np), 1024, s3, st>>>(d, c, c.t0, u0, np);
  } else {
    if ((e = launch_planes<TI>(d, c, f0, u0, st)) != hipSuccess) return e;
  }
  e = hipGetLastError();
  if (e != hipSuccess || !subtract_mean) return e;
  if ((e = launch_finalize(c.partial_u, coarse_num_partials(c), 1.0 / (double)N0, c.scalars + 1, st)) != hipSuccess)
    return e;
  return launch_sub_scalar<double>(u0, N0, c.scalars + 1, st);
}

template hipError_t launch_coarse<double>(const CoarseLaunch &, const double *, double *, bool, hipStream_t);
template hipError_t launch_coarse<float>(const CoarseLaunch &, const float *, double *, bool, hipStream_t);

}  // namespace sipg
