// Element-by-element application of the SIPG operator of eq. (A),
//   A = Mz x My x Lx + Mz x Ly x Mx + Lz x My x Mx,
// by sum factorization, and the inter-level transfers of Sec. 3.2.
//
// Each workgroup owns `epb` consecutive elements.  The element data is staged
// in LDS; one thread owns one 1D line of an element per direction, keeps the
// line in registers and applies the n x n element block of L_d (uniform table
// entries, loaded through the scalar cache).  Face coupling to the two
// neighbours in a direction needs, per line, the neighbour's value at the
// shared face and its one-sided derivative there (a dot product with the
// first or last row of D), so the neighbour line is read from global memory;
// XCD-aware block numbering keeps those re-reads in L2.
//
// With DL = D[0][:]/h, DR = D[p][:]/h the coupling of line v of element e to
// its right neighbour line vr and left neighbour line vl is
//   c[i] = DR[i] vr[0] - DL[i] vl[p]
//        - [i = p] (DL . vr + mu vr[0]) + [i = 0] (DR . vl - mu vl[p]).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

enum { MODE_APPLY = 0, MODE_RESID = 1, MODE_RESTRICT = 2 };

template <typename T, int N, int MODE, bool DOT>
__global__ void __launch_bounds__(1024)
apply_kernel(Mesh g, ApplyTabs<T> tb, const T *__restrict__ u, const T *__restrict__ f,
             T *__restrict__ out, int epb, T *__restrict__ partial, const T *__restrict__ J, int nc) {
  constexpr int N2 = N * N, N3 = N2 * N;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *su = reinterpret_cast<T *>(smem_raw);
  T *sy = su + epb * N3;
  __shared__ T red[16];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int e0 = blk * epb;
  const int nloc = min(epb, g.E - e0);
  const int tid = threadIdx.x, nth = blockDim.x;

  for (int idx = tid; idx < nloc * N3; idx += nth) su[idx] = u[(size_t)e0 * N3 + idx];
  __syncthreads();
  const int nlines = nloc * N2;

  // ---- x lines (le, k, j): contiguous
  {
    const T *__restrict__ Ld = tb.Ld[0];
    const T *__restrict__ DL = tb.DL[0];
    const T *__restrict__ DR = tb.DR[0];
    const T mu = tb.mu[0];
    for (int t = tid; t < nlines; t += nth) {
      const int le = t / N2, kj = t - le * N2;
      const int k = kj / N, j = kj - k * N;
      const int e = e0 + le;
      const int ex = e % g.ne[0], rest = e / g.ne[0];
      const int ey = rest % g.ne[1], ez = rest / g.ne[1];
      const T *lr = u + (size_t)elem_index(g, wrap(ex + 1, g.ne[0]), ey, ez) * N3 + kj * N;
      const T *ll = u + (size_t)elem_index(g, wrap(ex - 1, g.ne[0]), ey, ez) * N3 + kj * N;
      T v[N];
      T gR = 0, gL = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        v[i] = su[le * N3 + kj * N + i];
        gR += DL[i] * lr[i];
        gL += DR[i] * ll[i];
      }
      const T vR = lr[0], vL = ll[N - 1];
      const T sc = tb.M[2][k] * tb.M[1][j];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T acc = DR[i] * vR - DL[i] * vL;
#pragma unroll
        for (int q = 0; q < N; ++q) acc += Ld[i * N + q] * v[q];
        if (i == N - 1) acc -= gR + mu * vR;
        if (i == 0) acc += gL - mu * vL;
        sy[le * N3 + kj * N + i] = sc * acc;
      }
    }
  }
  __syncthreads();

  // ---- y lines (le, k, i): stride N
  {
    const T *__restrict__ Ld = tb.Ld[1];
    const T *__restrict__ DL = tb.DL[1];
    const T *__restrict__ DR = tb.DR[1];
    const T mu = tb.mu[1];
    for (int t = tid; t < nlines; t += nth) {
      const int le = t / N2, ki = t - le * N2;
      const int k = ki / N, i = ki - k * N;
      const int e = e0 + le;
      const int ex = e % g.ne[0], rest = e / g.ne[0];
      const int ey = rest % g.ne[1], ez = rest / g.ne[1];
      const int base = k * N2 + i;
      const T *lr = u + (size_t)elem_index(g, ex, wrap(ey + 1, g.ne[1]), ez) * N3 + base;
      const T *ll = u + (size_t)elem_index(g, ex, wrap(ey - 1, g.ne[1]), ez) * N3 + base;
      T v[N];
      T gR = 0, gL = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        v[j] = su[le * N3 + base + j * N];
        gR += DL[j] * lr[j * N];
        gL += DR[j] * ll[j * N];
      }
      const T vR = lr[0], vL = ll[(N - 1) * N];
      const T sc = tb.M[2][k] * tb.M[0][i];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        T acc = DR[j] * vR - DL[j] * vL;
#pragma unroll
        for (int q = 0; q < N; ++q) acc += Ld[j * N + q] * v[q];
        if (j == N - 1) acc -= gR + mu * vR;
        if (j == 0) acc += gL - mu * vL;
        sy[le * N3 + base + j * N] += sc * acc;
      }
    }
  }
  __syncthreads();

  // ---- z lines (le, j, i): stride N^2; finishes the operator
  T dot = 0;
  {
    const T *__restrict__ Ld = tb.Ld[2];
    const T *__restrict__ DL = tb.DL[2];
    const T *__restrict__ DR = tb.DR[2];
    const T mu = tb.mu[2];
    for (int t = tid; t < nlines; t += nth) {
      const int le = t / N2, ji = t - le * N2;
      const int j = ji / N, i = ji - j * N;
      const int e = e0 + le;
      const int ex = e % g.ne[0], rest = e / g.ne[0];
      const int ey = rest % g.ne[1], ez = rest / g.ne[1];
      const T *lr = u + (size_t)elem_index(g, ex, ey, wrap(ez + 1, g.ne[2])) * N3 + ji;
      const T *ll = u + (size_t)elem_index(g, ex, ey, wrap(ez - 1, g.ne[2])) * N3 + ji;
      T v[N];
      T gR = 0, gL = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        v[k] = su[le * N3 + ji + k * N2];
        gR += DL[k] * lr[k * N2];
        gL += DR[k] * ll[k * N2];
      }
      const T vR = lr[0], vL = ll[(N - 1) * N2];
      const T sc = tb.M[1][j] * tb.M[0][i];
#pragma unroll
      for (int k = 0; k < N; ++k) {
        T acc = DR[k] * vR - DL[k] * vL;
#pragma unroll
        for (int q = 0; q < N; ++q) acc += Ld[k * N + q] * v[q];
        if (k == N - 1) acc -= gR + mu * vR;
        if (k == 0) acc += gL - mu * vL;
        const int li = le * N3 + ji + k * N2;
        const T y = sy[li] + sc * acc;
        const size_t gi = (size_t)e0 * N3 + li;
        if (MODE == MODE_APPLY) {
          out[gi] = y;
          if (DOT) dot += v[k] * y;
        } else if (MODE == MODE_RESID) {
          out[gi] = f[gi] - y;
        } else {
          sy[li] = f[gi] - y;
        }
      }
    }
  }
  if (DOT) {
    T s = block_reduce_sum(dot, red);
    if (tid == 0) partial[blk] = s;
  }
  if (MODE != MODE_RESTRICT) return;

  // ---- restriction f_c = (J^T x J^T x J^T) r, element by element
  __syncthreads();
  // x: sy[le][k][j][i] -> su[le][k][j][a]
  for (int t = tid; t < nlines; t += nth) {
    const int le = t / N2, kj = t - le * N2;
    T v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = sy[le * N3 + kj * N + i];
    for (int a = 0; a < nc; ++a) {
      T acc = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) acc += J[i * nc + a] * v[i];
      su[le * N3 + kj * nc + a] = acc;
    }
  }
  __syncthreads();
  // y: su[le][k][j][a] -> sy[le][k][b][a]; lines (le, k, a)
  for (int t = tid; t < nloc * N * nc; t += nth) {
    const int le = t / (N * nc), ka = t - le * N * nc;
    const int k = ka / nc, a = ka - k * nc;
    T v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = su[le * N3 + (k * N + j) * nc + a];
    for (int b = 0; b < nc; ++b) {
      T acc = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) acc += J[j * nc + b] * v[j];
      sy[le * N3 + (k * nc + b) * nc + a] = acc;
    }
  }
  __syncthreads();
  // z: sy[le][k][b][a] -> out[e][c][b][a]; lines (le, b, a)
  const int nc2 = nc * nc, nc3 = nc2 * nc;
  for (int t = tid; t < nloc * nc2; t += nth) {
    const int le = t / nc2, ba = t - le * nc2;
    T v[N];
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = sy[le * N3 + k * nc2 + ba];
    for (int c = 0; c < nc; ++c) {
      T acc = 0;
#pragma unroll
      for (int k = 0; k < N; ++k) acc += J[k * nc + c] * v[k];
      out[(size_t)(e0 + le) * nc3 + c * nc2 + ba] = acc;
    }
  }
}

// u_f += (J x J x J)(u_c - mean), element by element; J is NF x nc.
template <typename T, typename TC, int NF>
__global__ void __launch_bounds__(1024)
prolong_kernel(int E, const T *__restrict__ J, int nc, const TC *__restrict__ uc,
               const double *__restrict__ mean, T *__restrict__ uf, int epb) {
  constexpr int NF2 = NF * NF, NF3 = NF2 * NF;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *s0 = reinterpret_cast<T *>(smem_raw);  // epb * NF3 each
  T *s1 = s0 + epb * NF3;
  T *s2 = s1 + epb * NF3;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int e0 = blk * epb;
  const int nloc = min(epb, E - e0);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int nc2 = nc * nc, nc3 = nc2 * nc;
  const T m = mean ? (T)(*mean) : (T)0;
  for (int idx = tid; idx < nloc * nc3; idx += nth) {
    const int le = idx / nc3, r = idx - le * nc3;
    s0[le * NF3 + r] = (T)uc[(size_t)e0 * nc3 + idx] - m;
  }
  __syncthreads();
  // x: s0[le][c][b][a] -> s1[le][c][b][i]
  for (int t = tid; t < nloc * nc2; t += nth) {
    const int le = t / nc2, cb = t - le * nc2;
    T v[NF];
#pragma unroll
    for (int a = 0; a < NF; ++a) v[a] = (a < nc) ? s0[le * NF3 + cb * nc + a] : (T)0;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < NF; ++a)
        if (a < nc) acc += J[i * nc + a] * v[a];
      s1[le * NF3 + cb * NF + i] = acc;
    }
  }
  __syncthreads();
  // y: s1[le][c][b][i] -> s2[le][c][j][i]; lines (le, c, i)
  for (int t = tid; t < nloc * nc * NF; t += nth) {
    const int le = t / (nc * NF), ci = t - le * nc * NF;
    const int c = ci / NF, i = ci - c * NF;
    T v[NF];
#pragma unroll
    for (int b = 0; b < NF; ++b) v[b] = (b < nc) ? s1[le * NF3 + (c * nc + b) * NF + i] : (T)0;
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < NF; ++b)
        if (b < nc) acc += J[j * nc + b] * v[b];
      s2[le * NF3 + (c * NF + j) * NF + i] = acc;
    }
  }
  __syncthreads();
  // z: s2[le][c][j][i] -> uf[e][k][j][i] += ...; lines (le, j, i)
  for (int t = tid; t < nloc * NF2; t += nth) {
    const int le = t / NF2, ji = t - le * NF2;
    T v[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) v[c] = (c < nc) ? s2[le * NF3 + c * NF2 + ji] : (T)0;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < NF; ++c)
        if (c < nc) acc += J[k * nc + c] * v[c];
      uf[(size_t)(e0 + le) * NF3 + k * NF2 + ji] += acc;
    }
  }
}

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

template <typename T, int N>
hipError_t launch_apply_n(const ApplyLaunch<T> &a, hipStream_t st) {
  constexpr int N2 = N * N, N3 = N2 * N;
  int epb = 256 / N2;
  if (epb < 1) epb = 1;
  if (a.mode == APPLY_RESTRICT && epb > 1) {
    // the restriction reuses the two element buffers; nothing else to size
  }
  const int nth = std::min(1024, round_up(epb * N2, 64));
  const int nblk = (a.mesh.E + epb - 1) / epb;
  const size_t shm = 2 * (size_t)epb * N3 * sizeof(T);
  if (shm > 64 * 1024) {
    hipError_t e = hipSuccess;
    if (a.mode == APPLY_PLAIN && a.partial)
      e = hipFuncSetAttribute((const void *)apply_kernel<T, N, MODE_APPLY, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    else if (a.mode == APPLY_PLAIN)
      e = hipFuncSetAttribute((const void *)apply_kernel<T, N, MODE_APPLY, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    else if (a.mode == APPLY_RESID)
      e = hipFuncSetAttribute((const void *)apply_kernel<T, N, MODE_RESID, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    else
      e = hipFuncSetAttribute((const void *)apply_kernel<T, N, MODE_RESTRICT, false>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  if (a.mode == APPLY_PLAIN && a.partial)
    apply_kernel<T, N, MODE_APPLY, true><<<nblk, nth, shm, st>>>(a.mesh, a.tabs, a.u, a.f, a.out, epb,
                                                                 a.partial, a.J, a.nc);
  else if (a.mode == APPLY_PLAIN)
    apply_kernel<T, N, MODE_APPLY, false><<<nblk, nth, shm, st>>>(a.mesh, a.tabs, a.u, a.f, a.out, epb,
                                                                  a.partial, a.J, a.nc);
  else if (a.mode == APPLY_RESID)
    apply_kernel<T, N, MODE_RESID, false><<<nblk, nth, shm, st>>>(a.mesh, a.tabs, a.u, a.f, a.out, epb,
                                                                  a.partial, a.J, a.nc);
  else
    apply_kernel<T, N, MODE_RESTRICT, false><<<nblk, nth, shm, st>>>(a.mesh, a.tabs, a.u, a.f, a.out, epb,
                                                                     a.partial, a.J, a.nc);
  return hipGetLastError();
}

template <typename T, typename TC, int NF>
hipError_t launch_prolong_n(const ProlongLaunch<T, TC> &a, hipStream_t st) {
  constexpr int NF2 = NF * NF, NF3 = NF2 * NF;
  int epb = 256 / NF2;
  if (epb < 1) epb = 1;
  const int nth = std::min(1024, round_up(epb * NF2, 64));
  const int nblk = (a.E + epb - 1) / epb;
  const size_t shm = 3 * (size_t)epb * NF3 * sizeof(T);
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)prolong_kernel<T, TC, NF>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  prolong_kernel<T, TC, NF><<<nblk, nth, shm, st>>>(a.E, a.J, a.nc, a.uc, a.mean, a.uf, epb);
  return hipGetLastError();
}

}  // namespace

int apply_num_blocks(int E, int n) {
  int epb = 256 / (n * n);
  if (epb < 1) epb = 1;
  return (E + epb - 1) / epb;
}

#define SIPG_ORDER_CASES(X) \
  X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17)

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

template hipError_t launch_apply<double>(const ApplyLaunch<double> &, hipStream_t);
template hipError_t launch_apply<float>(const ApplyLaunch<float> &, hipStream_t);
template hipError_t launch_prolong<double, double>(const ProlongLaunch<double, double> &, hipStream_t);
template hipError_t launch_prolong<float, float>(const ProlongLaunch<float, float> &, hipStream_t);
template hipError_t launch_prolong<float, double>(const ProlongLaunch<float, double> &, hipStream_t);

}  // namespace sipg
