// Local fast-diagonalization solves (Sec. 3.1) of subdomains that do not fit
// the LDS (wider than 32 nodes in some direction, up to 64), with every 1D
// contraction on the matrix cores: v_mfma_f64_16x16x4f64 for FP64 and
// v_mfma_f32_16x16x4f32 for FP32 (on gfx950 the FP64 and FP32 matrix peaks
// equal the vector peaks, but a matrix instruction takes its operands from
// two registers per lane for 1024 multiply-adds, where the vector path reads
// an LDS operand for every few multiply-adds and was bound by LDS reads).
//
// Same three phases as the vector plane kernels (kernels_large.hip), each on
// 2D planes of the subdomain in LDS, the correction tensor W = C[s] in HBM
// between the phases:
//   1  per z plane: gather R_s r, x forward, y forward
//   2  per y plane: z forward, divide by lam_x + lam_y + lam_z, z backward
//   3  per z plane: y backward, x backward (with the hat weights)
// Every wave works on planes of its own (no workgroup barrier after the
// table staging): it writes a plane into its LDS slot, issues the global
// loads of its next plane into registers, contracts the current plane while
// they are in flight, and stores the result.  A contraction of `count` plane
// lines with the table F (m x m, zero padded) is a product D = F^T X: the
// table is the A operand (16 outputs x 4 inputs), 16 plane lines the B
// operand (4 inputs x 16 lines); the wave accumulates all NLT x NOT output
// tiles of the plane over the inputs in steps of 4 (independent chains of
// matrix instructions), then writes them back in place.  The tables are
// stored fragment-major (entry (ot*KS + ks)*64 + lane is
// F[4 ks + lane/16][16 ot + lane%16]), so a fragment is 64 consecutive values,
// and staged in LDS once per workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "kernels.h"

namespace sipg {

namespace {

template <typename T>
struct MfmaOp;

template <>
struct MfmaOp<double> {
  typedef double V __attribute__((ext_vector_type(4)));
  __device__ static V mma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // output row (within the 16 x 16 tile) of item v of lane `lane`; the
  // column is lane % 16 (rows interleaved over the four lane groups)
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct MfmaOp<float> {
  typedef float V __attribute__((ext_vector_type(4)));
  __device__ static V mma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  // rows 4 (lane / 16) .. + 3 in the four items
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// Orders the LDS accesses of one wave around a point (the wave's lanes write
// what other lanes of it read next; LDS executes a wave's accesses in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place contraction of `count` lines (count <= 16 NLT) of the wave's plane
// P: line j has its entries at P[j * ls + a * ks] (a < m <= 16 NOT);
// afterwards entry o of line j is sum_a F[a][o] (old entry a).  Lines
// beyond the count read the last line (their results are dropped); inputs
// are read up to 4 ceil(m/4) (the plane's zero padding).  KS: the input
// steps ceil(m/4) when known at compile time (0: from m).
template <typename T, int NLT, int NOT, int KS>
__device__ __forceinline__ void wave_contract(T *P, int ls, int ks, int count, int m, const T *F) {
  using Op = MfmaOp<T>;
  using V = typename Op::V;
  const int lane = threadIdx.x & 63;
  const int nks = KS > 0 ? KS : (m + 3) >> 2;
  V acc[NLT][NOT];
  const T *pb[NLT];
#pragma unroll
  for (int lt = 0; lt < NLT; ++lt) {
    pb[lt] = P + min(lt * 16 + (lane & 15), count - 1) * ls + (lane >> 4) * ks;
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot) acc[lt][ot] = V{0, 0, 0, 0};
  }
  const T *fa = F + lane;
  const int step = 4 * ks;
  auto fetch = [&](int kk, T (&a)[NOT], T (&b)[NLT]) {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot) a[ot] = fa[(ot * nks + kk) * 64];
#pragma unroll
    for (int lt = 0; lt < NLT; ++lt) b[lt] = pb[lt][kk * step];
  };
  auto mmas = [&](const T (&a)[NOT], const T (&b)[NLT]) {
#pragma unroll
    for (int lt = 0; lt < NLT; ++lt)
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot) acc[lt][ot] = Op::mma(a[ot], b[lt], acc[lt][ot]);
  };
  if constexpr (KS > 0) {
    // operands of step kk + 1 in flight during the products of step kk
    T a[2][NOT], b[2][NLT];
    fetch(0, a[0], b[0]);
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      if (kk + 1 < KS) fetch(kk + 1, a[(kk + 1) & 1], b[(kk + 1) & 1]);
      mmas(a[kk & 1], b[kk & 1]);
    }
  } else {
    for (int kk = 0; kk < nks; ++kk) {
      T a[NOT], b[NLT];
      fetch(kk, a, b);
      mmas(a, b);
    }
  }
  wave_sync();
#pragma unroll
  for (int lt = 0; lt < NLT; ++lt) {
    const int line = lt * 16 + (lane & 15);
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = ot * 16 + Op::row(lane, v);
        if (o < m && line < count) P[line * ls + o * ks] = acc[lt][ot][v];
      }
  }
  wave_sync();
}

__host__ __device__ constexpr int frag_count(int m) { return ((m + 15) / 16) * ((m + 3) / 4) * 64; }
__host__ __device__ constexpr int pad4(int m) { return (m + 3) / 4 * 4; }
__host__ __device__ constexpr int ks_of(int m) { return m > 0 ? (m + 3) / 4 : 0; }

// Plane pitch in values: at least pad4(mx); rows of 16 lines x 2 (FP64) or
// 4 (FP32) inputs of one operand fragment fall on distinct LDS banks when
// the pitch is 2 mod 4 (FP64) or 4 mod 8 (FP32).
__host__ __device__ constexpr int plane_pitch(int mx, int eb) {
  int p = pad4(mx);
  while (eb == 8 ? p % 4 != 2 : p % 8 != 4) ++p;
  return p;
}

// Copies a table into LDS with the loads of 8 entries per thread in flight
// before any is written (a load-wait-write loop costs a memory latency per
// entry, comparable to the work on several planes).
template <typename T>
__device__ __forceinline__ void stage(T *dst, const T *__restrict__ src, int count) {
  constexpr int kU = 8;
  const int nth = blockDim.x;
  for (int i0 = threadIdx.x; i0 < count; i0 += kU * nth) {
    T v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * nth;
      v[u] = i < count ? src[i] : (T)0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int i = i0 + u * nth;
      if (i < count) dst[i] = v[u];
    }
  }
}

// The plane entries of one lane: entry j is number lane + 64 j of the plane
// (row-major, rows of length mu), at (u, v) = (idx % mu, idx / mu); walked
// incrementally without divisions.
struct LaneWalk {
  int u, v, du, dv, mu;
  __device__ LaneWalk(int lane, int mu_) : u(lane % mu_), v(lane / mu_), du(64 % mu_), dv(64 / mu_), mu(mu_) {}
  __device__ void next() {
    u += du;
    v += dv;
    if (u >= mu) u -= mu, ++v;
  }
};

// Subdomain shape of a kernel instantiation: compile-time (MX > 0, order
// N_ - 1) or taken from the tables at run time (MX = 0).  JM bounds the
// plane entries per lane (exact for compile-time shapes).
template <int N_, int MX, int MY, int MZ>
struct WShape {
  static constexpr bool ct = MX > 0;
};

// phase 1: planes (s, c), c the z index: gather R_s r into the xy plane
// (x fast, pitch pp, pad4(my) rows), x forward, y forward, store to W.
// A = ceil(mx/16), B = ceil(my/16); NW waves per workgroup.
template <typename T, int A, int B, int NW, int N_, int MX, int MY, int MZ>
__global__ void __launch_bounds__(64 * NW)
wide_mfma1(Mesh g, int n_rt, SchwarzTabs<T> tb, const T *__restrict__ r, T *__restrict__ W, int ppw, int pp_rt) {
  constexpr bool CT = MX > 0;
  constexpr int JM = CT ? (MX * MY + 63) / 64 : 4 * A * B;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int mx = CT ? MX : tb.m[0], my = CT ? MY : tb.m[1], mz = CT ? MZ : tb.m[2];
  const int n = CT ? N_ : n_rt, pp = CT ? plane_pitch(MX, sizeof(T)) : pp_rt;
  T *Fx = reinterpret_cast<T *>(smem_raw);
  T *Fy = Fx + frag_count(mx);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int plane = pad4(my) * pp;
  T *P = Fy + frag_count(my) + w * plane;
  stage(Fx, tb.frag[0][0], frag_count(mx));
  stage(Fy, tb.frag[0][1], frag_count(my));
  for (int i = lane; i < plane; i += 64) P[i] = (T)0;
  __syncthreads();
  const int V = mx * my, J = CT ? JM : (V + 63) >> 6, n3 = n * n * n;
  const int total = g.E * mz, first = (blockIdx.x * NW + w) * ppw;
  if (first >= total) return;
  auto valid = [&](int j) { return j < J && lane + 64 * j < V; };
  T buf[JM];
  int lo[CT ? JM : 1];  // compile-time shapes: LDS offsets
  if constexpr (CT) {
    LaneWalk it(lane, MX);
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      lo[j] = it.v * pp + it.u;
      it.next();
    }
  }
  // issues the loads of plane gp (subdomain s, z index c) into buf
  auto load = [&](int gp) {
    const int s = gp / mz, c = gp - s * mz;
    const int ex = s % g.ne[0], rest = s / g.ne[0];
    const int ey = rest % g.ne[1], ez = rest / g.ne[1];
    const int gz = c - tb.no[2], dz = gz < 0 ? -1 : (gz >= n ? 1 : 0);
    const T *rz = r + (size_t)wrap(ez + dz, g.ne[2]) * g.ne[1] * g.ne[0] * n3 + (gz - dz * n) * n * n;
    auto xy_off = [&](int u, int v) {
      const int gx = u - tb.no[0], gy = v - tb.no[1];
      const int dx = gx < 0 ? -1 : (gx >= n ? 1 : 0), dy = gy < 0 ? -1 : (gy >= n ? 1 : 0);
      return (wrap(ey + dy, g.ne[1]) * g.ne[0] + wrap(ex + dx, g.ne[0])) * n3 + ((gy - dy * n) * n + gx - dx * n);
    };
    LaneWalk it(lane, mx);
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      if (valid(j)) buf[j] = rz[xy_off(it.u, it.v)];
      it.next();
    }
  };
  // LDS offset of entry j (walk: the running position for runtime shapes)
  auto for_entries = [&](auto fn) {
    if constexpr (CT) {
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (valid(j)) fn(j, lo[j]);
    } else {
      LaneWalk it(lane, mx);
#pragma unroll
      for (int j = 0; j < JM; ++j) {
        if (valid(j)) fn(j, it.v * pp + it.u);
        it.next();
      }
    }
  };
  load(first);
  for (int q = 0; q < ppw; ++q) {
    const int gp = first + q;
    if (gp >= total) break;
    for_entries([&](int j, int o) { P[o] = buf[j]; });
    wave_sync();
    if (q + 1 < ppw && gp + 1 < total) load(gp + 1);
    wave_contract<T, B, A, ks_of(MX)>(P, pp, 1, my, mx, Fx);  // x: the lines are the rows
    wave_contract<T, A, B, ks_of(MY)>(P, 1, pp, mx, my, Fy);  // y: the lines are the columns
    T *Ws = W + (size_t)gp * V;                              // plane c of subdomain s
    for_entries([&](int j, int o) { Ws[lane + 64 * j] = P[o]; });
    wave_sync();
  }
}

// phase 2: planes (s, b), b the y index: the xz plane (x fast, pitch pp,
// pad4(mz) rows) of W, z forward, scaling, z backward.  A = ceil(mx/16),
// C = ceil(mz/16).
template <typename T, int A, int C, int NW, int N_, int MX, int MY, int MZ>
__global__ void __launch_bounds__(64 * NW)
wide_mfma2(int E, SchwarzTabs<T> tb, const T *__restrict__ ilam, T *__restrict__ W, int ppw, int pp_rt) {
  constexpr bool CT = MX > 0;
  constexpr int JM = CT ? (MX * MZ + 63) / 64 : 4 * A * C;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int mx = CT ? MX : tb.m[0], my = CT ? MY : tb.m[1], mz = CT ? MZ : tb.m[2];
  const int pp = CT ? plane_pitch(MX, sizeof(T)) : pp_rt;
  T *Ff = reinterpret_cast<T *>(smem_raw);
  T *Fb = Ff + frag_count(mz);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int plane = pad4(mz) * pp;
  T *P = Fb + frag_count(mz) + w * plane;
  stage(Ff, tb.frag[0][2], frag_count(mz));
  stage(Fb, tb.frag[1][2], frag_count(mz));
  for (int i = lane; i < plane; i += 64) P[i] = (T)0;
  __syncthreads();
  const int V = mx * mz, J = CT ? JM : (V + 63) >> 6;
  // the waves of a workgroup take adjacent planes at each step (plane
  // base + q NW + w at step q): a plane's rows of m_x values lie between
  // those of its y neighbours in W, so the workgroup reads and writes whole
  // cache lines together
  const int total = E * my, first = blockIdx.x * NW * ppw + w;
  if (first >= total) return;
  auto valid = [&](int j) { return j < J && lane + 64 * j < V; };
  T buf[JM], lam[JM];
  const size_t vol = (size_t)mx * my * mz;
  const int zs = my * mx;  // the z stride of W
  int lo[CT ? JM : 1], wo[CT ? JM : 1];  // compile-time shapes: LDS and W offsets
  if constexpr (CT) {
    LaneWalk it(lane, MX);
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      lo[j] = it.v * pp + it.u;
      wo[j] = it.v * zs + it.u;
      it.next();
    }
  }
  // fn(j, LDS offset, offset in the y plane of W)
  auto for_entries = [&](auto fn) {
    if constexpr (CT) {
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (valid(j)) fn(j, lo[j], wo[j]);
    } else {
      LaneWalk it(lane, mx);
#pragma unroll
      for (int j = 0; j < JM; ++j) {
        if (valid(j)) fn(j, it.v * pp + it.u, it.v * zs + it.u);
        it.next();
      }
    }
  };
  auto load = [&](int gp) {
    const int s = gp / my, b = gp - s * my;
    const T *src = W + s * vol + b * mx;
    for_entries([&](int j, int, int o) { buf[j] = src[o]; });
  };
  load(first);
  for (int q = 0; q < ppw; ++q) {
    const int gp = first + q * NW;
    if (gp >= total) break;
    const int s = gp / my, b = gp - s * my;
    // the scaling of this plane is loaded with it, in flight during the
    // forward contraction
    const T *lb = ilam + b * mx;
    for_entries([&](int j, int o, int wof) {
      P[o] = buf[j];
      lam[j] = lb[wof];
    });
    wave_sync();
    if (q + 1 < ppw && gp + NW < total) load(gp + NW);
    wave_contract<T, A, C, ks_of(MZ)>(P, 1, pp, mx, mz, Ff);
    for_entries([&](int j, int o, int) { P[o] *= lam[j]; });
    wave_sync();
    wave_contract<T, A, C, ks_of(MZ)>(P, 1, pp, mx, mz, Fb);
    T *dst = W + s * vol + b * mx;
    for_entries([&](int j, int o, int wof) { dst[wof] = P[o]; });
    wave_sync();
  }
}

// phase 3: planes (s, c): the xy plane of W, y backward, x backward
template <typename T, int A, int B, int NW, int N_, int MX, int MY, int MZ>
__global__ void __launch_bounds__(64 * NW)
wide_mfma3(int E, SchwarzTabs<T> tb, T *__restrict__ W, int ppw, int pp_rt) {
  constexpr bool CT = MX > 0;
  constexpr int JM = CT ? (MX * MY + 63) / 64 : 4 * A * B;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int mx = CT ? MX : tb.m[0], my = CT ? MY : tb.m[1], mz = CT ? MZ : tb.m[2];
  const int pp = CT ? plane_pitch(MX, sizeof(T)) : pp_rt;
  T *Fy = reinterpret_cast<T *>(smem_raw);
  T *Fx = Fy + frag_count(my);
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int plane = pad4(my) * pp;
  T *P = Fx + frag_count(mx) + w * plane;
  stage(Fy, tb.frag[1][1], frag_count(my));
  stage(Fx, tb.frag[1][0], frag_count(mx));
  for (int i = lane; i < plane; i += 64) P[i] = (T)0;
  __syncthreads();
  const int V = mx * my, J = CT ? JM : (V + 63) >> 6;
  const int total = E * mz, first = (blockIdx.x * NW + w) * ppw;
  if (first >= total) return;
  auto valid = [&](int j) { return j < J && lane + 64 * j < V; };
  T buf[JM];
  int lo[CT ? JM : 1];
  if constexpr (CT) {
    LaneWalk it(lane, MX);
#pragma unroll
    for (int j = 0; j < JM; ++j) {
      lo[j] = it.v * pp + it.u;
      it.next();
    }
  }
  auto for_entries = [&](auto fn) {
    if constexpr (CT) {
#pragma unroll
      for (int j = 0; j < JM; ++j)
        if (valid(j)) fn(j, lo[j]);
    } else {
      LaneWalk it(lane, mx);
#pragma unroll
      for (int j = 0; j < JM; ++j) {
        if (valid(j)) fn(j, it.v * pp + it.u);
        it.next();
      }
    }
  };
  auto load = [&](int gp) {
    const T *src = W + (size_t)gp * V;
#pragma unroll
    for (int j = 0; j < JM; ++j)
      if (valid(j)) buf[j] = src[lane + 64 * j];
  };
  load(first);
  for (int q = 0; q < ppw; ++q) {
    const int gp = first + q;
    if (gp >= total) break;
    for_entries([&](int j, int o) { P[o] = buf[j]; });
    wave_sync();
    if (q + 1 < ppw && gp + 1 < total) load(gp + 1);
    wave_contract<T, A, B, ks_of(MY)>(P, 1, pp, mx, my, Fy);
    wave_contract<T, B, A, ks_of(MX)>(P, pp, 1, my, mx, Fx);
    T *dst = W + (size_t)gp * V;
    for_entries([&](int j, int o) { dst[lane + 64 * j] = P[o]; });
    wave_sync();
  }
}

template <typename K>
hipError_t allow_lds(K kernel, size_t shm) {
  if (shm <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

inline int cdiv16(int m) { return (m + 15) / 16; }

}  // namespace

int wide_mfma_frag_count(int m) { return frag_count(m); }

// shapes with every direction of at most 64 nodes and at most 8 output tiles
// per plane in each phase
bool wide_mfma_supported(const int m[3]) {
  const int mmax = std::max(m[0], std::max(m[1], m[2]));
  return mmax <= 64 && cdiv16(m[0]) * cdiv16(m[1]) <= 8 && cdiv16(m[0]) * cdiv16(m[2]) <= 8;
}

namespace {

// Subdomain shapes (n, m_x, m_y, m_z) with compile-time wide kernels; other
// shapes within wide_mfma_supported take the run-time-shape instantiations.
#define SIPG_WIDE_SHAPES(X) X(17, 23, 51, 51)

// waves per workgroup: 4 when two workgroups fit the LDS of a CU, else 8
// when one fits (two waves per SIMD either way), else 4
int waves_for(size_t tables, size_t plane) {
  constexpr size_t lds = 160 * 1024;
  if (2 * (tables + 4 * plane) <= lds) return 4;
  if (tables + 8 * plane <= lds) return 8;
  return 4;
}

template <typename K>
hipError_t set_lds(K kernel, size_t shm) {
  if (shm > 160 * 1024) return hipErrorNotSupported;
  return allow_lds(kernel, shm);
}

template <typename T, int A, int B, int C, int N_, int MX, int MY, int MZ>
hipError_t launch_abc(const SchwarzLaunch<T> &a, hipStream_t st) {
  const int *m = a.tabs.m;
  const size_t eb = sizeof(T);
  const int pp = plane_pitch(m[0], (int)eb);
  const size_t t13 = ((size_t)frag_count(m[0]) + frag_count(m[1])) * eb, p13 = (size_t)pad4(m[1]) * pp * eb;
  const size_t t2 = 2 * (size_t)frag_count(m[2]) * eb, p2 = (size_t)pad4(m[2]) * pp * eb;
  const int w13 = waves_for(t13, p13), w2 = waves_for(t2, p2);
  const size_t s13 = t13 + w13 * p13, s2 = t2 + w2 * p2;
  const int E = a.mesh.E;
  // planes per wave (the tables are staged once per workgroup): about three
  // rounds of workgroups over the CUs (two resident per CU with 4 waves, one
  // with 8), at most 8
  auto ppw_for = [&](int planes, int nw) {
    if (a.wide_planes > 0) return a.wide_planes;
    const int slots = 256 * (nw == 4 ? 2 : 1);
    return std::max(1, std::min(8, E * planes / (3 * nw * slots)));
  };
  hipError_t e;
  {
    const int ppw = ppw_for(m[2], w13), grid = (E * m[2] + w13 * ppw - 1) / (w13 * ppw);
    if (w13 == 8) {
      if ((e = set_lds(wide_mfma1<T, A, B, 8, N_, MX, MY, MZ>, s13)) != hipSuccess) return e;
      wide_mfma1<T, A, B, 8, N_, MX, MY, MZ><<<grid, 512, s13, st>>>(a.mesh, a.n, a.tabs, a.r, a.C, ppw, pp);
    } else {
      if ((e = set_lds(wide_mfma1<T, A, B, 4, N_, MX, MY, MZ>, s13)) != hipSuccess) return e;
      wide_mfma1<T, A, B, 4, N_, MX, MY, MZ><<<grid, 256, s13, st>>>(a.mesh, a.n, a.tabs, a.r, a.C, ppw, pp);
    }
  }
  {
    const int ppw = ppw_for(m[1], w2), grid = (E * m[1] + w2 * ppw - 1) / (w2 * ppw);
    if (w2 == 8) {
      if ((e = set_lds(wide_mfma2<T, A, C, 8, N_, MX, MY, MZ>, s2)) != hipSuccess) return e;
      wide_mfma2<T, A, C, 8, N_, MX, MY, MZ><<<grid, 512, s2, st>>>(E, a.tabs, a.ilam, a.C, ppw, pp);
    } else {
      if ((e = set_lds(wide_mfma2<T, A, C, 4, N_, MX, MY, MZ>, s2)) != hipSuccess) return e;
      wide_mfma2<T, A, C, 4, N_, MX, MY, MZ><<<grid, 256, s2, st>>>(E, a.tabs, a.ilam, a.C, ppw, pp);
    }
  }
  {
    const int ppw = ppw_for(m[2], w13), grid = (E * m[2] + w13 * ppw - 1) / (w13 * ppw);
    if (w13 == 8) {
      if ((e = set_lds(wide_mfma3<T, A, B, 8, N_, MX, MY, MZ>, s13)) != hipSuccess) return e;
      wide_mfma3<T, A, B, 8, N_, MX, MY, MZ><<<grid, 512, s13, st>>>(E, a.tabs, a.C, ppw, pp);
    } else {
      if ((e = set_lds(wide_mfma3<T, A, B, 4, N_, MX, MY, MZ>, s13)) != hipSuccess) return e;
      wide_mfma3<T, A, B, 4, N_, MX, MY, MZ><<<grid, 256, s13, st>>>(E, a.tabs, a.C, ppw, pp);
    }
  }
  return hipGetLastError();
}

template <typename T, int A, int B>
hipError_t launch_ab(const SchwarzLaunch<T> &a, int c, hipStream_t st) {
  switch (c) {
    case 1: return launch_abc<T, A, B, 1, 0, 0, 0, 0>(a, st);
    case 2: return launch_abc<T, A, B, 2, 0, 0, 0, 0>(a, st);
    case 3: if constexpr (A * 3 <= 8) return launch_abc<T, A, B, 3, 0, 0, 0, 0>(a, st); break;
    case 4: if constexpr (A * 4 <= 8) return launch_abc<T, A, B, 4, 0, 0, 0, 0>(a, st); break;
  }
  return hipErrorNotSupported;
}

template <typename T, int A>
hipError_t launch_a(const SchwarzLaunch<T> &a, int b, int c, hipStream_t st) {
  switch (b) {
    case 1: return launch_ab<T, A, 1>(a, c, st);
    case 2: return launch_ab<T, A, 2>(a, c, st);
    case 3: if constexpr (A * 3 <= 8) return launch_ab<T, A, 3>(a, c, st); break;
    case 4: if constexpr (A * 4 <= 8) return launch_ab<T, A, 4>(a, c, st); break;
  }
  return hipErrorNotSupported;
}

constexpr int cdiv16c(int m) { return (m + 15) / 16; }

}  // namespace

template <typename T>
hipError_t launch_schwarz_wide_mfma(const SchwarzLaunch<T> &a, hipStream_t st) {
  const int *m = a.tabs.m;
  if (!wide_mfma_supported(m)) return hipErrorNotSupported;
  for (int k = 0; k < 2; ++k)
    for (int d = 0; d < 3; ++d)
      if (!a.tabs.frag[k][d]) return hipErrorNotSupported;
  // 32-bit offsets into r and into one subdomain's W
  if ((int64_t)a.mesh.E * a.n * a.n * a.n >= ((int64_t)1 << 31)) return hipErrorNotSupported;
#define SIPG_TRY(NN, AX, AY, AZ)                                                                      \
  if (a.n == NN && m[0] == AX && m[1] == AY && m[2] == AZ)                                            \
    return launch_abc<T, cdiv16c(AX), cdiv16c(AY), cdiv16c(AZ), NN, AX, AY, AZ>(a, st);
  SIPG_WIDE_SHAPES(SIPG_TRY)
#undef SIPG_TRY
  const int A = cdiv16(m[0]), B = cdiv16(m[1]), C = cdiv16(m[2]);
  switch (A) {
    case 1: return launch_a<T, 1>(a, B, C, st);
    case 2: return launch_a<T, 2>(a, B, C, st);
    case 3: return launch_a<T, 3>(a, B, C, st);
    case 4: return launch_a<T, 4>(a, B, C, st);
  }
  return hipErrorNotSupported;
}

template hipError_t launch_schwarz_wide_mfma<double>(const SchwarzLaunch<double> &, hipStream_t);
template hipError_t launch_schwarz_wide_mfma<float>(const SchwarzLaunch<float> &, hipStream_t);

}  // namespace sipg
