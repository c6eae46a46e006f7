// Local fast-diagonalization solves of the Schwarz smoother in FP16 on the
// matrix cores (MFMA, FP32 accumulation), for the single-precision
// preconditioner (Sec. 3: C_s = W_s (S x S x S) Lambda^{-1} (S x S x S)^T R_s r,
// the six 1D contractions of the tensor-product solve, eq. (FDM)).
//
// A wavefront solves one subdomain (the element-centred m^3 box, m <= 16,
// overlap of at most one element per side) with v_mfma_f32_16x16x16_f16,
// in a tile buffer of its own: the subdomain tensor T[z][y][x] in FP16,
// x contiguous (16 positions, zero beyond m), rows of PY halves, planes of
// PZ halves.  Every 1D contraction takes 16 tensor lines at a time as the B
// operand and the 16 x 16 (zero-padded) 1D table as the A operand:
//   D[o][line] = sum_k A[o][k] T[line][k],
// forward A[o][k] = S[k][o], backward A[o][k] = w[o] S[o][k].  Lane l
// (q = l / 16, c = l % 16) holds A[c][4q..4q+3], B[4q..4q+3][c] and
// D[4q..4q+3][c] of one instruction, so it reads entries 4q..4q+3 of line c
// and writes outputs 4q..4q+3 of the same line back in place: every entry
// is read and written by one lane, and a phase needs no ordering between
// lanes.  Lines along x are read and written 8 bytes at a time, lines along
// y and z entry by entry; PY and PZ are chosen so that the four groups of
// 16 lanes fall on different LDS banks.  The forward z result, scaled by
// 1/lambda, is lane for lane the B operand of the backward z product.
//
// Range: the residual of the subdomain is scaled by a power of two so that
// its largest entry is below 1 (exact), and every table is divided by its
// largest absolute column (forward) or row (backward) sum and 1/lambda by
// its maximum, so no intermediate exceeds 1 in magnitude; the product of
// those factors (kout) and the power of two are applied in FP32 to the
// result.

#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace sipg {
namespace {

typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <int N, int M>
struct MShape {
  static_assert(M <= 16 && M >= N && (M - N) % 2 == 0 && (M - N) / 2 <= N, "unsupported subdomain");
  static constexpr int NO = (M - N) / 2;
  static constexpr int PY = 20;  // halves per row: 16 positions + 4 (row groups 10 banks apart)
  // halves per plane: at least M rows, a multiple of 4, and 4 planes apart
  // (a lane group's stride along z) 16, 24, 40 or 48 banks modulo 64
  static constexpr int pz() {
    for (int p = M * PY;; p += 4) {
      const int b = (2 * p) % 64;
      if (b == 16 || b == 24 || b == 40 || b == 48) return p;
    }
  }
  static constexpr int PZ = pz();
  static constexpr int BUF = M * PZ;               // halves per wavefront
  static constexpr int TILES = (M * M + 15) / 16;  // 16-line tiles of the M^2 lines of a direction
  static constexpr int VOL = M * M * M;
  // wavefronts per SIMD the LDS allows, at most 6 (5 for m = 11, whose
  // unrolled code needs more than the 80 registers of 6)
  static constexpr int CAP = M == 11 ? 5 : 6;
  static constexpr int eu_waves(int wpb) {
    return (160 * 1024 / (wpb * BUF * 2)) * wpb / 4 < CAP ? (160 * 1024 / (wpb * BUF * 2)) * wpb / 4 : CAP;
  }
};

__device__ __forceinline__ f4 mfma(h4 a, h4 b) {
  const f4 z = {0.f, 0.f, 0.f, 0.f};
  return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, z, 0, 0, 0);
}

__device__ __forceinline__ h4 to_h4(f4 v) { return __builtin_convertvector(v, h4); }

// Orders the wavefront's LDS accesses between phases: its earlier LDS
// operations have completed before any later one is issued.
__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
}

// entries 4q..4q+3 of a line with stride ST (halves), zero beyond M
template <int M, int ST>
__device__ __forceinline__ h4 read_line(const _Float16 *p, int q) {
  h4 b;
#pragma unroll
  for (int r = 0; r < 4; ++r) b[r] = 4 * q + r < M ? p[(4 * q + r) * ST] : (_Float16)0;
  return b;
}

template <int M, int ST>
__device__ __forceinline__ void write_line(_Float16 *p, int q, h4 d) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (4 * q + r < M) p[(4 * q + r) * ST] = d[r];
}

// one contraction along y (AX = 1) or z (AX = 2), forward or backward,
// in place: lines (z, x) resp. (y, x)
template <int N, int M, int AX>
__device__ __forceinline__ void phase_yz(_Float16 *buf, h4 tab, int c, int q) {
  using Sh = MShape<N, M>;
  constexpr int ST = AX == 1 ? Sh::PY : Sh::PZ, OT = AX == 1 ? Sh::PZ : Sh::PY;
#pragma unroll
  for (int t = 0; t < Sh::TILES; ++t) {
    const int L = t * 16 + c, o = L / M, x = L - o * M;
    _Float16 *p = buf + o * OT + x;
    const bool ok = L < M * M;
    const h4 b = ok ? read_line<M, ST>(p, q) : h4{0, 0, 0, 0};
    const f4 d = mfma(tab, b);
    if (ok) write_line<M, ST>(p, q, to_h4(d));
  }
  lds_fence();
}

// R_s r of subdomain s into v: lane (x = c, y = 4 yb + q), every z.  The
// offset of an entry splits into a part uniform over the wavefront (z) and
// a per-lane part (x, y); 32-bit offsets (the launcher checks E n^3 < 2^30).
template <int N, int M>
__device__ __forceinline__ void gather(const Mesh &g, const float *__restrict__ r, int s, int c, int q,
                                       float (&v)[M][(M + 3) / 4]) {
  constexpr int NO = (M - N) / 2, MP4 = (M + 3) / 4, N3 = N * N * N;
  auto split = [](int a, int &d, int &loc) {
    d = a < NO ? -1 : (a < NO + N ? 0 : 1);
    loc = a - NO - d * N;
  };
  const int ex = s % g.ne[0], rest = s / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  int dxl, xl;
  split(c, dxl, xl);
  const bool xin = c < M;
  const unsigned xpart = (unsigned)(wrap(ex + dxl, g.ne[0]) * N3 + xl);
  const unsigned plane = (unsigned)(g.ne[0] * g.ne[1] * N3);  // one element layer in z
  unsigned ty[MP4];
  bool ok[MP4];
#pragma unroll
  for (int yb = 0; yb < MP4; ++yb) {
    const int y = 4 * yb + q;
    int dyl, yl;
    split(y, dyl, yl);
    ok[yb] = xin && y < M;
    // byte offset (below 2^32): base in scalar registers + 32-bit lane
    // offset; lanes outside the subdomain read a valid entry and drop it,
    // so every load is issued unconditionally
    ty[yb] = ok[yb] ? 4u * (xpart + (unsigned)(wrap(ey + dyl, g.ne[1]) * g.ne[0] * N3 + yl * N)) : 0u;
  }
#pragma unroll
  for (int z = 0; z < M; ++z) {
    int dzl, zl;
    split(z, dzl, zl);
    const char *rz = reinterpret_cast<const char *>(r + ((size_t)wrap(ez + dzl, g.ne[2]) * plane +
                                                        (unsigned)(zl * N * N)));
#pragma unroll
    for (int yb = 0; yb < MP4; ++yb) {
      const float val = *reinterpret_cast<const float *>(rz + ty[yb]);
      v[z][yb] = ok[yb] ? val : 0.f;
    }
  }
}

// R_s r of subdomain s by rows (n a multiple of 4): lane l takes the x rows
// L = it * 64 + l (L = z m + y) and loads each as three runs, the left
// neighbour's last NO entries, the element's n entries (16-byte loads) and
// the right neighbour's first NO entries.
template <int N, int M>
struct RowGather {
  static constexpr int NO = (M - N) / 2, RPL = (M * M + 63) / 64;
};

template <int N, int M>
__device__ __forceinline__ void gather_rows(const Mesh &g, const float *__restrict__ r, int s, int l,
                                            float (&v)[RowGather<N, M>::RPL][M]) {
  constexpr int NO = (M - N) / 2, N3 = N * N * N;
  static_assert(N % 4 == 0 && NO <= 2, "row gather: n a multiple of 4, at most 2 overlap layers");
  auto split = [](int a, int &d, int &loc) {
    d = a < NO ? -1 : (a < NO + N ? 0 : 1);
    loc = a - NO - d * N;
  };
  const int ex = s % g.ne[0], rest = s / g.ne[0];
  const int ey = rest % g.ne[1], ez = rest / g.ne[1];
  const int exm = wrap(ex - 1, g.ne[0]), exp = wrap(ex + 1, g.ne[0]);
#pragma unroll
  for (int it = 0; it < RowGather<N, M>::RPL; ++it) {
    const int L0 = it * 64 + l, L = L0 < M * M ? L0 : 0;  // idle lanes read row 0 and drop it
    const int z = L / M, y = L - z * M;
    int dzl, zl, dyl, yl;
    split(z, dzl, zl);
    split(y, dyl, yl);
    const int lay = (wrap(ez + dzl, g.ne[2]) * g.ne[1] + wrap(ey + dyl, g.ne[1])) * g.ne[0];
    const unsigned row = (unsigned)((zl * N + yl) * N);
    const float *own = r + ((size_t)(lay + ex) * N3 + row);
    const float *lft = r + ((size_t)(lay + exm) * N3 + row + N - NO);
    const float *rgt = r + ((size_t)(lay + exp) * N3 + row);
    float e[M];
#pragma unroll
    for (int j = 0; j < N / 4; ++j) {
      const f4 o4 = reinterpret_cast<const f4 *>(own)[j];
#pragma unroll
      for (int k = 0; k < 4; ++k) e[NO + 4 * j + k] = o4[k];
    }
    if constexpr (NO == 2) {
      typedef float f2 __attribute__((ext_vector_type(2)));
      const f2 a = *reinterpret_cast<const f2 *>(lft), b = *reinterpret_cast<const f2 *>(rgt);
      e[0] = a[0], e[1] = a[1], e[M - 2] = b[0], e[M - 1] = b[1];
    } else if constexpr (NO == 1) {
      e[0] = *lft, e[M - 1] = *rgt;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) v[it][k] = L0 < M * M ? e[k] : 0.f;
  }
}

// One wavefront per subdomain, WPB wavefronts per workgroup; registers
// capped so that as many wavefronts per SIMD are resident as the LDS allows.
template <int N, int M, int WPB>
__global__ void __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(MShape<N, M>::eu_waves(WPB))))
schwarz_fdm_mfma(Mesh g, MfmaTabs tb, const float *__restrict__ r, float *__restrict__ C, bool tiled) {
  using Sh = MShape<N, M>;
  constexpr int PY = Sh::PY, PZ = Sh::PZ, TILES = Sh::TILES;
  __shared__ __align__(16) _Float16 tile[WPB][Sh::BUF];
  // the wavefront index is uniform over the wavefront: keep it (and the
  // subdomain index) in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
  _Float16 *buf = tile[w];
  const int s = group_first_element(g, xcd_block(blockIdx.x, gridDim.x), WPB, tiled) + w;
  if (s >= g.E) return;  // wavefronts never wait for each other

  auto lane_tab = [&](const _Float16 *p) { return reinterpret_cast<const h4 *>(p)[l]; };
  const h4 fx = lane_tab(tb.fwd[0]), fy = lane_tab(tb.fwd[1]), fz = lane_tab(tb.fwd[2]);
  const h4 bx = lane_tab(tb.bwd[0]), by = lane_tab(tb.bwd[1]), bz = lane_tab(tb.bwd[2]);
  // R_s r scaled by a power of two (largest entry below 1) into T[z][y][x],
  // zero for x >= m
  float unscale;
  if constexpr (N % 4 == 0) {
    constexpr int RPL = RowGather<N, M>::RPL;
    float v[RPL][M];
    gather_rows<N, M>(g, r, s, l, v);
    float mx = 0.f;
#pragma unroll
    for (int it = 0; it < RPL; ++it)
#pragma unroll
      for (int k = 0; k < M; ++k) mx = fmaxf(mx, fabsf(v[it][k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    int ex2 = 0;
    if (mx > 0.f) (void)frexpf(mx, &ex2);  // mx = f 2^ex2, f in [0.5, 1)
    const float scale = ldexpf(1.f, -ex2);
    unscale = ldexpf(tb.kout, ex2);
#pragma unroll
    for (int it = 0; it < RPL; ++it) {
      const int L = it * 64 + l, z = L / M, y = L - z * M;
      if (L < M * M) {
        h4 *row = reinterpret_cast<h4 *>(buf + z * PZ + y * PY);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          h4 hv;
#pragma unroll
          for (int k = 0; k < 4; ++k) hv[k] = 4 * j + k < M ? (_Float16)(v[it][4 * j + k] * scale) : (_Float16)0;
          row[j] = hv;
        }
      }
    }
  } else {
    float v[M][(M + 3) / 4];
    gather<N, M>(g, r, s, c, q, v);
    float mx = 0.f;
#pragma unroll
    for (int z = 0; z < M; ++z)
#pragma unroll
      for (int yb = 0; yb < (M + 3) / 4; ++yb) mx = fmaxf(mx, fabsf(v[z][yb]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    int ex2 = 0;
    if (mx > 0.f) (void)frexpf(mx, &ex2);
    const float scale = ldexpf(1.f, -ex2);
    unscale = ldexpf(tb.kout, ex2);
#pragma unroll
    for (int z = 0; z < M; ++z)
#pragma unroll
      for (int yb = 0; yb < (M + 3) / 4; ++yb)
        if (4 * yb + q < M) buf[z * PZ + (4 * yb + q) * PY + c] = (_Float16)(v[z][yb] * scale);
  }
  lds_fence();

  // forward x: lines (z, y), entries 4q..4q+3 of a line in one 8-byte access
#pragma unroll
  for (int t = 0; t < TILES; ++t) {
    const int L = t * 16 + c, z = L / M, y = L - z * M;
    h4 *p = reinterpret_cast<h4 *>(buf + z * PZ + y * PY + 4 * q);
    const bool ok = L < M * M;
    const h4 b = ok ? *p : h4{0, 0, 0, 0};
    const f4 d = mfma(fx, b);
    if (ok) *p = to_h4(d);
  }
  lds_fence();
  phase_yz<N, M, 1>(buf, fy, c, q);  // forward y
  // forward z, 1/lambda, backward z: lines (y, x)
  {
    const f4 *il = reinterpret_cast<const f4 *>(tb.ilam);
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
      const int L = t * 16 + c, y = L / M, x = L - y * M;
      _Float16 *p = buf + y * PY + x;
      const bool ok = L < M * M;
      const h4 b = ok ? read_line<M, PZ>(p, q) : h4{0, 0, 0, 0};
      const f4 d = mfma(fz, b) * il[t * 64 + l];  // D[k = 4q + r][line]
      const f4 u = mfma(bz, to_h4(d));            // D[z' = 4q + r][line]
      if (ok) write_line<M, PZ>(p, q, to_h4(u));
    }
    lds_fence();
  }
  phase_yz<N, M, 1>(buf, by, c, q);  // backward y
  // backward x into C[s] (layout [z][y][x]), times kout 2^ex2
  float *Cs = C + (int64_t)s * Sh::VOL;
#pragma unroll
  for (int t = 0; t < TILES; ++t) {
    const int L = t * 16 + c, z = L / M, y = L - z * M;
    const bool ok = L < M * M;
    const h4 b = ok ? *reinterpret_cast<const h4 *>(buf + z * PZ + y * PY + 4 * q) : h4{0, 0, 0, 0};
    const f4 d = mfma(bx, b) * unscale;  // D[x' = 4q + r][line]
    if (ok) {
      float *row = Cs + (z * M + y) * M;
      if constexpr (M % 4 == 0) {
        if (4 * q < M) *reinterpret_cast<f4 *>(row + 4 * q) = d;
      } else {
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
          if (4 * q + rr < M) row[4 * q + rr] = d[rr];
      }
    }
  }
}

constexpr int kWpb = 4;

template <int N, int M>
hipError_t launch_mfma(const Mesh &mesh, const MfmaTabs &tb, const float *r, float *C, hipStream_t st) {
  if ((int64_t)mesh.E * N * N * N >= ((int64_t)1 << 30)) return hipErrorInvalidValue;
  // column-tile visiting order when an xy plane of r exceeds half an L2 (the
  // gather of R_s r then finds the z neighbours' layers still in L2)
  const bool tiled = (int64_t)mesh.ne[0] * mesh.ne[1] * N * N * N * (int64_t)sizeof(float) >= (2 << 20);
  schwarz_fdm_mfma<N, M, kWpb><<<(mesh.E + kWpb - 1) / kWpb, 64 * kWpb, 0, st>>>(mesh, tb, r, C, tiled);
  return hipGetLastError();
}

}  // namespace

// the (n, m) pairs with a compiled kernel: P = 7 and 8 with one and two
// overlap layers
#define SIPG_MFMA_SHAPES(X) X(8, 10) X(8, 12) X(9, 11) X(9, 13)

bool mfma_fdm_supported(int n, const int m[3]) {
  if (m[0] != m[1] || m[1] != m[2]) return false;
#define SIPG_HAS(NN, MM) \
  if (n == NN && m[0] == MM) return true;
  SIPG_MFMA_SHAPES(SIPG_HAS)
#undef SIPG_HAS
  return false;
}

int mfma_fdm_tiles(int m) { return (m * m + 15) / 16; }

hipError_t launch_schwarz_mfma(const Mesh &mesh, int n, const int m[3], const MfmaTabs &tb, const float *r,
                               float *C, hipStream_t st) {
  if (!mfma_fdm_supported(n, m)) return hipErrorInvalidValue;
#define SIPG_GO(NN, MM) \
  if (n == NN && m[0] == MM) return launch_mfma<NN, MM>(mesh, tb, r, C, st);
  SIPG_MFMA_SHAPES(SIPG_GO)
#undef SIPG_GO
  return hipErrorInvalidValue;
}

}  // namespace sipg
