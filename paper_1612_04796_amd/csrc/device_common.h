// Device-side common definitions for the gfx950 kernels: table views passed
// by value to kernels, XCD-aware block numbering and small helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sipg {

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Renumbering so that XCD x works on one contiguous range
// of blocks keeps face neighbours (which are read again by the next blocks)
// in the same L2.  The map is a bijection of [0, nblocks).
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  constexpr int kXcd = 8;
  const int q = nblocks / kXcd, r = nblocks % kXcd;
  const int x = b % kXcd, local = b / kXcd;
  return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Outputs larger than this many bytes are written with non-temporal stores:
// they cannot stay in the 256 MB last-level cache together with the other
// arrays a kernel and its successor touch (measured faster at 32^3, P = 7;
// at 16^3 the next kernel reads smaller outputs back from that cache).
constexpr long long kStreamOutBytes = 96ll << 20;

template <typename T>
__device__ __forceinline__ void store_out(T *p, T v, bool nt) {
  if (nt) __builtin_nontemporal_store(v, p);
  else *p = v;
}

struct Mesh {
  int ne[3];   // elements per direction
  int E;       // ne[0]*ne[1]*ne[2]
};

__device__ __forceinline__ int elem_index(const Mesh &g, int ex, int ey, int ez) {
  return (ez * g.ne[1] + ey) * g.ne[0] + ex;
}

// First element of the group of EPB consecutive elements that workgroup
// `blk` owns.  When the groups tile the x rows (ne_x divisible by EPB) they
// are visited in column tiles of about 8 x 8 elements in x and y, each tile
// marching along z: a tile's z neighbours were read a tile layer (a few
// hundred KB) earlier and are still in the XCD's L2, where in plain linear
// order they were a whole xy plane (megabytes) earlier and came back from
// memory.  Used when an xy plane of the vector exceeds half an L2 (2 MB);
// otherwise, or when the groups do not tile the rows, linear order.  Both
// orders are bijections onto the groups.  Used by the operator kernel and
// the FP16 local solves; the same order for the FP64/FP32 local solves and
// the assembly was slower (their neighbour reads are already served by
// linear order).
__device__ __forceinline__ int group_first_element(const Mesh &g, int blk, int epb, bool tiled) {
  if (!tiled || g.ne[0] % epb != 0) return blk * epb;
  constexpr int TY = 8;
  const int ngx = g.ne[0] / epb, tgx = epb >= 8 ? 1 : 8 / epb;
  const int n1 = g.ne[1], n2 = g.ne[2];
  const int row = ngx * TY * n2;  // groups in a full row of tiles
  const int ty = blk / row;
  int q = blk - ty * row;
  const int h = min(TY, n1 - ty * TY);
  const int tx = q / (tgx * h * n2);
  q -= tx * tgx * h * n2;
  const int w = min(tgx, ngx - tx * tgx);
  const int ez = q / (w * h);
  q -= ez * w * h;
  const int y = q / w, x = q - y * w;
  return elem_index(g, (tx * tgx + x) * epb, ty * TY + y, ez);
}

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// 1D operator data of one level (eq. (A)): per direction the element diagonal
// block Ld (n x n), the mass diagonal, the scaled face-derivative rows
// DL = D[0][:]/h, DR = D[p][:]/h (GLL) and the penalty.
template <typename T>
struct ApplyTabs {
  const T *Ld[3];
  const T *M[3];
  const T *DL[3];
  const T *DR[3];
  T mu[3];
  // even-odd form of Ld (centro-symmetric: Ld[i][j] = Ld[n-1-i][n-1-j]),
  // h = n/2: Ae[i][j] = (Ld[i][j] + Ld[i][n-1-j])/2, Ao[i][j] = (Ld[i][j] -
  // Ld[i][n-1-j])/2 (i, j < h), then for odd n Ld[i][h] (i < h) and the
  // centre row Ld[h][j] (j <= h)
  const T *LdEO[3];
  // GL basis (gl = 1): the traces TL = phi(-1), TR = phi(+1), full vectors;
  // DL, DR are then (1/h) phi'(-1), (1/h) phi'(+1).  Unused for GLL.
  const T *TL[3];
  const T *TR[3];
  int gl;
};

// Fast-diagonalization data of one level (Sec. 3.1): per direction the
// eigenvectors S (m x m, S[a*m+j] = node a of pair j), the weighted
// eigenvectors WS = diag(w) S and the eigenvalues, with m = n + 2 N_O.
// A table pointer passed through an empty asm statement: loads through the
// returned pointer cannot be hoisted above this point.  Fully unrolled
// contractions take a fresh one per table row, so at most a row of table
// entries (uniform values in scalar registers) is live at a time; with every
// entry loadable up front the compiler fetched them all at the start and
// spilled scalar registers into vector lanes (the even-odd local solves of
// FP64 subdomains of 13 nodes or more per direction: up to 70 % of their
// vector instructions were those spill moves).
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T *;  // read-only, scalar-loadable
template <typename T>
__device__ __forceinline__ ConstPtr<T> row_fence(const T *p) {
  ConstPtr<T> q = (ConstPtr<T>)p;
  asm volatile("" : "+s"(q));
  return q;
}
template <typename T>
struct SchwarzTabs {
  const T *S[3];
  const T *WS[3];
  const T *WST[3];  // (W S)^T: WST[o*m + a] = WS[a*m + o]
  const T *lam[3];
  int m[3];
  int no[3];
  // even-odd form of the same transforms (compile-time-shape kernel): per
  // direction the packed forward and weighted backward half tables, and
  // 1 / (lam_x + lam_y + lam_z) with each direction's modes in even-odd order
  const T *EO[3];
  const T *ilam_eo;
  // matrix-core form of the forward (S, [0]) and weighted backward
  // ((W S)^T, [1]) tables of subdomains wider than the LDS kernels take:
  // fragment-major, entry (ot*KS + ks)*64 + lane = F[4 ks + lane/16][16 ot +
  // lane%16] with F = S or (W S)^T, zero beyond m, KS = ceil(m/4); null when
  // the level has none
  const T *frag[2][3];
};

template <typename T>
__device__ __forceinline__ T block_reduce_sum(T v, T *sh) {
  // deterministic tree reduction over the whole block (blockDim.x <= 1024)
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  T s = 0;
  if (tid == 0)
    for (int w = 0; w < nw; ++w) s += sh[w];
  return s;  // valid in thread 0
}

}  // namespace sipg
