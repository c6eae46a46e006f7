// C ABI of the solver (include/sipg_mg.h): context set-up, the multigrid
// V-cycle of Algorithm 1, the MG and flexible-CG solvers, and the host-only
// table queries.  Every device operation is a kernel launch on the context
// stream; host synchronization happens only where a solver reads a residual
// norm.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "host_tables.h"
#include "kernels.h"
#include "sipg_mg.h"
#include "solver_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

struct HipFailure : std::runtime_error {
  explicit HipFailure(const std::string &s) : std::runtime_error(s) {}
};

void check(hipError_t e, const char *what) {
  if (e != hipSuccess) throw HipFailure(std::string(what) + ": " + hipGetErrorString(e));
}

// Device table views of one level in precision T.
template <typename T>
struct LevelTabs {
  sipg::ApplyTabs<T> apply;
  sipg::SchwarzTabs<T> schwarz;
  const T *J = nullptr;  // n x n_prev (levels >= 1)
  const T *ilam = nullptr;  // 1 / (lam_x + lam_y + lam_z) per subdomain entry (levels >= 1)
  sipg::MfmaTabs mfma{};    // FP16 matrix-core local solves (FP32 levels that have them)
  bool has_mfma = false;
  int apply_epb = 0;        // launch parameters chosen by sipg_autotune (0: defaults)
  int schwarz_spb = 0;
  int n = 0, nc = 0;
  int64_t ndof = 0;
};

// Work vectors of the V-cycle in precision T.
template <typename T>
struct Work {
  std::vector<T *> u, f;  // levels 0..L-1 (u[0] unused), plus top-level pair for internal use
  T *uL = nullptr, *fL = nullptr;
  T *r = nullptr;         // residual scratch, top-level size
  T *C = nullptr;         // Schwarz correction scratch
  T *big = nullptr;       // scratch of the large-element (n = 33) operator and transfers
  bool ready = false;
};

// Arena for uploading tables: host staging with aligned offsets.
struct Arena {
  std::vector<unsigned char> host;
  template <typename T>
  size_t put(const std::vector<double> &v) {
    size_t off = (host.size() + 255) / 256 * 256;
    host.resize(off + v.size() * sizeof(T));
    T *p = reinterpret_cast<T *>(host.data() + off);
    for (size_t i = 0; i < v.size(); ++i) p[i] = (T)v[i];
    return off;
  }
};

}  // namespace

struct sipg_ctx {
  sipg::HierarchyHost H;
  hipStream_t stream = nullptr;
  int device = 0;                       // device current at sipg_setup
  int L = 0;
  sipg::Mesh mesh{};
  std::vector<void *> allocs;
  unsigned char *tab_dev = nullptr;
  std::vector<LevelTabs<double>> t64;
  std::vector<LevelTabs<float>> t32;
  sipg::CoarseLaunch coarse{};
  double *u0 = nullptr;                 // level-0 solution, always FP64
  Work<double> w64;
  Work<float> w32;
  // flexible CG vectors (FP64, top level) and device scalars
  double *cg_r = nullptr, *cg_p = nullptr, *cg_q = nullptr, *cg_z = nullptr;
  double *cg_b = nullptr;               // the solvers' right side, projected onto 1^perp
  double f_mean = 0.0;                  // Euclidean mean removed from f by the last solve
  double *scal = nullptr;               // the FS_COUNT slots of FcgScalar
  double *partial = nullptr;            // 2 * kDotBlocks
  double *host_scal = nullptr;          // pinned host mirror
  double *host_scal_dev = nullptr;      // its device-mapped address
  int *rhs_k = nullptr;
  double *rhs_phi = nullptr, *rhs_amp = nullptr;
  const double *xi_top = nullptr, *mass_top[3] = {nullptr, nullptr, nullptr};
  std::vector<double> hist;
  size_t bytes = 0;
  int wide_planes = 0;                  // SIPG_OPT_WIDE_PLANES (0: automatic)
  bool use_graph = false;               // replay the preconditioner from a captured graph
  hipGraphExec_t precond_graph = nullptr;
  bool graph_failed = false;
  bool x_pending = false;  // flexible CG: x += alpha p not yet applied
  // SIPG_OPT_TRACE_KERNEL: event pairs around the launches of one top-level
  // FP64 kernel (none while a graph is being captured)
  int trace_kernel = -1;
  bool capturing = false;
  std::vector<hipEvent_t> trace_ev;  // 2 * kTraceMax, created on first use
  int trace_n = 0;

  template <typename T>
  T *alloc(size_t count) {
    void *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e == hipErrorOutOfMemory) throw std::bad_alloc();
    check(e, "hipMalloc");
    allocs.push_back(p);
    bytes += count * sizeof(T);
    return static_cast<T *>(p);
  }
  ~sipg_ctx() {
    if (precond_graph) (void)hipGraphExecDestroy(precond_graph);
    for (hipEvent_t e : trace_ev) (void)hipEventDestroy(e);
    for (void *p : allocs) (void)hipFree(p);
    if (host_scal) (void)hipHostFree(host_scal);
  }
};

namespace {

template <typename T>
LevelTabs<T> &tabs_of(sipg_ctx *c, int l);
template <>
LevelTabs<double> &tabs_of<double>(sipg_ctx *c, int l) { return c->t64[l]; }
template <>
LevelTabs<float> &tabs_of<float>(sipg_ctx *c, int l) { return c->t32[l]; }
template <typename T>
Work<T> &work_of(sipg_ctx *c);
template <>
Work<double> &work_of<double>(sipg_ctx *c) { return c->w64; }
template <>
Work<float> &work_of<float>(sipg_ctx *c) { return c->w32; }

size_t max_sub(const sipg::HierarchyHost &H) {
  size_t mx = 1;
  for (size_t l = 1; l < H.lev.size(); ++l)
    mx = std::max(mx, (size_t)H.lev[l].dir[0].m * H.lev[l].dir[1].m * H.lev[l].dir[2].m);
  return mx;
}

int64_t level_ndof(const sipg::HierarchyHost &H, int l) {
  const int64_t E = (int64_t)H.prm.ne[0] * H.prm.ne[1] * H.prm.ne[2];
  const int64_t n = H.lev[l].n;
  return E * n * n * n;
}

// Bytes of one precision's V-cycle work space (without the scratch of the
// large-element operator, big_bytes).
size_t work_bytes(const sipg::HierarchyHost &H, size_t eb) {
  const int L = (int)H.lev.size() - 1;
  const int64_t E = (int64_t)H.prm.ne[0] * H.prm.ne[1] * H.prm.ne[2];
  size_t b = 0;
  for (int l = 0; l < L; ++l) b += 2 * (size_t)level_ndof(H, l) * eb;
  b += 3 * (size_t)level_ndof(H, L) * eb;  // r plus an internal top-level u, f pair
  b += (size_t)E * max_sub(H) * eb;
  return b;
}

// Values of the scratch of the top level's large-element operator passes
// and transfers (0 when the top order fits the LDS kernels).
size_t big_count(const sipg::HierarchyHost &H) {
  const int L = (int)H.lev.size() - 1;
  const int64_t E = (int64_t)H.prm.ne[0] * H.prm.ne[1] * H.prm.ne[2];
  const int nt = H.lev[L].n;
  if (L == 0 || !sipg::apply_is_large(nt)) return 0;
  return (size_t)E * ((size_t)nt * nt * nt + (size_t)nt * nt * H.lev[L - 1].n);
}

// the large-element scratch of precision T (allocated on first use)
template <typename T>
T *ensure_big(sipg_ctx *c) {
  Work<T> &w = work_of<T>(c);
  if (!w.big) {
    const size_t n = big_count(c->H);
    if (n) w.big = c->alloc<T>(n);
  }
  return w.big;
}

template <typename T>
void ensure_work(sipg_ctx *c) {
  Work<T> &w = work_of<T>(c);
  if (w.ready) return;
  const sipg::HierarchyHost &H = c->H;
  w.u.assign(c->L + 1, nullptr);
  w.f.assign(c->L + 1, nullptr);
  for (int l = 0; l < c->L; ++l) {
    w.u[l] = c->alloc<T>(level_ndof(H, l));
    w.f[l] = c->alloc<T>(level_ndof(H, l));
  }
  w.uL = c->alloc<T>(level_ndof(H, c->L));
  w.fL = c->alloc<T>(level_ndof(H, c->L));
  w.r = c->alloc<T>(level_ndof(H, c->L));
  w.C = c->alloc<T>((size_t)c->mesh.E * max_sub(H));
  ensure_big<T>(c);
  w.ready = true;
}

// Even-odd form of the element block Ld of one direction (see ApplyTabs):
// [Ae (h x h), Ao (h x h), for odd n: Ld[i][h] (h), Ld[h][j] (h + 1)].
std::vector<double> pack_ld_even_odd(const sipg::Dir1D &D) {
  const int n = D.n, h = n / 2;
  auto L = [&](int i, int j) { return D.Ld[(size_t)i * n + j]; };
  std::vector<double> t;
  for (int i = 0; i < h; ++i)
    for (int j = 0; j < h; ++j) t.push_back(0.5 * (L(i, j) + L(i, n - 1 - j)));
  for (int i = 0; i < h; ++i)
    for (int j = 0; j < h; ++j) t.push_back(0.5 * (L(i, j) - L(i, n - 1 - j)));
  if (n & 1) {
    for (int i = 0; i < h; ++i) t.push_back(L(i, h));
    for (int j = 0; j <= h; ++j) t.push_back(L(h, j));
  }
  return t;
}

// Even-odd half tables of one direction, in the layout the compile-time-shape
// Schwarz kernel reads (H = m/2, NE = m - H even modes, NO = H odd modes):
//   forward  FE[a][j] = S[a][j] (a < H, j < NE),  FC[j] = S[H][j] (m odd),
//            FO[a][j] = S[a][NE + j] (a < H, j < H)
//   backward BE, BC, BO: the same entries times the hat weight w[a]
// with S the even-odd eigenvectors (even modes first).  The forward transform
// then contracts sums and differences of mirrored entries; the backward one
// forms E_a (even part) and O_a (odd part), x[a] = E_a + O_a and
// x[m-1-a] = E_a - O_a (the weights are symmetric).
std::vector<double> pack_even_odd(const sipg::Dir1D &D) {
  const int m = D.m, H = m / 2, NE = m - H, odd = m & 1;
  std::vector<double> t;
  t.reserve(2 * ((size_t)H * NE + (size_t)odd * NE + (size_t)H * H));
  for (int pass = 0; pass < 2; ++pass) {
    auto wt = [&](int a) { return pass ? D.wsub[a] : 1.0; };
    for (int a = 0; a < H; ++a)
      for (int j = 0; j < NE; ++j) t.push_back(wt(a) * D.S_eo[(size_t)a * m + j]);
    if (odd)
      for (int j = 0; j < NE; ++j) t.push_back(wt(H) * D.S_eo[(size_t)H * m + j]);
    for (int a = 0; a < H; ++a)
      for (int j = 0; j < H; ++j) t.push_back(wt(a) * D.S_eo[(size_t)a * m + NE + j]);
  }
  return t;
}

// Tables of the FP16 matrix-core local solves of one level (cubic
// subdomains): per direction the forward operand S / f_d and the backward
// operand W S / g_d in the lane order of a 16 x 16 MFMA operand, and 1/lambda
// over its maximum in the order of the forward z result; see MfmaTabs.
struct MfmaHost {
  std::vector<double> fwd[3], bwd[3], ilam;
  double kout = 1.0;
};

MfmaHost build_mfma_tables(const sipg::LevelHost &lv) {
  MfmaHost h;
  const int m = lv.dir[0].m, tiles = sipg::mfma_fdm_tiles(m);
  for (int d = 0; d < 3; ++d) {
    const sipg::Dir1D &D = lv.dir[d];
    double f = 0.0, g = 0.0;
    for (int j = 0; j < m; ++j) {
      double cs = 0.0, rs = 0.0;
      for (int a = 0; a < m; ++a) {
        cs += std::fabs(D.S[(size_t)a * m + j]);
        rs += std::fabs(D.wsub[j] * D.S[(size_t)j * m + a]);
      }
      f = std::max(f, cs);
      g = std::max(g, rs);
    }
    h.fwd[d].assign(256, 0.0);
    h.bwd[d].assign(256, 0.0);
    for (int l = 0; l < 64; ++l)
      for (int v = 0; v < 4; ++v) {
        const int k = 4 * (l / 16) + v, c = l % 16;
        if (k < m && c < m) {
          h.fwd[d][l * 4 + v] = D.S[(size_t)k * m + c] / f;
          h.bwd[d][l * 4 + v] = D.wsub[c] * D.S[(size_t)c * m + k] / g;
        }
      }
    h.kout *= f * g;
  }
  const sipg::Dir1D &X = lv.dir[0], &Y = lv.dir[1], &Z = lv.dir[2];
  double imax = 0.0;
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) imax = std::max(imax, 1.0 / (X.lam[i] + Y.lam[j] + Z.lam[k]));
  h.ilam.assign((size_t)tiles * 256, 0.0);
  for (int t = 0; t < tiles; ++t)
    for (int l = 0; l < 64; ++l)
      for (int v = 0; v < 4; ++v) {
        const int line = t * 16 + l % 16, jy = line / m, jx = line % m, jz = 4 * (l / 16) + v;
        if (line < m * m && jz < m)
          h.ilam[((size_t)t * 64 + l) * 4 + v] = 1.0 / (X.lam[jx] + Y.lam[jy] + Z.lam[jz]) / imax;
      }
  h.kout *= imax;
  return h;
}

// Offsets of one level's tables in the arena.
struct TabOff {
  size_t Ld[3], LdEO[3], M[3], DL[3], DR[3], TL[3], TR[3], S[3], WS[3], WST[3], lam[3], EO[3], J, ilam, ilam_eo;
  size_t mf[3], mb[3], mil;
  double kout;
  bool mfma;
  size_t frag[2][3];
  bool wide_mfma;
};

// Fragment-major matrix-core table of one direction (see SchwarzTabs::frag):
// F[a][o] = S[a][o] (forward) or w[o] S[o][a] (weighted backward).
std::vector<double> wide_frag_table(const sipg::Dir1D &D, bool backward) {
  const int m = D.m, OT = (m + 15) / 16, KS = (m + 3) / 4;
  std::vector<double> t((size_t)sipg::wide_mfma_frag_count(m), 0.0);
  for (int ot = 0; ot < OT; ++ot)
    for (int ks = 0; ks < KS; ++ks)
      for (int lane = 0; lane < 64; ++lane) {
        const int a = 4 * ks + lane / 16, o = 16 * ot + lane % 16;
        if (a < m && o < m)
          t[((size_t)ot * KS + ks) * 64 + lane] =
              backward ? D.wsub[o] * D.S[(size_t)o * m + a] : D.S[(size_t)a * m + o];
      }
  return t;
}

// Every device table of a context, staged on the host (built by
// build_table_arena, uploaded by upload_tables; its size is part of
// sipg_footprint).
struct TableArena {
  Arena A;
  std::vector<TabOff> o64, o32;
  size_t cS[3], cC[3], cL[3], oxi, omass[3];
};

TableArena build_table_arena(const sipg::HierarchyHost &H, int64_t E) {
  const int L = (int)H.lev.size() - 1;
  TableArena T_;
  Arena &A = T_.A;
  std::vector<TabOff> &o64 = T_.o64, &o32 = T_.o32;
  o64.assign(L + 1, TabOff{});
  o32.assign(L + 1, TabOff{});
  auto put_level = [&](auto tag, std::vector<TabOff> &off) {
    using T = decltype(tag);
    for (int l = 0; l <= L; ++l) {
      const sipg::LevelHost &lv = H.lev[l];
      for (int d = 0; d < 3; ++d) {
        const sipg::Dir1D &D = lv.dir[d];
        off[l].Ld[d] = A.put<T>(D.Ld);
        off[l].LdEO[d] = A.put<T>(pack_ld_even_odd(D));
        off[l].M[d] = A.put<T>(D.mass);
        off[l].DL[d] = A.put<T>(D.DLs);
        off[l].DR[d] = A.put<T>(D.DRs);
        off[l].TL[d] = A.put<T>(D.TL);
        off[l].TR[d] = A.put<T>(D.TR);
        if (l > 0) {
          std::vector<double> WS(D.S);
          for (int a = 0; a < D.m; ++a)
            for (int j = 0; j < D.m; ++j) WS[a * D.m + j] *= D.wsub[a];
          std::vector<double> WST(WS.size());
          for (int a = 0; a < D.m; ++a)
            for (int j = 0; j < D.m; ++j) WST[j * D.m + a] = WS[a * D.m + j];
          off[l].S[d] = A.put<T>(D.S);
          off[l].WS[d] = A.put<T>(WS);
          off[l].WST[d] = A.put<T>(WST);
          off[l].lam[d] = A.put<T>(D.lam);
          off[l].EO[d] = A.put<T>(pack_even_odd(D));
        }
      }
      if (l > 0) {
        off[l].J = A.put<T>(lv.J);
        const sipg::Dir1D &X = lv.dir[0], &Y = lv.dir[1], &Z = lv.dir[2];
        std::vector<double> il((size_t)X.m * Y.m * Z.m);
        for (int cz = 0; cz < Z.m; ++cz)
          for (int by = 0; by < Y.m; ++by)
            for (int ax = 0; ax < X.m; ++ax)
              il[((size_t)cz * Y.m + by) * X.m + ax] = 1.0 / (X.lam[ax] + Y.lam[by] + Z.lam[cz]);
        off[l].ilam = A.put<T>(il);
        for (int cz = 0; cz < Z.m; ++cz)
          for (int by = 0; by < Y.m; ++by)
            for (int ax = 0; ax < X.m; ++ax)
              il[((size_t)cz * Y.m + by) * X.m + ax] = 1.0 / (X.lam_eo[ax] + Y.lam_eo[by] + Z.lam_eo[cz]);
        off[l].ilam_eo = A.put<T>(il);
        const int m3[3] = {X.m, Y.m, Z.m};
        off[l].wide_mfma = !sipg::schwarz_fits_lds(m3, sizeof(double)) && sipg::wide_mfma_supported(m3);
        if (off[l].wide_mfma)
          for (int k = 0; k < 2; ++k)
            for (int d = 0; d < 3; ++d) off[l].frag[k][d] = A.put<T>(wide_frag_table(lv.dir[d], k == 1));
        off[l].mfma = std::is_same<T, float>::value && sipg::mfma_fdm_supported(lv.n, m3) &&
                      E * lv.n * lv.n * lv.n < ((int64_t)1 << 30);
        if (off[l].mfma) {
          const MfmaHost mh = build_mfma_tables(lv);
          for (int d = 0; d < 3; ++d) {
            off[l].mf[d] = A.put<_Float16>(mh.fwd[d]);
            off[l].mb[d] = A.put<_Float16>(mh.bwd[d]);
          }
          off[l].mil = A.put<float>(mh.ilam);
          off[l].kout = mh.kout;
        }
      }
    }
  };
  put_level(double(), o64);
  put_level(float(), o32);
  size_t *cS = T_.cS, *cC = T_.cC, *cL = T_.cL;
  for (int d = 0; d < 3; ++d) {
    const int N = H.coarse.N[d];
    std::vector<double> cs(N, 0.0);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) cs[j] += H.coarse.S[d][i * N + j];
    cS[d] = A.put<double>(H.coarse.S[d]);
    cC[d] = A.put<double>(cs);
    cL[d] = A.put<double>(H.coarse.lam[d]);
  }
  T_.oxi = A.put<double>(H.lev[L].dir[0].xi);
  for (int d = 0; d < 3; ++d) T_.omass[d] = A.put<double>(H.lev[L].dir[d].mass);
  return T_;
}

void upload_tables(sipg_ctx *c) {
  const sipg::HierarchyHost &H = c->H;
  TableArena T_ = build_table_arena(H, c->mesh.E);
  Arena &A = T_.A;
  std::vector<TabOff> &o64 = T_.o64, &o32 = T_.o32;
  const size_t *cS = T_.cS, *cC = T_.cC, *cL = T_.cL, oxi = T_.oxi, *omass = T_.omass;

  c->tab_dev = c->alloc<unsigned char>(A.host.size());
  check(hipMemcpyAsync(c->tab_dev, A.host.data(), A.host.size(), hipMemcpyHostToDevice, c->stream),
        "table upload");
  check(hipStreamSynchronize(c->stream), "table upload");

  auto fill = [&](auto tag, std::vector<TabOff> &off, auto &dst) {
    using T = decltype(tag);
    dst.assign(c->L + 1, {});
    for (int l = 0; l <= c->L; ++l) {
      const sipg::LevelHost &lv = H.lev[l];
      auto &t = dst[l];
      t.n = lv.n;
      t.nc = l > 0 ? H.lev[l - 1].n : 0;
      t.ndof = level_ndof(H, l);
      t.apply.gl = H.prm.basis == SIPG_BASIS_GL;
      for (int d = 0; d < 3; ++d) {
        t.apply.Ld[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].Ld[d]);
        t.apply.M[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].M[d]);
        t.apply.LdEO[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].LdEO[d]);
        t.apply.DL[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].DL[d]);
        t.apply.DR[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].DR[d]);
        t.apply.TL[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].TL[d]);
        t.apply.TR[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].TR[d]);
        t.apply.mu[d] = (T)lv.dir[d].mu;
        if (l > 0) {
          t.schwarz.S[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].S[d]);
          t.schwarz.WS[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].WS[d]);
          t.schwarz.lam[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].lam[d]);
          t.schwarz.EO[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].EO[d]);
          t.schwarz.WST[d] = reinterpret_cast<const T *>(c->tab_dev + off[l].WST[d]);
          t.schwarz.m[d] = lv.dir[d].m;
          t.schwarz.no[d] = lv.dir[d].no;
        }
      }
      if (l > 0) {
        t.J = reinterpret_cast<const T *>(c->tab_dev + off[l].J);
        t.ilam = reinterpret_cast<const T *>(c->tab_dev + off[l].ilam);
        t.schwarz.ilam_eo = reinterpret_cast<const T *>(c->tab_dev + off[l].ilam_eo);
        for (int k = 0; k < 2; ++k)
          for (int d = 0; d < 3; ++d)
            t.schwarz.frag[k][d] =
                off[l].wide_mfma ? reinterpret_cast<const T *>(c->tab_dev + off[l].frag[k][d]) : nullptr;
        t.has_mfma = off[l].mfma;
        if (t.has_mfma) {
          for (int d = 0; d < 3; ++d) {
            t.mfma.fwd[d] = reinterpret_cast<const _Float16 *>(c->tab_dev + off[l].mf[d]);
            t.mfma.bwd[d] = reinterpret_cast<const _Float16 *>(c->tab_dev + off[l].mb[d]);
          }
          t.mfma.ilam = reinterpret_cast<const float *>(c->tab_dev + off[l].mil);
          t.mfma.kout = (float)off[l].kout;
        }
      }
    }
  };
  fill(double(), o64, c->t64);
  fill(float(), o32, c->t32);
  for (int d = 0; d < 3; ++d) {
    c->coarse.ne[d] = H.prm.ne[d];
    c->coarse.N[d] = H.coarse.N[d];
    c->coarse.S[d] = reinterpret_cast<const double *>(c->tab_dev + cS[d]);
    c->coarse.colsum[d] = reinterpret_cast<const double *>(c->tab_dev + cC[d]);
    c->coarse.lam[d] = reinterpret_cast<const double *>(c->tab_dev + cL[d]);
    c->coarse.zero[d] = H.coarse.zero[d];
  }
  c->xi_top = reinterpret_cast<const double *>(c->tab_dev + oxi);
  for (int d = 0; d < 3; ++d) c->mass_top[d] = reinterpret_cast<const double *>(c->tab_dev + omass[d]);
}

// ---- level operations -----------------------------------------------------
constexpr int kTraceMax = 1024;

// Opens a traced launch of `kernel` on level l in precision T: returns the
// slot of its event pair (its start event recorded), or -1 when not traced.
// Traced: top-level launches in the preconditioner's precision (FP64, or
// FP32 for precond_bits 32 and 16).
template <typename T>
int trace_begin(sipg_ctx *c, int kernel, int l) {
  const bool prec = std::is_same<T, double>::value == (c->H.prm.precond_bits == 64);
  if (c->trace_kernel != kernel || l != c->L || !prec || c->capturing || c->trace_n >= kTraceMax) return -1;
  const int k = c->trace_n++;
  check(hipEventRecord(c->trace_ev[2 * k], c->stream), "trace event");
  return k;
}

void trace_end(sipg_ctx *c, int k) {
  if (k >= 0) check(hipEventRecord(c->trace_ev[2 * k + 1], c->stream), "trace event");
}

template <typename T>
void run_apply(sipg_ctx *c, const sipg::ApplyLaunch<T> &a, const char *what) {
  if (sipg::apply_is_large(a.n)) {
    check(sipg::launch_apply_large<T>(a, ensure_big<T>(c), c->stream), what);
  } else {
    check(sipg::launch_apply<T>(a, c->stream), what);
  }
}

template <typename T>
void op_apply(sipg_ctx *c, int l, const T *u, T *y, T *partial) {
  const LevelTabs<T> &t = tabs_of<T>(c, l);
  sipg::ApplyLaunch<T> a{c->mesh, t.n, t.apply, u, nullptr, y, sipg::APPLY_PLAIN, partial, nullptr, 0, t.apply_epb};
  run_apply<T>(c, a, "apply_A");
}

// r = f - A u; with `partial`, also one partial sum of r.r per workgroup
template <typename T>
void op_residual(sipg_ctx *c, int l, const T *u, const T *f, T *r, T *partial = nullptr) {
  const LevelTabs<T> &t = tabs_of<T>(c, l);
  sipg::ApplyLaunch<T> a{c->mesh, t.n, t.apply, u, f, r, sipg::APPLY_RESID, partial, nullptr, 0, t.apply_epb};
  const int k = trace_begin<T>(c, SIPG_KERNEL_RESIDUAL, l);
  run_apply<T>(c, a, "residual");
  trace_end(c, k);
}

// ||f - A u||^2 into scal[slot], r = f - A u (FP64, top level)
// ||f - A u||^2 into scal[slot]; with publish the scalar block is also
// written to the host mirror
void residual_norm2(sipg_ctx *c, const double *u, const double *f, double *r, int slot, bool publish = false) {
  op_residual<double>(c, c->L, u, f, r, c->partial);
  check(sipg::launch_finalize(c->partial, sipg::apply_num_blocks(c->mesh.E, c->H.lev[c->L].n, c->t64[c->L].apply_epb),
                              1.0, c->scal + slot, c->stream, c->scal, publish ? c->host_scal_dev : nullptr,
                              sipg::FS_COUNT),
        "residual norm");
}

template <typename T>
void op_residual_restrict(sipg_ctx *c, int l, const T *u, const T *f, T *fc) {
  const LevelTabs<T> &t = tabs_of<T>(c, l);
  sipg::ApplyLaunch<T> a{c->mesh, t.n, t.apply, u, f, fc, sipg::APPLY_RESTRICT, nullptr, t.J, t.nc, t.apply_epb};
  const int k = trace_begin<T>(c, SIPG_KERNEL_RESTRICT, l);
  run_apply<T>(c, a, "residual_restrict");
  trace_end(c, k);
}

// the FP16 matrix-core local solves: FP32 levels of a precond_bits = 16 context
template <typename T>
const sipg::MfmaTabs *mfma_of(const sipg_ctx *c, const LevelTabs<T> &t) {
  return std::is_same<T, float>::value && c->H.prm.precond_bits == 16 && t.has_mfma ? &t.mfma : nullptr;
}

// C: the corrections' scratch (default: the context's work space)
template <typename T>
void op_schwarz(sipg_ctx *c, int l, const T *r, const T *u_in, T *u_out, T *C = nullptr) {
  const LevelTabs<T> &t = tabs_of<T>(c, l);
  sipg::SchwarzLaunch<T> a{c->mesh, t.n, t.schwarz, r, C ? C : work_of<T>(c).C, t.ilam, u_in, u_out,
                          mfma_of(c, t), t.schwarz_spb, c->wide_planes};
  int k = trace_begin<T>(c, SIPG_KERNEL_SCHWARZ_SOLVE, l);
  check(sipg::launch_schwarz_local<T>(a, c->stream), "schwarz");
  trace_end(c, k);
  k = trace_begin<T>(c, SIPG_KERNEL_SCHWARZ_ASSEMBLE, l);
  check(sipg::launch_schwarz_assemble<T>(a, c->stream), "schwarz");
  trace_end(c, k);
}

// u_l += I_l u_{l-1}; with_mean: u_{l-1} is the level-0 solution whose
// Euclidean mean (from the coarse solve's row sums) is removed on the fly
template <typename T, typename TC>
void op_prolong(sipg_ctx *c, int l, const TC *uc, bool with_mean, T *uf) {
  const LevelTabs<T> &t = tabs_of<T>(c, l);
  const int64_t N0 = level_ndof(c->H, 0);
  sipg::ProlongLaunch<T, TC> a{c->mesh.E, t.n, t.nc, t.J, uc,
                               with_mean ? c->coarse.partial_u : nullptr,
                               sipg::coarse_num_partials(c->coarse), 1.0 / (double)N0, uf};
  const int k = trace_begin<T>(c, SIPG_KERNEL_PROLONG, l);
  if (sipg::apply_is_large(t.n)) {
    check(sipg::launch_prolong_large<T, TC>(a, ensure_big<T>(c), c->stream), "prolong");
  } else {
    check(sipg::launch_prolong<T, TC>(a, c->stream), "prolong");
  }
  trace_end(c, k);
}

template <typename T>
void op_fill_zero(sipg_ctx *c, T *x, int64_t n) {
  // a zero vector through a kernel (no memset nodes in captured graphs)
  check(sipg::launch_fill<T>(x, n, (T)0, c->stream), "fill");
}

// One V-cycle (Algorithm 1).  uL is the top-level iterate (in place); if
// zero_start it is treated as zero.  r_top, if given, is f - A uL already
// computed for the first pre-smoothing step.
template <typename T>
void vcycle_impl(sipg_ctx *c, T *uL, const T *fL, bool zero_start, const T *r_top, T *u_out = nullptr) {
  // u_out (optional): the cycle reads the top-level iterate from uL and
  // writes the new one to u_out, leaving uL untouched
  ensure_work<T>(c);
  Work<T> &w = work_of<T>(c);
  const int L = c->L;
  const sipg::HierarchyHost &H = c->H;
  const int growth = H.prm.smooth_growth;
  auto nsteps = [&](int base, int l) {
    int s = base;
    for (int k = l; k < L; ++k) s *= growth;
    return s;
  };
  T *top = u_out ? u_out : uL;
  if (L == 0) {
    check(sipg::launch_coarse<T>(c->coarse, fL, c->u0, true, c->stream), "coarse");
    check(sipg::launch_convert<T, double>(c->u0, top, level_ndof(H, 0), c->stream), "coarse copy");
    return;
  }
  for (int l = L; l >= 1; --l) {
    T *ul = (l == L) ? top : w.u[l];
    const T *fl = (l == L) ? fL : w.f[l];
    const bool zero = (l < L) || zero_start;
    const int ns = nsteps(H.prm.nsmooth_pre, l);
    if (l == L && u_out && !zero && (ns == 0 || !r_top))
      check(sipg::launch_convert<T, T>(uL, u_out, level_ndof(H, L), c->stream), "copy");
    for (int s = 0; s < ns; ++s) {
      if (zero && s == 0) {
        op_schwarz<T>(c, l, fl, nullptr, ul);
      } else if (s == 0 && l == L && r_top) {
        op_schwarz<T>(c, l, r_top, u_out ? uL : ul, ul);
      } else {
        op_residual<T>(c, l, ul, fl, w.r);
        op_schwarz<T>(c, l, w.r, ul, ul);
      }
    }
    if (ns == 0 && zero) op_fill_zero<T>(c, ul, level_ndof(H, l));
    op_residual_restrict<T>(c, l, ul, fl, w.f[l - 1]);
  }
  check(sipg::launch_coarse<T>(c->coarse, w.f[0], c->u0, false, c->stream), "coarse");
  for (int l = 1; l <= L; ++l) {
    T *ul = (l == L) ? top : w.u[l];
    const T *fl = (l == L) ? fL : w.f[l];
    if (l == 1) op_prolong<T, double>(c, 1, c->u0, true, ul);
    else op_prolong<T, T>(c, l, w.u[l - 1], false, ul);
    const int ns = nsteps(H.prm.nsmooth_post, l);
    for (int s = 0; s < ns; ++s) {
      op_residual<T>(c, l, ul, fl, w.r);
      op_schwarz<T>(c, l, w.r, ul, ul);
    }
  }
}

}  // namespace

namespace {

// z = B r with B one V-cycle from zero in the preconditioner precision.
void precond_body(sipg_ctx *c, const double *r, double *z) {
  const int64_t N = level_ndof(c->H, c->L);
  if (c->H.prm.precond_bits == 64) {
    vcycle_impl<double>(c, z, r, true, nullptr);
    return;
  }
  ensure_work<float>(c);
  Work<float> &w = c->w32;
  check(sipg::launch_convert<float, double>(r, w.fL, N, c->stream), "precond cast");
  vcycle_impl<float>(c, w.uL, w.fL, true, nullptr);
  check(sipg::launch_convert<double, float>(w.uL, z, N, c->stream), "precond cast");
}

void precond_impl(sipg_ctx *c, const double *r, double *z) { precond_body(c, r, z); }

// The preconditioner inside the flexible CG: one V-cycle from zero on the
// context's own vectors.  FP64: from cg_r into cg_z.  FP32: from the single
// precision copy of r (w32.fL, written by the residual update) into w32.uL,
// which the CG kernels read directly, so no conversion passes are needed.
void fcg_precond_body(sipg_ctx *c) {
  if (c->H.prm.precond_bits == 64) vcycle_impl<double>(c, c->cg_z, c->cg_r, true, nullptr);
  else vcycle_impl<float>(c, c->w32.uL, c->w32.fL, true, nullptr);
}

// Captured once into a HIP graph (kernel nodes only) and replayed when the
// context asks for it.
void fcg_precond(sipg_ctx *c) {
  const bool graphable = c->use_graph && !c->graph_failed && c->stream != nullptr;
  if (!graphable) {
    fcg_precond_body(c);
    return;
  }
  if (!c->precond_graph) {
    // every work buffer of the preconditioner exists before the capture (no
    // allocation inside it)
    if (c->H.prm.precond_bits == 64) ensure_work<double>(c);
    else ensure_work<float>(c);
    check(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed), "graph capture");
    hipGraph_t g = nullptr;
    c->capturing = true;
    try {
      fcg_precond_body(c);
    } catch (...) {
      c->capturing = false;
      (void)hipStreamEndCapture(c->stream, &g);
      if (g) (void)hipGraphDestroy(g);
      c->graph_failed = true;
      throw;
    }
    c->capturing = false;
    check(hipStreamEndCapture(c->stream, &g), "graph capture");
    hipError_t e = hipGraphInstantiate(&c->precond_graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->precond_graph = nullptr;
      c->graph_failed = true;
      fcg_precond_body(c);
      return;
    }
  }
  check(hipGraphLaunch(c->precond_graph, c->stream), "graph launch");
}


// ||x||^2 into scal[slot]
void norm2(sipg_ctx *c, const double *x, int64_t n, int slot) {
  check(sipg::launch_dot_partials<double, double>(x, x, n, c->partial, c->stream), "dot");
  check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0, c->scal + slot, c->stream), "dot");
}

void dot(sipg_ctx *c, const double *x, const double *y, int64_t n, int slot) {
  check(sipg::launch_dot_partials<double, double>(x, y, n, c->partial, c->stream), "dot");
  check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0, c->scal + slot, c->stream), "dot");
}

// The periodic problem is singular with null space the constants (Sec. 3.2):
// the solvers work on f projected onto the range 1^perp, cg_b = f - mean(f)
// (the mean in scal[FS_MEAN]), and return the solution of zero Euclidean mean
// (the minimum-norm one, as the coarse pseudo-inverse of Algorithm 1).
void project_rhs(sipg_ctx *c, const double *f) {
  const int64_t N = level_ndof(c->H, c->L);
  check(sipg::launch_sum_partials<double>(f, N, c->partial, c->stream), "rhs mean");
  check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0 / (double)N, c->scal + sipg::FS_MEAN, c->stream),
        "rhs mean");
  check(sipg::launch_sub_scalar_copy<double>(f, c->cg_b, N, c->scal + sipg::FS_MEAN, c->stream), "rhs mean");
}

// x -= mean(x) (the mean in scal[FS_XMEAN])
void remove_mean(sipg_ctx *c, double *x) {
  const int64_t N = level_ndof(c->H, c->L);
  check(sipg::launch_sum_partials<double>(x, N, c->partial, c->stream), "solution mean");
  check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0 / (double)N, c->scal + sipg::FS_XMEAN, c->stream),
        "solution mean");
  check(sipg::launch_sub_scalar<double>(x, N, c->scal + sipg::FS_XMEAN, c->stream), "solution mean");
}

// MG solve.  When the convergence rate observed so far predicts that the
// current iterate cannot have converged yet, the next V-cycle is enqueued
// before the host reads the residual norm, so the device does not wait for the
// host; x is backed up first and restored if the prediction was wrong (the
// result is the same as checking first).
int mg_solve_impl(sipg_ctx *c, double *u, const double *f, double rtol, int maxcyc, int *ncyc,
                  double *relres) {
  const int64_t N = level_ndof(c->H, c->L);
  ensure_work<double>(c);
  project_rhs(c, f);
  f = c->cg_b;
  // two iterate buffers: the caller's u and a work vector free during FP64
  // V-cycles; a speculative cycle writes the new iterate into the other one
  double *cur = u, *alt = c->w64.uL;
  c->hist.clear();
  double r0 = -1.0;
  hipEvent_t ev = nullptr;
  check(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event");
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() { (void)hipEventDestroy(e); }
  } guard{ev};
  bool spec = false;
  for (int cyc = 0;; ++cyc) {
    residual_norm2(c, cur, f, c->cg_r, sipg::FS_RR, true);
    check(hipEventRecord(ev, c->stream), "event");
    spec = spec && cyc < maxcyc;
    if (spec) vcycle_impl<double>(c, cur, f, false, c->cg_r, alt);
    check(hipEventSynchronize(ev), "residual norm");
    const double rn = std::sqrt(c->host_scal[sipg::FS_RR]);
    c->hist.push_back(rn);
    if (r0 < 0) r0 = rn, c->f_mean = c->host_scal[sipg::FS_MEAN];
    if (ncyc) *ncyc = cyc;
    if (relres) *relres = r0 > 0 ? rn / r0 : 0.0;
    if (!std::isfinite(rn) || rn <= rtol * r0 || cyc >= maxcyc) {
      // the checked iterate is cur; a speculative cycle's result is dropped
      if (cur != u) check(sipg::launch_convert<double, double>(cur, u, N, c->stream), "result copy");
      if (std::isfinite(rn)) remove_mean(c, u);
      check(hipStreamSynchronize(c->stream), "mg_solve");
      if (!std::isfinite(rn)) return fail(SIPG_ENOTFINITE, "residual norm is not finite");
      if (rn <= rtol * r0) return SIPG_OK;
      return fail(SIPG_ENOCONV, "mg_solve: tolerance not reached");
    }
    if (spec) std::swap(cur, alt);
    else vcycle_impl<double>(c, cur, f, false, c->cg_r);
    // speculate on the next check if the observed rate says it cannot pass
    const size_t h = c->hist.size();
    spec = h >= 2 && c->hist[h - 2] > 0 && rn * (rn / c->hist[h - 2]) > 10.0 * rtol * r0;
  }
}

int pcg_solve_impl(sipg_ctx *c, double *x, const double *b, double rtol, int maxit, int *iters,
                   double *relres) {
  c->hist.clear();
  if (iters) *iters = 0;
  sipg::detail::fcg_start(c, x, b);
  check(hipStreamSynchronize(c->stream), "fcg");
  const double r0 = std::sqrt(c->host_scal[sipg::FS_RR]);
  c->f_mean = c->host_scal[sipg::FS_MEAN];
  c->hist.push_back(r0);
  if (!std::isfinite(r0)) return fail(SIPG_ENOTFINITE, "initial residual is not finite");
  if (relres) *relres = 0.0;
  if (r0 == 0.0) {
    remove_mean(c, x);
    check(hipStreamSynchronize(c->stream), "fcg");
    return SIPG_OK;
  }
  sipg::detail::fcg_first_precond(c);
  for (int it = 1; it <= maxit; ++it) {
    sipg::detail::fcg_apply_update(c);
    check(hipStreamSynchronize(c->stream), "fcg");
    const double pq = c->host_scal[sipg::FS_PQ];
    double rn = std::sqrt(c->host_scal[sipg::FS_RR]);
    if (iters) *iters = it;
    if (!(pq > 0.0) || !std::isfinite(pq)) {
      if (relres) *relres = c->hist.back() / r0;
      return fail(SIPG_EBREAKDOWN, "flexible CG breakdown (p.Ap <= 0 or not finite)");
    }
    if (!std::isfinite(rn)) return fail(SIPG_ENOTFINITE, "residual norm is not finite");
    if (rn <= rtol * r0) {
      sipg::detail::fcg_confirm(c, x);
      check(hipStreamSynchronize(c->stream), "fcg");
      const double rt = std::sqrt(c->host_scal[sipg::FS_RR]);
      if (rt <= rtol * r0) {
        c->hist.push_back(rt);
        if (relres) *relres = rt / r0;
        return SIPG_OK;
      }
      sipg::detail::fcg_restart_from_true(c);
      rn = rt;
    }
    c->hist.push_back(rn);
    if (relres) *relres = rn / r0;
    sipg::detail::fcg_precond_update(c, x);
  }
  return fail(SIPG_ENOCONV, "pcg_solve: tolerance not reached");
}

int resolve_level(const sipg_ctx *c, int level) {
  if (level == -1) return c->L;
  if (level < 0 || level > c->L) return -2;
  return level;
}

template <typename F>
int guarded(F &&fn) {
  try {
    return fn();
  } catch (const HipFailure &e) {
    return fail(SIPG_EHIP, e.what());
  } catch (const std::bad_alloc &) {
    return fail(SIPG_ENOMEM, "device or host allocation failed");
  } catch (const std::invalid_argument &e) {
    return fail(SIPG_EINVAL, e.what());
  } catch (const std::exception &e) {
    return fail(SIPG_EINVAL, e.what());
  }
}

// ---- cohort V-cycles (serving): several contexts of one preconditioner
// signature run their V-cycles level by level on one stream, the local
// solves and assemblies of all of them in one launch each ----------------

// every context's work on stream st while in scope
struct StreamSwap {
  sipg_ctx *const *cs;
  int k;
  hipStream_t saved[sipg::kMaxApplySegments];
  StreamSwap(sipg_ctx *const *cs_, int k_, hipStream_t st) : cs(cs_), k(k_) {
    for (int i = 0; i < k; ++i) {
      saved[i] = cs[i]->stream;
      cs[i]->stream = st;
    }
  }
  ~StreamSwap() {
    for (int i = 0; i < k; ++i) cs[i]->stream = saved[i];
  }
};

template <typename T>
bool level_segmentable(const sipg_ctx *c, int l, std::vector<int> &sig) {
  const LevelTabs<T> &t = tabs_of<T>(const_cast<sipg_ctx *>(c), l);
  sipg::SchwarzLaunch<T> a{c->mesh, t.n, t.schwarz, nullptr, nullptr, t.ilam, nullptr, nullptr,
                           mfma_of(c, t), t.schwarz_spb, c->wide_planes};
  if (!sipg::schwarz_segments_supported<T>(a)) return false;
  sig.insert(sig.end(), {t.n, t.schwarz.m[0], t.schwarz.m[1], t.schwarz.m[2]});
  return true;
}

// the weighted Schwarz correction of level l of every context in one launch
// of the local solves and one of the assembly: u_out[i] = u_in[i] + sum_s ...
template <typename T>
void schwarz_cohort(sipg_ctx *const *cs, int k, int l, const T *const *r, const T *const *u_in, T *const *u_out) {
  sipg::SchwarzLaunch<T> a[sipg::kMaxApplySegments];
  const int spb = tabs_of<T>(cs[0], l).schwarz_spb;
  for (int i = 0; i < k; ++i) {
    const LevelTabs<T> &t = tabs_of<T>(cs[i], l);
    a[i] = sipg::SchwarzLaunch<T>{cs[i]->mesh, t.n, t.schwarz, r[i], work_of<T>(cs[i]).C, t.ilam, u_in[i],
                                  u_out[i], mfma_of(cs[i], t), spb, cs[i]->wide_planes};
  }
  check(sipg::launch_schwarz_segments<T>(a, k, cs[0]->stream), "schwarz cohort");
}

// one operator-kernel step (residual or residual + restriction) of every
// context: one segmented launch, or one launch per context where their
// launch shapes differ
template <typename T>
void apply_cohort(sipg_ctx *const *cs, int k, const sipg::ApplyLaunch<T> *a, const char *what) {
  const hipError_t e = sipg::launch_apply_segments<T>(a, k, cs[0]->stream);
  if (e == hipSuccess) return;
  if (e != hipErrorInvalidValue) check(e, what);
  (void)hipGetLastError();
  for (int i = 0; i < k; ++i) run_apply<T>(cs[i], a[i], what);
}

template <typename T>
void residual_cohort(sipg_ctx *const *cs, int k, int l, T *const *u, const T *const *f, T *const *r) {
  sipg::ApplyLaunch<T> a[sipg::kMaxApplySegments];
  for (int i = 0; i < k; ++i) {
    const LevelTabs<T> &t = tabs_of<T>(cs[i], l);
    a[i] = sipg::ApplyLaunch<T>{cs[i]->mesh, t.n, t.apply, u[i], f[i], r[i], sipg::APPLY_RESID, nullptr, nullptr, 0,
                                t.apply_epb};
  }
  apply_cohort<T>(cs, k, a, "residual cohort");
}

template <typename T>
void restrict_cohort(sipg_ctx *const *cs, int k, int l, T *const *u, const T *const *f, T *const *fc) {
  sipg::ApplyLaunch<T> a[sipg::kMaxApplySegments];
  for (int i = 0; i < k; ++i) {
    const LevelTabs<T> &t = tabs_of<T>(cs[i], l);
    a[i] = sipg::ApplyLaunch<T>{cs[i]->mesh, t.n, t.apply, u[i], f[i], fc[i], sipg::APPLY_RESTRICT, nullptr, t.J, t.nc,
                                t.apply_epb};
  }
  apply_cohort<T>(cs, k, a, "restrict cohort");
}

// u_l += I_l u_{l-1} for every context (level 1: from the level-0 solution
// with its mean removed, as op_prolong)
template <typename T, typename TC>
void prolong_cohort(sipg_ctx *const *cs, int k, int l, const TC *const *uc, T *const *uf) {
  sipg::ProlongLaunch<T, TC> a[sipg::kMaxApplySegments];
  for (int i = 0; i < k; ++i) {
    const LevelTabs<T> &t = tabs_of<T>(cs[i], l);
    const int64_t N0 = level_ndof(cs[i]->H, 0);
    a[i] = sipg::ProlongLaunch<T, TC>{cs[i]->mesh.E, t.n, t.nc, t.J, uc[i],
                                      l == 1 ? cs[i]->coarse.partial_u : nullptr,
                                      sipg::coarse_num_partials(cs[i]->coarse), 1.0 / (double)N0, uf[i]};
  }
  check(sipg::launch_prolong_segments<T, TC>(a, k, cs[0]->stream), "prolong cohort");
}

// vcycle_impl from a zero start for every context, in the same order of
// steps, each step of all contexts in one launch (the coarse solves per
// context)
template <typename T>
void vcycle_cohort(sipg_ctx *const *cs, int k, T *const *uL, const T *const *fL) {
  constexpr int KM = sipg::kMaxApplySegments;
  const sipg::HierarchyHost &H = cs[0]->H;
  const int L = cs[0]->L;
  auto nsteps = [&](int base, int l) {
    int s = base;
    for (int q = l; q < L; ++q) s *= H.prm.smooth_growth;
    return s;
  };
  T *ul[KM], *rr[KM], *fc[KM], *uc[KM];
  const T *fl[KM], *none[KM] = {};
  const double *u0[KM];
  auto level_vectors = [&](int l) {
    for (int i = 0; i < k; ++i) {
      Work<T> &w = work_of<T>(cs[i]);
      ul[i] = (l == L) ? uL[i] : w.u[l];
      fl[i] = (l == L) ? fL[i] : w.f[l];
      rr[i] = w.r;
      fc[i] = w.f[l - 1];
      uc[i] = w.u[l - 1];
      u0[i] = cs[i]->u0;
    }
  };
  auto smooth_from_residual = [&](int l) {
    residual_cohort<T>(cs, k, l, ul, fl, rr);
    schwarz_cohort<T>(cs, k, l, rr, ul, ul);
  };
  for (int l = L; l >= 1; --l) {
    level_vectors(l);
    const int ns = nsteps(H.prm.nsmooth_pre, l);
    for (int s = 0; s < ns; ++s) {
      if (s == 0) schwarz_cohort<T>(cs, k, l, fl, none, ul);
      else smooth_from_residual(l);
    }
    if (ns == 0)
      for (int i = 0; i < k; ++i) op_fill_zero<T>(cs[i], ul[i], level_ndof(cs[i]->H, l));
    restrict_cohort<T>(cs, k, l, ul, fl, fc);
  }
  for (int i = 0; i < k; ++i)
    check(sipg::launch_coarse<T>(cs[i]->coarse, work_of<T>(cs[i]).f[0], cs[i]->u0, false, cs[i]->stream), "coarse");
  for (int l = 1; l <= L; ++l) {
    level_vectors(l);
    if (l == 1) prolong_cohort<T, double>(cs, k, 1, u0, ul);
    else prolong_cohort<T, T>(cs, k, l, uc, ul);
    const int ns = nsteps(H.prm.nsmooth_post, l);
    for (int s = 0; s < ns; ++s) smooth_from_residual(l);
  }
}

// the cohort's preconditioner V-cycles z = B r (the FP64 or FP32 vectors of
// fcg_precond), every context's work on stream st
void precond_cohort(sipg_ctx *const *cs, int k, hipStream_t st) {
  StreamSwap swap(cs, k, st);
  constexpr int KM = sipg::kMaxApplySegments;
  if (cs[0]->H.prm.precond_bits == 64) {
    double *u[KM];
    const double *f[KM];
    for (int i = 0; i < k; ++i) u[i] = cs[i]->cg_z, f[i] = cs[i]->cg_r;
    vcycle_cohort<double>(cs, k, u, f);
  } else {
    float *u[KM];
    const float *f[KM];
    for (int i = 0; i < k; ++i) u[i] = cs[i]->w32.uL, f[i] = cs[i]->w32.fL;
    vcycle_cohort<float>(cs, k, u, f);
  }
}

}  // namespace

// ---- flexible CG in enqueue-only pieces (shared by sipg_pcg_solve and the
// serving loop, so both run the same kernel sequence) ----------------------
namespace sipg {
namespace detail {

// With a single-precision preconditioner the search direction p is kept in
// single precision (in the first half of the cg_p buffer): p = z + beta p is
// formed in double and rounded once, and x += alpha p, q = A p (in double)
// use that same rounded p, so x and r stay consistent and only the
// direction, not the accuracy of the iterate, carries the rounding (flexible
// CG tolerates a perturbed direction).  Orders whose operator takes the
// large-element path keep p in double.
bool p_single(const sipg_ctx *c) {
  return c->H.prm.precond_bits != 64 && !sipg::apply_is_large(c->t64[c->L].n);
}
float *p32_of(sipg_ctx *c) { return reinterpret_cast<float *>(c->cg_p); }

// q = A p (with per-block partials of p.q when partial is given)
void fcg_apply_p(sipg_ctx *c, double *partial) {
  if (p_single(c)) {
    const LevelTabs<double> &t = c->t64[c->L];
    sipg::ApplyLaunch<double> a{c->mesh, t.n, t.apply, nullptr, nullptr, c->cg_q, sipg::APPLY_PLAIN, partial,
                                nullptr, 0, t.apply_epb, p32_of(c)};
    check(sipg::launch_apply<double>(a, c->stream), "apply_A");
  } else {
    op_apply<double>(c, c->L, c->cg_p, c->cg_q, partial);
  }
}

void fcg_start(sipg_ctx *c, double *x, const double *b) {
  project_rhs(c, b);
  residual_norm2(c, x, c->cg_b, c->cg_r, sipg::FS_RR, true);
}

void fcg_first_precond(sipg_ctx *c) {
  const int64_t N = level_ndof(c->H, c->L);
  const bool single = c->H.prm.precond_bits != 64;
  if (single) {
    ensure_work<float>(c);
    check(sipg::launch_convert<float, double>(c->cg_r, c->w32.fL, N, c->stream), "precond cast");
  }
  fcg_precond(c);
  if (single) {
    check(sipg::launch_dot_partials<double, float>(c->cg_r, c->w32.uL, N, c->partial, c->stream), "dot");
    if (p_single(c)) check(sipg::launch_convert<float, float>(c->w32.uL, p32_of(c), N, c->stream), "copy");
    else check(sipg::launch_convert<double, float>(c->w32.uL, c->cg_p, N, c->stream), "copy");
  } else {
    check(sipg::launch_dot_partials<double, double>(c->cg_r, c->cg_z, N, c->partial, c->stream), "dot");
    check(sipg::launch_convert<double, double>(c->cg_z, c->cg_p, N, c->stream), "copy");
  }
  check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0, c->scal + sipg::FS_RZ, c->stream), "dot");
  c->x_pending = false;
}

void fcg_after_apply(sipg_ctx *c, hipStream_t st) {
  const int64_t N = level_ndof(c->H, c->L);
  check(sipg::launch_finalize(c->partial,
                              sipg::apply_num_blocks(c->mesh.E, c->t64[c->L].n, c->t64[c->L].apply_epb), 1.0,
                              c->scal + sipg::FS_PQ, st),
        "dot");
  float *r32 = c->H.prm.precond_bits != 64 ? c->w32.fL : nullptr;
  check(sipg::launch_fcg_r(c->cg_r, c->cg_q, N, c->scal, c->partial, r32, st), "fcg update");
  check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0, c->scal + sipg::FS_RR, st, c->scal,
                              c->host_scal_dev, sipg::FS_COUNT),
        "dot");
  c->x_pending = true;
}

void fcg_after_apply_batched(sipg_ctx *const *cs, int k, hipStream_t st) {
  sipg::FinalizeSegs pq{}, rr{};
  sipg::FcgRSegs up{};
  pq.n = rr.n = up.n = k;
  for (int i = 0; i < k; ++i) {
    sipg_ctx *c = cs[i];
    pq.s[i] = sipg::FinalizeSeg{c->partial,
                                sipg::apply_num_blocks(c->mesh.E, c->t64[c->L].n, c->t64[c->L].apply_epb),
                                c->scal + sipg::FS_PQ, nullptr, nullptr, 0};
    up.s[i] = sipg::FcgRSeg{c->cg_r, c->cg_q, level_ndof(c->H, c->L), c->scal, c->partial,
                            c->H.prm.precond_bits != 64 ? c->w32.fL : nullptr};
    rr.s[i] = sipg::FinalizeSeg{c->partial, sipg::kDotBlocks, c->scal + sipg::FS_RR, c->scal, c->host_scal_dev,
                                sipg::FS_COUNT};
  }
  check(sipg::launch_finalize_segments(pq, st), "dot");
  check(sipg::launch_fcg_r_segments(up, st), "fcg update");
  check(sipg::launch_finalize_segments(rr, st), "dot");
  for (int i = 0; i < k; ++i) cs[i]->x_pending = true;
}

bool fcg_apply_launch(sipg_ctx *c, sipg::ApplyLaunch<double> *a) {
  const LevelTabs<double> &t = c->t64[c->L];
  if (sipg::apply_is_large(t.n)) return false;
  const bool ps = p_single(c);
  *a = sipg::ApplyLaunch<double>{c->mesh, t.n, t.apply, ps ? nullptr : c->cg_p, nullptr, c->cg_q,
                                 sipg::APPLY_PLAIN, c->partial, nullptr, 0,
                                 sipg::apply_launch_epb(c->mesh.E, t.n, t.apply_epb), ps ? p32_of(c) : nullptr};
  return true;
}

void fcg_apply_update(sipg_ctx *c) {
  fcg_apply_p(c, c->partial);
  fcg_after_apply(c, c->stream);
}

void fcg_confirm(sipg_ctx *c, double *x) {
  const int64_t N = level_ndof(c->H, c->L);
  if (c->x_pending) {
    if (p_single(c)) check(sipg::launch_fcg_x<float>(x, p32_of(c), N, c->scal, c->stream), "fcg update");
    else check(sipg::launch_fcg_x<double>(x, c->cg_p, N, c->scal, c->stream), "fcg update");
  }
  c->x_pending = false;
  // the returned iterate has zero mean (A 1 = 0: the residual is unchanged)
  remove_mean(c, x);
  residual_norm2(c, x, c->cg_b, c->cg_q, sipg::FS_RR, true);
}

void fcg_restart_from_true(sipg_ctx *c) {
  const int64_t N = level_ndof(c->H, c->L);
  check(sipg::launch_convert<double, double>(c->cg_q, c->cg_r, N, c->stream), "copy");
  if (c->H.prm.precond_bits != 64)
    check(sipg::launch_convert<float, double>(c->cg_r, c->w32.fL, N, c->stream), "precond cast");
  fcg_apply_p(c, nullptr);
}

// after z = B r: beta, rz, x += alpha p if pending, p = z + beta p
void fcg_after_precond(sipg_ctx *c, double *x) {
  const int64_t N = level_ndof(c->H, c->L);
  if (c->H.prm.precond_bits != 64) {
    check(sipg::launch_fcg_dot2<float>(c->w32.uL, c->cg_q, c->cg_r, N, c->partial, c->stream), "dot2");
    check(sipg::launch_fcg_finalize2(c->partial, c->scal, c->stream), "dot2");
    if (p_single(c))
      check(sipg::launch_fcg_xp<float, float>(x, p32_of(c), c->w32.uL, N, c->scal, c->x_pending, c->stream),
            "fcg update");
    else
      check(sipg::launch_fcg_xp<float, double>(x, c->cg_p, c->w32.uL, N, c->scal, c->x_pending, c->stream),
            "fcg update");
  } else {
    check(sipg::launch_fcg_dot2<double>(c->cg_z, c->cg_q, c->cg_r, N, c->partial, c->stream), "dot2");
    check(sipg::launch_fcg_finalize2(c->partial, c->scal, c->stream), "dot2");
    check(sipg::launch_fcg_xp<double, double>(x, c->cg_p, c->cg_z, N, c->scal, c->x_pending, c->stream),
          "fcg update");
  }
  c->x_pending = false;
}

void fcg_precond_update(sipg_ctx *c, double *x) {
  fcg_precond(c);
  fcg_after_precond(c, x);
}

std::vector<int> precond_signature(const sipg_ctx *c) {
  const sipg_params &p = c->H.prm;
  if (c->L < 1) return {};
  std::vector<int> sig{p.precond_bits, c->L, p.nsmooth_pre, p.nsmooth_post, p.smooth_growth};
  for (int l = 1; l <= c->L; ++l) {
    const bool ok = p.precond_bits == 64 ? level_segmentable<double>(c, l, sig) : level_segmentable<float>(c, l, sig);
    if (!ok) return {};
  }
  return sig;
}

// k in range, equal non-empty signatures, work vectors allocated (a capture
// must not allocate)
void check_cohort(sipg_ctx *const *cs, int k) {
  if (k < 1 || k > sipg::kMaxApplySegments) throw std::invalid_argument("cohort size out of range");
  const std::vector<int> sig = precond_signature(cs[0]);
  if (sig.empty()) throw std::invalid_argument("context cannot join a cohort");
  for (int i = 1; i < k; ++i)
    if (precond_signature(cs[i]) != sig) throw std::invalid_argument("cohort signatures differ");
  for (int i = 0; i < k; ++i) {
    if (cs[i]->H.prm.precond_bits == 64) ensure_work<double>(cs[i]);
    else ensure_work<float>(cs[i]);
  }
}

void fcg_precond_update_cohort(sipg_ctx *const *cs, double *const *xs, int k, hipStream_t st,
                               hipGraphExec_t graph) {
  check_cohort(cs, k);
  if (graph) {
    check(hipGraphLaunch(graph, st), "cohort graph launch");
  } else {
    precond_cohort(cs, k, st);
  }
  StreamSwap swap(cs, k, st);
  for (int i = 0; i < k; ++i) fcg_after_precond(cs[i], xs[i]);
}

hipGraphExec_t capture_cohort_precond(sipg_ctx *const *cs, int k, hipStream_t st) {
  check_cohort(cs, k);
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
  try {
    precond_cohort(cs, k, st);
  } catch (...) {
    (void)hipStreamEndCapture(st, &g);
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipStreamEndCapture(st, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return ex;
}

const double *host_scalars(const sipg_ctx *c) { return c->host_scal; }
hipStream_t ctx_stream(const sipg_ctx *c) { return c->stream; }
void enable_graph(sipg_ctx *c, bool on) { c->use_graph = on; }
int64_t ctx_ndof(const sipg_ctx *c) { return level_ndof(c->H, c->L); }
size_t ctx_bytes(const sipg_ctx *c) { return c->bytes; }
std::string last_error() { return g_err; }
void set_error(const std::string &m) { g_err = m; }

}  // namespace detail
}  // namespace sipg

// ---- autotuner ------------------------------------------------------------
namespace {

// process-wide choices by (precision bits, level order n, m_x, m_y, m_z,
// elements, matrix-core local solves): {elements per workgroup of the
// operator kernel, subdomains per workgroup of the local-solve kernel}
std::mutex g_tune_mu;
std::map<std::array<int, 7>, std::array<int, 2>> g_tuned;

// mean duration (ms) of one of `reps` launches after one untimed launch
template <typename F>
double time_launches(sipg_ctx *c, int reps, F &&launch) {
  launch();
  hipEvent_t e0, e1;
  check(hipEventCreate(&e0), "event");
  check(hipEventCreate(&e1), "event");
  check(hipEventRecord(e0, c->stream), "event");
  for (int i = 0; i < reps; ++i) launch();
  check(hipEventRecord(e1, c->stream), "event");
  check(hipEventSynchronize(e1), "event");
  float el = 0.f;
  check(hipEventElapsedTime(&el, e0, e1), "event");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)el / reps;
}

template <typename T>
void tune_level(sipg_ctx *c, int l, int reps) {
  LevelTabs<T> &t = tabs_of<T>(c, l);
  const sipg::MfmaTabs *mf = mfma_of(c, t);
  const std::array<int, 7> key{(int)(8 * sizeof(T)), t.n, t.schwarz.m[0], t.schwarz.m[1], t.schwarz.m[2],
                               c->mesh.E, mf != nullptr};
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      t.apply_epb = it->second[0];
      t.schwarz_spb = it->second[1];
      return;
    }
  }
  const int64_t N = level_ndof(c->H, l);
  T *u, *f, *r;
  // a context with a single-precision preconditioner runs FP64 kernels only
  // in the outer flexible CG (the top-level operator): time that one on the
  // CG vectors, without the FP64 work space its footprint does not hold
  const bool outer_only = std::is_same<T, double>::value && c->H.prm.precond_bits != 64;
  if (outer_only) {
    if (l != c->L) return;
    u = reinterpret_cast<T *>(c->cg_p), f = reinterpret_cast<T *>(c->cg_b), r = reinterpret_cast<T *>(c->cg_q);
  } else {
    ensure_work<T>(c);
    Work<T> &w = work_of<T>(c);
    u = w.uL, f = w.fL, r = w.r;
  }
  check(sipg::launch_fill<T>(u, N, (T)0.25, c->stream), "fill");
  check(sipg::launch_fill<T>(f, N, (T)0.5, c->stream), "fill");
  check(sipg::launch_fill<T>(r, N, (T)0.75, c->stream), "fill");
  // operator: powers of two up to the full packing, and the full packing
  const int full = sipg::apply_max_epb(t.n);
  if (full > 1) {
    std::vector<int> cand;
    for (int e = 1; e < full; e *= 2) cand.push_back(e);
    cand.push_back(full);
    double best = 1e30;
    int pick = 0;
    for (int e : cand) {
      t.apply_epb = e;
      const double ms = time_launches(c, reps, [&] { op_residual<T>(c, l, u, f, r); });
      if (ms < best) best = ms, pick = e;
    }
    t.apply_epb = pick;
  }
  // compile-time-shape local solves: 1 .. the most subdomains that fit
  const int maxspb = mf || outer_only ? 0 : sipg::schwarz_fixed_max_spb(t.n, t.schwarz.m);
  if (maxspb > 1) {
    Work<T> &w = work_of<T>(c);
    double best = 1e30;
    int pick = 0;
    for (int sp = 1; sp <= maxspb; ++sp) {
      t.schwarz_spb = sp;
      sipg::SchwarzLaunch<T> sa{c->mesh, t.n, t.schwarz, r, w.C, t.ilam, u, u, mf, sp};
      const double ms = time_launches(c, reps, [&] { check(sipg::launch_schwarz_local<T>(sa, c->stream), "schwarz"); });
      if (ms < best) best = ms, pick = sp;
    }
    t.schwarz_spb = pick;
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tuned[key] = {t.apply_epb, t.schwarz_spb};
}

template <typename T>
bool take_cached(sipg_ctx *c, int l) {
  LevelTabs<T> &t = tabs_of<T>(c, l);
  const std::array<int, 7> key{(int)(8 * sizeof(T)), t.n, t.schwarz.m[0], t.schwarz.m[1], t.schwarz.m[2],
                               c->mesh.E, mfma_of(c, t) != nullptr};
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tuned.find(key);
  if (it == g_tuned.end()) return false;
  t.apply_epb = it->second[0];
  t.schwarz_spb = it->second[1];
  return true;
}

// value of `"key": <int>` in a JSON object's text
bool json_int(const std::string &obj, const char *key, long *out) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = obj.find(k);
  if (p == std::string::npos) return false;
  p = obj.find(':', p + k.size());
  if (p == std::string::npos) return false;
  char *end = nullptr;
  const long v = std::strtol(obj.c_str() + p + 1, &end, 10);
  if (end == obj.c_str() + p + 1) return false;
  *out = v;
  return true;
}

}  // namespace

namespace sipg {
namespace detail {

int apply_cached_tuning(sipg_ctx *c) {
  int took = 0;
  for (int l = 1; l <= c->L; ++l) {
    took += take_cached<double>(c, l);
    if (c->H.prm.precond_bits != 64) took += take_cached<float>(c, l);
  }
  return took;
}

}  // namespace detail
}  // namespace sipg

namespace {

// Device bytes sipg_setup allocates for hierarchy H: the table arena, the
// level-0 and flexible-CG vectors, the scalars and partial sums, the
// preconditioner's work space and the FP64 large-element scratch (every
// buffer sipg_pcg_solve and sipg_precond use; FP64 entry points on a context
// with precond_bits 32 or 16 add the FP64 work space on first use).
size_t context_bytes(const sipg::HierarchyHost &H) {
  auto al = [](size_t count, size_t eb) { return std::max<size_t>(count, 1) * eb; };
  const int L = (int)H.lev.size() - 1;
  const int64_t E = (int64_t)H.prm.ne[0] * H.prm.ne[1] * H.prm.ne[2];
  const int64_t N0 = level_ndof(H, 0), N = level_ndof(H, L);
  sipg::CoarseLaunch cl{};
  for (int d = 0; d < 3; ++d) cl.ne[d] = H.prm.ne[d], cl.N[d] = H.coarse.N[d];
  const size_t np = (size_t)sipg::coarse_num_partials(cl);
  size_t b = al(build_table_arena(H, E).A.host.size(), 1);
  b += 2 * al(N0, 8) + 2 * al(np, 8) + al(4, 8);                     // u0, coarse work, plane sums
  b += 5 * al(N, 8);                                                 // r, p, q, z, projected b
  b += al(sipg::FS_COUNT, 8);
  b += al(std::max<size_t>(2 * sipg::kDotBlocks, sipg::apply_num_blocks((int)E, H.lev[L].n, 1)), 8);
  b += al(64 * 3, 4) + al(64 * 3, 8) + al(64, 8);                    // Fourier modes
  const size_t eb = H.prm.precond_bits == 64 ? 8 : 4;
  if (L > 0) {
    b += work_bytes(H, eb) + (big_count(H) ? big_count(H) * eb : 0);
    if (eb != 8 && big_count(H)) b += big_count(H) * 8;
  } else {
    b += work_bytes(H, eb);
  }
  return b;
}

}  // namespace

namespace {

// level index (1..L) of `level` (-1 = top), or 0 if invalid
int level_arg(const sipg_ctx *c, int level) {
  const int l = level == -1 ? c->L : level;
  return (l >= 1 && l <= c->L) ? l : 0;
}

template <typename T>
void tuning_limits_of(const sipg_ctx *c, const LevelTabs<T> &t, int *max_epb, int *max_spb) {
  *max_epb = sipg::apply_max_epb(t.n);
  *max_spb = mfma_of(c, t) ? 0 : sipg::schwarz_fixed_max_spb(t.n, t.schwarz.m);
}

}  // namespace

extern "C" {

void sipg_default_params(sipg_params *p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->ne[0] = p->ne[1] = p->ne[2] = 4;
  p->len[0] = p->len[1] = p->len[2] = 1.0;
  p->P = 4;
  p->penalty = 1.0;
  p->overlap_mode = SIPG_OVL_MIN;
  p->overlap = 0.08;
  p->nsmooth_pre = 1;
  p->nsmooth_post = 1;
  p->smooth_growth = 1;
  p->precond_bits = 64;
  p->basis = SIPG_BASIS_GLL;
  p->overlap_floor = 0;
}

const char *sipg_last_error(void) { return g_err.c_str(); }

int sipg_footprint(const sipg_params *p, size_t *bytes) {
  if (!p || !bytes) return fail(SIPG_EINVAL, "null argument");
  return guarded([&]() {
    sipg::HierarchyHost H;
    sipg::build_hierarchy(*p, H);
    *bytes = context_bytes(H);
    return (int)SIPG_OK;
  });
}

int sipg_setup(const sipg_params *p, void *hip_stream, sipg_ctx **out) {
  if (!p || !out) return fail(SIPG_EINVAL, "null argument");
  *out = nullptr;
  std::unique_ptr<sipg_ctx> c(new (std::nothrow) sipg_ctx());
  if (!c) return fail(SIPG_ENOMEM, "host allocation failed");
  int rc = guarded([&]() {
    sipg::build_hierarchy(*p, c->H);
    c->stream = static_cast<hipStream_t>(hip_stream);
    check(hipGetDevice(&c->device), "hipGetDevice");
    // address of the fixed scratch of sipg_schwarz_noalloc on this device
    check(sipg::noalloc_scratch_init(c->device), "scratch address");
    c->L = (int)c->H.lev.size() - 1;
    for (int d = 0; d < 3; ++d) c->mesh.ne[d] = p->ne[d];
    c->mesh.E = p->ne[0] * p->ne[1] * p->ne[2];
    upload_tables(c.get());
    const int64_t N0 = level_ndof(c->H, 0), N = level_ndof(c->H, c->L);
    c->u0 = c->alloc<double>(N0);
    c->coarse.t0 = c->alloc<double>(N0);
    c->coarse.partial = c->alloc<double>(sipg::coarse_num_partials(c->coarse));
    c->coarse.partial_u = c->alloc<double>(sipg::coarse_num_partials(c->coarse));
    c->coarse.scalars = c->alloc<double>(4);
    c->cg_r = c->alloc<double>(N);
    c->cg_p = c->alloc<double>(N);
    c->cg_q = c->alloc<double>(N);
    c->cg_z = c->alloc<double>(N);
    c->cg_b = c->alloc<double>(N);
    c->scal = c->alloc<double>(sipg::FS_COUNT);
    // partial sums: the reductions use 2 * kDotBlocks, the fused p.Ap of the
    // top-level apply one per apply workgroup
    c->partial = c->alloc<double>(
        std::max<size_t>(2 * sipg::kDotBlocks, sipg::apply_num_blocks(c->mesh.E, c->H.lev[c->L].n, 1)));
    c->rhs_k = c->alloc<int>(64 * 3);
    c->rhs_phi = c->alloc<double>(64 * 3);
    c->rhs_amp = c->alloc<double>(64);
    if (hipHostMalloc((void **)&c->host_scal, sipg::FS_COUNT * sizeof(double),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
      throw std::bad_alloc();
    check(hipHostGetDevicePointer((void **)&c->host_scal_dev, c->host_scal, 0), "host mirror");
    check(sipg::launch_fill<double>(c->scal, sipg::FS_COUNT, 0.0, c->stream), "init");
    // the preconditioner's work space, and the FP64 large-element scratch of
    // the outer operator (so that sipg_pcg_solve allocates nothing)
    if (p->precond_bits == 64) ensure_work<double>(c.get());
    else ensure_work<float>(c.get());
    ensure_big<double>(c.get());
    check(hipStreamSynchronize(c->stream), "setup");
    return (int)SIPG_OK;
  });
  if (rc != SIPG_OK) return rc;
  *out = c.release();
  return SIPG_OK;
}

int sipg_destroy(sipg_ctx *c) {
  if (!c) return SIPG_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  delete c;
  return SIPG_OK;
}

int sipg_nlevels(const sipg_ctx *c, int *nlevels) {
  if (!c || !nlevels) return fail(SIPG_EINVAL, "null argument");
  *nlevels = c->L + 1;
  return SIPG_OK;
}

int sipg_level_info(const sipg_ctx *c, int level, int *order, int no[3], int64_t *ndof) {
  if (!c) return fail(SIPG_EINVAL, "null context");
  const int l = resolve_level(c, level);
  if (l < 0) return fail(SIPG_EINVAL, "level out of range");
  if (order) *order = c->H.lev[l].p;
  if (no)
    for (int d = 0; d < 3; ++d) no[d] = c->H.lev[l].dir[d].no;
  if (ndof) *ndof = level_ndof(c->H, l);
  return SIPG_OK;
}

int sipg_ndof(const sipg_ctx *c, int level, int64_t *n) {
  if (!c || !n) return fail(SIPG_EINVAL, "null argument");
  const int l = resolve_level(c, level);
  if (l < 0) return fail(SIPG_EINVAL, "level out of range");
  *n = level_ndof(c->H, l);
  return SIPG_OK;
}

int sipg_rhs_mean(const sipg_ctx *c, double *mean) {
  if (!c || !mean) return fail(SIPG_EINVAL, "null argument");
  *mean = c->f_mean;
  return SIPG_OK;
}

int sipg_device_bytes(const sipg_ctx *c, size_t *bytes) {
  if (!c || !bytes) return fail(SIPG_EINVAL, "null argument");
  *bytes = c->bytes;
  return SIPG_OK;
}

int sipg_rhs_fourier(sipg_ctx *c, int nmodes, const int32_t *k, const double *phi, const double *amp,
                     double *b) {
  if (!c || !k || !phi || !amp || !b) return fail(SIPG_EINVAL, "null argument");
  if (nmodes < 1 || nmodes > 64) return fail(SIPG_EINVAL, "nmodes must be in 1..64");
  for (int i = 0; i < 3 * nmodes; ++i)
    if (!std::isfinite(phi[i])) return fail(SIPG_EINVAL, "non-finite phase");
  for (int i = 0; i < nmodes; ++i)
    if (!std::isfinite(amp[i])) return fail(SIPG_EINVAL, "non-finite amplitude");
  return guarded([&]() {
    const sipg::HierarchyHost &H = c->H;
    check(hipMemcpyAsync(c->rhs_k, k, 3 * nmodes * sizeof(int), hipMemcpyHostToDevice, c->stream), "rhs");
    check(hipMemcpyAsync(c->rhs_phi, phi, 3 * nmodes * sizeof(double), hipMemcpyHostToDevice, c->stream), "rhs");
    check(hipMemcpyAsync(c->rhs_amp, amp, nmodes * sizeof(double), hipMemcpyHostToDevice, c->stream), "rhs");
    sipg::RhsLaunch a{};
    a.mesh = c->mesh;
    a.n = H.lev[c->L].n;
    a.xi = c->xi_top;
    for (int d = 0; d < 3; ++d) {
      a.mass[d] = c->mass_top[d];
      a.h[d] = H.prm.len[d] / H.prm.ne[d];
      a.len[d] = H.prm.len[d];
    }
    a.nmodes = nmodes;
    a.k = c->rhs_k;
    a.phi = c->rhs_phi;
    a.amp = c->rhs_amp;
    check(sipg::launch_rhs(a, b, c->stream), "rhs");
    const int64_t N = level_ndof(H, c->L);
    check(sipg::launch_sum_partials<double>(b, N, c->partial, c->stream), "rhs mean");
    check(sipg::launch_finalize(c->partial, sipg::kDotBlocks, 1.0 / (double)N, c->scal + sipg::FS_MEAN,
                                c->stream),
          "rhs mean");
    check(sipg::launch_sub_scalar<double>(b, N, c->scal + sipg::FS_MEAN, c->stream), "rhs mean");
    // the host-side copies of k/phi/amp must stay valid until the copies ran
    check(hipStreamSynchronize(c->stream), "rhs");
    return (int)SIPG_OK;
  });
}

int sipg_apply_A(sipg_ctx *c, int level, const double *u, double *y) {
  if (!c || !u || !y) return fail(SIPG_EINVAL, "null argument");
  if (u == y) return fail(SIPG_EINVAL, "u and y must not alias");
  const int l = resolve_level(c, level);
  if (l < 0) return fail(SIPG_EINVAL, "level out of range");
  return guarded([&]() {
    op_apply<double>(c, l, u, y, nullptr);
    return (int)SIPG_OK;
  });
}

int sipg_residual(sipg_ctx *c, int level, const double *u, const double *f, double *r) {
  if (!c || !u || !f || !r) return fail(SIPG_EINVAL, "null argument");
  if (u == r) return fail(SIPG_EINVAL, "u and r must not alias");
  const int l = resolve_level(c, level);
  if (l < 0) return fail(SIPG_EINVAL, "level out of range");
  return guarded([&]() {
    op_residual<double>(c, l, u, f, r);
    return (int)SIPG_OK;
  });
}

int sipg_schwarz(sipg_ctx *c, int level, const double *r, double *u) {
  if (!c || !r || !u) return fail(SIPG_EINVAL, "null argument");
  if (r == u) return fail(SIPG_EINVAL, "r and u must not alias");
  const int l = resolve_level(c, level);
  if (l < 1) return fail(SIPG_EINVAL, "Schwarz smoothing needs level >= 1");
  return guarded([&]() {
    ensure_work<double>(c);
    op_schwarz<double>(c, l, r, u, u);
    return (int)SIPG_OK;
  });
}

int sipg_schwarz_noalloc(sipg_ctx *c, int level, const double *r, double *u) {
  if (!c || !r || !u) return fail(SIPG_EINVAL, "null argument");
  if (r == u) return fail(SIPG_EINVAL, "r and u must not alias");
  const int l = resolve_level(c, level);
  if (l < 1) return fail(SIPG_EINVAL, "Schwarz smoothing needs level >= 1");
  const sipg::SchwarzTabs<double> &t = c->t64[l].schwarz;
  const size_t need = (size_t)c->mesh.E * t.m[0] * t.m[1] * t.m[2] * sizeof(double);
  if (need > sipg::kNoallocScratchBytes)
    return fail(SIPG_EINVAL, "sipg_schwarz_noalloc: level " + std::to_string(l) + " needs " + std::to_string(need) +
                                 " bytes of correction scratch, more than its fixed " +
                                 std::to_string(sipg::kNoallocScratchBytes) + " bytes");
  double *C = static_cast<double *>(sipg::noalloc_scratch(c->device));
  if (!C) return fail(SIPG_EHIP, "sipg_schwarz_noalloc: scratch address unknown on this device");
  return guarded([&]() {
    op_schwarz<double>(c, l, r, u, u, C);
    return (int)SIPG_OK;
  });
}

int sipg_smooth(sipg_ctx *c, int level, double *u, const double *f, int nsteps) {
  if (!c || !u || !f) return fail(SIPG_EINVAL, "null argument");
  if (u == f) return fail(SIPG_EINVAL, "u and f must not alias");
  if (nsteps < 0) return fail(SIPG_EINVAL, "nsteps must be >= 0");
  const int l = resolve_level(c, level);
  if (l < 1) return fail(SIPG_EINVAL, "smoothing needs level >= 1");
  return guarded([&]() {
    ensure_work<double>(c);
    for (int s = 0; s < nsteps; ++s) {
      op_residual<double>(c, l, u, f, c->w64.r);
      op_schwarz<double>(c, l, c->w64.r, u, u);
    }
    return (int)SIPG_OK;
  });
}

int sipg_restrict(sipg_ctx *c, int level, const double *r_fine, double *f_coarse) {
  if (!c || !r_fine || !f_coarse) return fail(SIPG_EINVAL, "null argument");
  const int l = resolve_level(c, level);
  if (l < 1) return fail(SIPG_EINVAL, "restriction needs level >= 1");
  return guarded([&]() {
    // J^T r = J^T (r - A 0): the fused residual-restriction kernel with u = 0
    ensure_work<double>(c);
    double *zero = c->w64.uL;
    check(sipg::launch_fill<double>(zero, level_ndof(c->H, l), 0.0, c->stream), "fill");
    op_residual_restrict<double>(c, l, zero, r_fine, f_coarse);
    return (int)SIPG_OK;
  });
}

int sipg_prolong_add(sipg_ctx *c, int level, const double *u_coarse, double *u_fine) {
  if (!c || !u_coarse || !u_fine) return fail(SIPG_EINVAL, "null argument");
  const int l = resolve_level(c, level);
  if (l < 1) return fail(SIPG_EINVAL, "prolongation needs level >= 1");
  return guarded([&]() {
    op_prolong<double, double>(c, l, u_coarse, false, u_fine);
    return (int)SIPG_OK;
  });
}

int sipg_coarse_solve(sipg_ctx *c, const double *f0, double *u0) {
  if (!c || !f0 || !u0) return fail(SIPG_EINVAL, "null argument");
  if (f0 == u0) return fail(SIPG_EINVAL, "f0 and u0 must not alias");
  return guarded([&]() {
    check(sipg::launch_coarse<double>(c->coarse, f0, u0, true, c->stream), "coarse");
    return (int)SIPG_OK;
  });
}

int sipg_vcycle(sipg_ctx *c, double *u, const double *f) {
  if (!c || !u || !f) return fail(SIPG_EINVAL, "null argument");
  if (u == f) return fail(SIPG_EINVAL, "u and f must not alias");
  return guarded([&]() {
    vcycle_impl<double>(c, u, f, false, nullptr);
    return (int)SIPG_OK;
  });
}

int sipg_precond(sipg_ctx *c, const double *r, double *z) {
  if (!c || !r || !z) return fail(SIPG_EINVAL, "null argument");
  if (r == z) return fail(SIPG_EINVAL, "r and z must not alias");
  return guarded([&]() {
    precond_impl(c, r, z);
    return (int)SIPG_OK;
  });
}

int sipg_mg_solve(sipg_ctx *c, double *u, const double *f, double rtol, int maxcyc, int *ncyc,
                  double *relres) {
  if (!c || !u || !f) return fail(SIPG_EINVAL, "null argument");
  if (u == f) return fail(SIPG_EINVAL, "u and f must not alias");
  if (!(rtol > 0.0) || maxcyc < 0) return fail(SIPG_EINVAL, "need rtol > 0 and maxcyc >= 0");
  return guarded([&]() { return mg_solve_impl(c, u, f, rtol, maxcyc, ncyc, relres); });
}

int sipg_pcg_solve(sipg_ctx *c, double *u, const double *f, double rtol, int maxit, int *iters,
                   double *relres) {
  if (!c || !u || !f) return fail(SIPG_EINVAL, "null argument");
  if (u == f) return fail(SIPG_EINVAL, "u and f must not alias");
  if (!(rtol > 0.0) || maxit < 0) return fail(SIPG_EINVAL, "need rtol > 0 and maxit >= 0");
  return guarded([&]() { return pcg_solve_impl(c, u, f, rtol, maxit, iters, relres); });
}

int sipg_time_kernel(sipg_ctx *c, int kernel, int level, int bits, int reps, double *ms) {
  if (!c || !ms) return fail(SIPG_EINVAL, "null argument");
  if (reps < 1 || reps > 100000) return fail(SIPG_EINVAL, "reps must be in 1..100000");
  if (bits != 64 && bits != 32) return fail(SIPG_EINVAL, "bits must be 64 or 32");
  const int l = resolve_level(c, level);
  if (l < 1) return fail(SIPG_EINVAL, "level must be >= 1");
  if (kernel < SIPG_KERNEL_RESIDUAL || kernel > SIPG_KERNEL_PROLONG) return fail(SIPG_EINVAL, "unknown kernel");
  return guarded([&]() {
    auto run = [&](auto tag) {
      using T = decltype(tag);
      ensure_work<T>(c);
      Work<T> &w = work_of<T>(c);
      const int64_t N = level_ndof(c->H, l);
      T *u = w.uL, *f = w.fL, *r = w.r;
      check(sipg::launch_fill<T>(u, N, (T)0.25, c->stream), "fill");
      check(sipg::launch_fill<T>(f, N, (T)0.5, c->stream), "fill");
      check(sipg::launch_fill<T>(r, N, (T)0.75, c->stream), "fill");
      const LevelTabs<T> &t = tabs_of<T>(c, l);
      sipg::SchwarzLaunch<T> sa{c->mesh, t.n, t.schwarz, r, w.C, t.ilam, u, u, mfma_of(c, t), t.schwarz_spb};
      check(sipg::launch_schwarz_local<T>(sa, c->stream), "schwarz");  // valid corrections in C
      hipEvent_t e0, e1;
      check(hipEventCreate(&e0), "event");
      check(hipEventCreate(&e1), "event");
      // one untimed launch first: the first launch of a kernel in a process
      // also loads its code
      for (int i = -1; i < reps; ++i) {
        if (i == 0) check(hipEventRecord(e0, c->stream), "event");
        switch (kernel) {
          case SIPG_KERNEL_RESIDUAL: op_residual<T>(c, l, u, f, r); break;
          case SIPG_KERNEL_SCHWARZ_SOLVE: check(sipg::launch_schwarz_local<T>(sa, c->stream), "schwarz"); break;
          case SIPG_KERNEL_SCHWARZ_ASSEMBLE: check(sipg::launch_schwarz_assemble<T>(sa, c->stream), "assemble"); break;
          case SIPG_KERNEL_RESTRICT: op_residual_restrict<T>(c, l, u, f, w.f[l - 1]); break;
          case SIPG_KERNEL_PROLONG:
            if (l == 1) op_prolong<T, double>(c, 1, c->u0, false, u);
            else op_prolong<T, T>(c, l, w.u[l - 1], false, u);
            break;
        }
      }
      check(hipEventRecord(e1, c->stream), "event");
      check(hipEventSynchronize(e1), "event");
      float el = 0.f;
      check(hipEventElapsedTime(&el, e0, e1), "event");
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      *ms = (double)el / reps;
    };
    if (bits == 64) run(double());
    else run(float());
    return (int)SIPG_OK;
  });
}

int sipg_autotune(sipg_ctx *c, int reps) {
  if (!c) return fail(SIPG_EINVAL, "null context");
  if (reps < 1 || reps > 1000) return fail(SIPG_EINVAL, "reps must be in 1..1000");
  return guarded([&]() {
    // a captured preconditioner holds the old launch shapes
    if (c->precond_graph) {
      check(hipStreamSynchronize(c->stream), "sync");
      check(hipGraphExecDestroy(c->precond_graph), "graph");
      c->precond_graph = nullptr;
    }
    for (int l = 1; l <= c->L; ++l) tune_level<double>(c, l, reps);
    if (c->H.prm.precond_bits != 64)
      for (int l = 1; l <= c->L; ++l) tune_level<float>(c, l, reps);
    check(hipStreamSynchronize(c->stream), "autotune");
    return (int)SIPG_OK;
  });
}

int sipg_tuning_cache_save(const char *path) {
  if (!path) return fail(SIPG_EINVAL, "null path");
  std::string out = "{\"sipg_tuning_cache\": 1, \"entries\": [";
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    bool first = true;
    for (const auto &kv : g_tuned) {
      const auto &k = kv.first;
      char buf[256];
      std::snprintf(buf, sizeof buf,
                    "%s\n  {\"bits\": %d, \"n\": %d, \"mx\": %d, \"my\": %d, \"mz\": %d, \"elements\": %d, "
                    "\"mfma\": %d, \"apply_epb\": %d, \"schwarz_spb\": %d}",
                    first ? "" : ",", k[0], k[1], k[2], k[3], k[4], k[5], k[6], kv.second[0], kv.second[1]);
      out += buf;
      first = false;
    }
  }
  out += "\n]}\n";
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(SIPG_EINVAL, std::string("cannot write ") + tmp);
  const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
  if (std::fclose(f) != 0 || !ok || std::rename(tmp.c_str(), path) != 0)
    return fail(SIPG_EINVAL, std::string("cannot write ") + path);
  return SIPG_OK;
}

int sipg_tuning_cache_load(const char *path, int *nloaded) {
  if (!path) return fail(SIPG_EINVAL, "null path");
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(SIPG_EINVAL, std::string("cannot read ") + path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  if (text.find("\"sipg_tuning_cache\"") == std::string::npos) return fail(SIPG_EINVAL, "not a tuning cache");
  size_t p = text.find("\"entries\"");
  if (p == std::string::npos) return fail(SIPG_EINVAL, "tuning cache without entries");
  std::vector<std::pair<std::array<int, 7>, std::array<int, 2>>> got_entries;
  while ((p = text.find('{', p)) != std::string::npos) {
    const size_t q = text.find('}', p);
    if (q == std::string::npos) return fail(SIPG_EINVAL, "malformed tuning cache");
    const std::string obj = text.substr(p, q - p + 1);
    const char *keys[9] = {"bits", "n", "mx", "my", "mz", "elements", "mfma", "apply_epb", "schwarz_spb"};
    long v[9];
    for (int i = 0; i < 9; ++i)
      if (!json_int(obj, keys[i], &v[i])) return fail(SIPG_EINVAL, std::string("tuning cache entry without ") + keys[i]);
    const bool ok = (v[0] == 32 || v[0] == 64) && v[1] >= 2 && v[1] <= sipg::kMaxOrder + 1 && v[2] >= 1 &&
                    v[2] <= 256 && v[3] >= 1 && v[3] <= 256 && v[4] >= 1 && v[4] <= 256 && v[5] >= 1 &&
                    (v[6] == 0 || v[6] == 1) && v[7] >= 0 && v[7] <= 1024 && v[8] >= 0 && v[8] <= 64;
    if (!ok) return fail(SIPG_EINVAL, "tuning cache entry out of range");
    got_entries.push_back({{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], (int)v[5], (int)v[6]},
                           {(int)v[7], (int)v[8]}});
    p = q + 1;
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto &e : got_entries) g_tuned[e.first] = e.second;
  }
  if (nloaded) *nloaded = (int)got_entries.size();
  return SIPG_OK;
}

int sipg_tuning(const sipg_ctx *c, int level, int bits, int *apply_epb, int *schwarz_spb) {
  if (!c || !apply_epb || !schwarz_spb) return fail(SIPG_EINVAL, "null argument");
  if (bits != 64 && bits != 32) return fail(SIPG_EINVAL, "bits must be 64 or 32");
  const int l = level == -1 ? c->L : level;
  if (l < 1 || l > c->L) return fail(SIPG_EINVAL, "level must be in 1..L or -1");
  if (bits == 64) {
    *apply_epb = c->t64[l].apply_epb;
    *schwarz_spb = c->t64[l].schwarz_spb;
  } else {
    *apply_epb = c->t32[l].apply_epb;
    *schwarz_spb = c->t32[l].schwarz_spb;
  }
  return SIPG_OK;
}

int sipg_tuning_limits(const sipg_ctx *c, int level, int bits, int *max_apply_epb, int *max_schwarz_spb) {
  if (!c || !max_apply_epb || !max_schwarz_spb) return fail(SIPG_EINVAL, "null argument");
  if (bits != 64 && bits != 32) return fail(SIPG_EINVAL, "bits must be 64 or 32");
  if (bits == 32 && c->H.prm.precond_bits == 64) return fail(SIPG_EINVAL, "an FP64 context has no FP32 levels");
  const int l = level_arg(c, level);
  if (!l) return fail(SIPG_EINVAL, "level must be in 1..L or -1");
  if (bits == 64)
    tuning_limits_of<double>(c, c->t64[l], max_apply_epb, max_schwarz_spb);
  else
    tuning_limits_of<float>(c, c->t32[l], max_apply_epb, max_schwarz_spb);
  return SIPG_OK;
}

int sipg_set_tuning(sipg_ctx *c, int level, int bits, int apply_epb, int schwarz_spb) {
  int me = 0, ms = 0;
  const int st = sipg_tuning_limits(c, level, bits, &me, &ms);
  if (st != SIPG_OK) return st;
  if (apply_epb < 0 || apply_epb > std::max(me, 0) || (apply_epb > 0 && me < 1))
    return fail(SIPG_EINVAL, "apply_epb out of range for this level");
  if (schwarz_spb < 0 || schwarz_spb > std::max(ms, 0) || (schwarz_spb > 0 && ms < 1))
    return fail(SIPG_EINVAL, "schwarz_spb out of range for this level");
  return guarded([&]() {
    if (c->precond_graph) {
      check(hipStreamSynchronize(c->stream), "sync");
      check(hipGraphExecDestroy(c->precond_graph), "graph");
      c->precond_graph = nullptr;
    }
    const int l = level_arg(c, level);
    if (bits == 64) {
      c->t64[l].apply_epb = apply_epb;
      c->t64[l].schwarz_spb = schwarz_spb;
    } else {
      c->t32[l].apply_epb = apply_epb;
      c->t32[l].schwarz_spb = schwarz_spb;
    }
    return (int)SIPG_OK;
  });
}

int sipg_set_option(sipg_ctx *c, int option, int value) {
  if (!c) return fail(SIPG_EINVAL, "null context");
  if (option == SIPG_OPT_GRAPH) {
    c->use_graph = value != 0;
    return SIPG_OK;
  }
  if (option == SIPG_OPT_WIDE_PLANES) {
    if (value < 0 || value > 16) return fail(SIPG_EINVAL, "wide planes must be in 0..16");
    c->wide_planes = value;
    if (c->precond_graph) {  // captured with the previous launch shapes
      (void)hipGraphExecDestroy(c->precond_graph);
      c->precond_graph = nullptr;
    }
    return SIPG_OK;
  }
  if (option != SIPG_OPT_TRACE_KERNEL) return fail(SIPG_EINVAL, "unknown option");
  if (value != -1 && (value < SIPG_KERNEL_RESIDUAL || value > SIPG_KERNEL_PROLONG))
    return fail(SIPG_EINVAL, "trace kernel must be -1 or a SIPG_KERNEL_* value");
  return guarded([&]() {
    if (value >= 0 && c->trace_ev.empty()) {
      c->trace_ev.assign(2 * kTraceMax, nullptr);
      // device-scope release: no system-wide cache flush at each record
      for (hipEvent_t &e : c->trace_ev) check(hipEventCreateWithFlags(&e, hipEventReleaseToDevice), "trace event");
    }
    c->trace_kernel = value;
    c->trace_n = 0;
    return (int)SIPG_OK;
  });
}

int sipg_traced_kernel_ms(sipg_ctx *c, double *mean_ms, int *count) {
  if (!c || !mean_ms || !count) return fail(SIPG_EINVAL, "null argument");
  return guarded([&]() {
    double sum = 0.0;
    const int n = c->trace_n;
    if (n > 0) check(hipEventSynchronize(c->trace_ev[2 * n - 1]), "trace event");
    for (int k = 0; k < n; ++k) {
      float ms = 0.f;
      check(hipEventElapsedTime(&ms, c->trace_ev[2 * k], c->trace_ev[2 * k + 1]), "trace event");
      sum += ms;
    }
    *count = n;
    *mean_ms = n > 0 ? sum / n : 0.0;
    c->trace_n = 0;
    return (int)SIPG_OK;
  });
}

int sipg_residual_history(const sipg_ctx *c, double *out, int cap, int *n) {
  if (!c || !n) return fail(SIPG_EINVAL, "null argument");
  *n = (int)c->hist.size();
  if (out)
    for (int i = 0; i < cap && i < *n; ++i) out[i] = c->hist[i];
  return SIPG_OK;
}

int sipg_host_table(const sipg_params *p, int level, int dir, int which, double *out, int cap, int *count) {
  if (!p || !count) return fail(SIPG_EINVAL, "null argument");
  if (dir < 0 || dir > 2) return fail(SIPG_EINVAL, "dir must be 0, 1 or 2");
  return guarded([&]() {
    sipg::HierarchyHost H;
    sipg::build_hierarchy(*p, H);
    const int L = (int)H.lev.size() - 1;
    const int l = level == -1 ? L : level;
    if (l < 0 || l > L) throw std::invalid_argument("level out of range");
    const sipg::Dir1D &D = H.lev[l].dir[dir];
    std::vector<double> v;
    switch (which) {
      case SIPG_TAB_NODES: v = D.xi; break;
      case SIPG_TAB_WEIGHTS: v = D.w; break;
      case SIPG_TAB_DERIV: v = D.D; break;
      case SIPG_TAB_MASS: v = D.mass; break;
      case SIPG_TAB_LDIAG: v = D.Ld; break;
      case SIPG_TAB_LUPPER: v = D.U; break;
      case SIPG_TAB_OVERLAP: v = {(double)D.no}; break;
      case SIPG_TAB_SUB_L: v = D.Ls; break;
      case SIPG_TAB_SUB_M: v = D.Ms; break;
      case SIPG_TAB_SUB_LAM: v = D.lam; break;
      case SIPG_TAB_SUB_S: v = D.S; break;
      case SIPG_TAB_SUB_W: v = D.wsub; break;
      case SIPG_TAB_INTERP: v = H.lev[l].J; break;
      case SIPG_TAB_COARSE_LAM: v = H.coarse.lam[dir]; break;
      case SIPG_TAB_COARSE_S: v = H.coarse.S[dir]; break;
      case SIPG_TAB_SUB_LAM_EO: v = D.lam_eo; break;
      case SIPG_TAB_SUB_S_EO: v = D.S_eo; break;
      default: throw std::invalid_argument("unknown table");
    }
    if (((which >= SIPG_TAB_SUB_L && which <= SIPG_TAB_SUB_W) || which == SIPG_TAB_SUB_LAM_EO ||
         which == SIPG_TAB_SUB_S_EO) && l == 0)
      throw std::invalid_argument("level 0 has no subdomain tables");
    if (which == SIPG_TAB_INTERP && l == 0) throw std::invalid_argument("level 0 has no interpolation");
    *count = (int)v.size();
    if (out)
      for (int i = 0; i < cap && i < (int)v.size(); ++i) out[i] = v[i];
    return (int)SIPG_OK;
  });
}

}  // extern "C"
