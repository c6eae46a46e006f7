/*
 * sipg_mg.h -- C ABI of the MI355X p-multigrid / weighted overlapping Schwarz
 * solver for the nodal symmetric interior penalty DG (SIPG) discretization of
 * the periodic Poisson problem -lap u = f on [0,lx] x [0,ly] x [0,lz]
 * (Stiller, "Robust Multigrid for Cartesian Interior Penalty DG Formulations
 * of the Poisson Equation in 3D", arXiv 1612.04796).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Vectors.  All vector arguments are DEVICE pointers (HIP global memory of
 *   the current device), owned by the caller, holding one level's
 *   coefficients in element-major order: index
 *       ((ez*ney + ey)*nex + ex) * n^3 + (k*n + j)*n + i
 *   with n = P_l + 1 GLL nodes per direction, x fastest inside and across
 *   elements.  Level l has E*n_l^3 values (E = nex*ney*nez).  double* means
 *   FP64; the precision of the preconditioner (sipg_params.precond_bits)
 *   changes only internal storage.  Input and output vectors must not alias
 *   unless the entry point says "in place".
 * Levels.  Level 0 is the coarsest (P_0 = 1), level L the top (P_L = P);
 *   the orders are 1, 2, 4, ..., 2^k < P, P (P_l = 2^l when P is a power of
 *   two, Sec. 3.2).  level = -1 means the top level.
 * Streams.  Every device operation is enqueued on the stream given to
 *   sipg_setup (NULL = the default stream).  Entry points marked "async"
 *   return without synchronizing; the solvers synchronize to read residual
 *   norms.
 * Errors.  Every entry point returns a sipg_status; on failure the message is
 *   in sipg_last_error() (thread local) and the outputs are unspecified
 *   unless the entry point says otherwise.  Invalid arguments are rejected
 *   before any device work is enqueued.
 */
#ifndef SIPG_MG_H
#define SIPG_MG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sipg_ctx sipg_ctx; /* opaque: hierarchy, tables and work space in HBM */

typedef enum {
  SIPG_OK = 0,
  SIPG_EINVAL = -1,      /* invalid argument or unsupported configuration      */
  SIPG_ENOMEM = -2,      /* device or host allocation failed                   */
  SIPG_EHIP = -3,        /* a HIP runtime call or kernel launch failed         */
  SIPG_ENOCONV = -4,     /* tolerance not reached within the iteration limit   */
  SIPG_EBREAKDOWN = -5,  /* flexible CG breakdown (p.Ap <= 0 or not finite)    */
  SIPG_ENOTFINITE = -6   /* a residual norm became NaN or infinite            */
} sipg_status;

/* Overlap of the element-centred Schwarz subdomains (Sec. 3.1, Tables 1-2):
 *   MIN: one node layer from each neighbour (N_O = 1);
 *   REL: width delta_O = omega * h_d in direction d;
 *   MAX: width min(omega * max_k h_k, h_d).
 * N_O on each level counts the neighbour nodes whose distance from the shared
 * face is at most delta_O (GLL) or below it (GL: possibly 0, the subdomain is
 * then the element), and is at least overlap_floor. */
typedef enum { SIPG_OVL_MIN = 0, SIPG_OVL_REL = 1, SIPG_OVL_MAX = 2 } sipg_overlap_mode;

/* Nodal basis of every level (Sec. 2; Table 1): Gauss-Lobatto-Legendre nodes
 * (end points are nodes: a face trace is one nodal value) or Gauss-Legendre
 * nodes (no node at the ends: traces and normal derivatives at a face are
 * combinations of a whole element line). */
typedef enum { SIPG_BASIS_GLL = 0, SIPG_BASIS_GL = 1 } sipg_basis;

typedef struct {
  int32_t ne[3];          /* elements per direction (x, y, z); 3..1024, and >= 4 in
                             a direction whose subdomain takes whole neighbours
                             (and in every direction with the GL basis)          */
  double len[3];          /* domain lengths lx, ly, lz > 0                         */
  int32_t P;              /* polynomial order, 1..16 or 32                         */
  double penalty;         /* c_mu: mu_d = c_mu P_l (P_l + 1) / h_d on level l;
                             must exceed 1/2 (the stability threshold); 1.0 is
                             the paper's setting read as twice the threshold      */
  int32_t overlap_mode;   /* sipg_overlap_mode                                      */
  double overlap;         /* omega in [0, 1]; ignored for SIPG_OVL_MIN             */
  int32_t nsmooth_pre;    /* pre-smoothing steps on the top level  (V(1,1): 1)     */
  int32_t nsmooth_post;   /* post-smoothing steps on the top level (V(1,1): 1)     */
  int32_t smooth_growth;  /* steps on level l are multiplied by growth^(L-l);
                             1 = fixed V-cycle, 3 = the variable V-cycle of Table 2 */
  int32_t precond_bits;   /* precision of the multigrid preconditioner inside
                             sipg_pcg_solve and of sipg_precond: 64, 32 (FP32
                             storage and arithmetic, coarse solve in FP64) or 16
                             (as 32, but the local fast-diagonalization solves of
                             levels with cubic subdomains of 10-13 nodes (P = 7, 8)
                             run in FP16 on the matrix cores with FP32
                             accumulation and per-subdomain power-of-two scaling) */
  int32_t basis;          /* SIPG_BASIS_GLL (0, the default) or SIPG_BASIS_GL; GL
                             needs ne >= 4 in every direction                      */
  int32_t overlap_floor;  /* lower bound of N_O on every level for REL and MAX
                             overlaps, 0..2 (0: none; Table 1 rows 13-14 use 1)    */
} sipg_params;

/* Fills *p with the defaults: ne = 4^3, unit cube, P = 4, penalty 1.0,
 * minimal overlap, omega 0.08, V(1,1), growth 1, precond_bits 64, GLL basis,
 * no overlap floor. */
void sipg_default_params(sipg_params *p);

/* Builds the level hierarchy (Sec. 3.2): for every level and direction the
 * GLL rule, the 1D mass and SIPG stiffness blocks of eq. (A), the overlap
 * layers N_O, the generalized eigenpairs of the restricted 1D pairs used by
 * the fast diagonalization of Sec. 3.1, the hat weights, the interpolation
 * matrices, and the global level-0 eigenpairs of the coarse pseudo-inverse;
 * then allocates all level vectors and work space on the current device and
 * uploads the tables on `hip_stream` (a hipStream_t, may be NULL).
 * On success *out owns everything; release it with sipg_destroy. */
int sipg_setup(const sipg_params *p, void *hip_stream, sipg_ctx **out);

/* Frees all device and host memory of the context (NULL is accepted). */
int sipg_destroy(sipg_ctx *c);

/* Device bytes sipg_setup allocates for *p (for admission control), computed
 * on the host without touching the device: the tables, the level-0 and
 * flexible-CG vectors, the work space of the preconditioner precision and the
 * scratch of the outer FP64 operator, i.e. everything sipg_pcg_solve and
 * sipg_precond use, so neither allocates after sipg_setup.  The FP64 entry
 * points (sipg_vcycle, sipg_mg_solve, sipg_smooth, ...) on a context with
 * precond_bits 32 or 16 allocate the FP64 work space on their first call,
 * beyond this figure. */
int sipg_footprint(const sipg_params *p, size_t *bytes);

/* Device bytes the context holds now (sipg_footprint plus what FP64 entry
 * points allocated on an FP32/FP16-preconditioned context). */
int sipg_device_bytes(const sipg_ctx *c, size_t *bytes);

/* Number of levels L + 1. */
int sipg_nlevels(const sipg_ctx *c, int *nlevels);

/* Unknowns E*n_l^3 of level l (level -1: the top), the length of every
 * vector argument on that level. */
int sipg_ndof(const sipg_ctx *c, int level, int64_t *n);

/* Order P_l, overlap layers N_O per direction and unknowns E*n^3 of level l. */
int sipg_level_info(const sipg_ctx *c, int level, int *order, int no[3], int64_t *ndof);

/* Discrete right-hand side of a Fourier load, async:
 *   f(x) = sum_q amp[q] prod_d sin(2 pi k[3q+d] x_d / l_d + phi[3q+d]),
 *   b = (Mz x My x Mx) f(GLL nodes)  (GLL quadrature of int v f, Sec. 2),
 * followed by removal of the Euclidean mean of b (projection onto the range
 * of the singular periodic operator).  k, phi, amp are HOST arrays of
 * nmodes*3, nmodes*3 and nmodes entries (1 <= nmodes <= 64); b is a device
 * vector of the top level. */
int sipg_rhs_fourier(sipg_ctx *c, int nmodes, const int32_t *k, const double *phi,
                     const double *amp, double *b);

/* y = A_l u, async.  A_l is the Kronecker-sum operator of eq. (A) on level l,
 * applied element by element by sum factorization with face coupling to the
 * six neighbours. */
int sipg_apply_A(sipg_ctx *c, int level, const double *u, double *y);

/* r = f - A_l u, async (the residual form of Sec. 3.1). */
int sipg_residual(sipg_ctx *c, int level, const double *u, const double *f, double *r);

/* u += sum_s R_s^T W_s A_ss^{-1} R_s r on level l >= 1, async: one weighted
 * additive Schwarz correction (eq. (correction:global)) with every local
 * problem solved by fast diagonalization.  In place on u. */
int sipg_schwarz(sipg_ctx *c, int level, const double *r, double *u);

/* sipg_schwarz for callers that cannot allocate device memory at call time
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same computation and kernels, async, in place on u, with
 * the per-subdomain corrections kept in a fixed device array of the library
 * (96 MiB per device, held until the process ends) instead of the context's
 * work space, and no allocation of any kind (sipg_schwarz allocates the FP64
 * work space on its first call on a context with precond_bits 32 or 16).
 * SIPG_EINVAL when level l needs more than 96 MiB of corrections (E times
 * m_x m_y m_z doubles).  The array is shared by every call on a device:
 * calls that overlap on one device (several streams or threads) race and
 * must be serialized by the caller. */
int sipg_schwarz_noalloc(sipg_ctx *c, int level, const double *r, double *u);

/* nsteps smoothing steps on level l >= 1, in place on u, async: each step is
 * r = f - A_l u followed by sipg_schwarz. */
int sipg_smooth(sipg_ctx *c, int level, double *u, const double *f, int nsteps);

/* f_{l-1} = I_l^T r_l, async: transposed embedded interpolation (level l >= 1). */
int sipg_restrict(sipg_ctx *c, int level, const double *r_fine, double *f_coarse);

/* u_l += I_l u_{l-1}, async: embedded interpolation (level l >= 1), in place
 * on u_fine. */
int sipg_prolong_add(sipg_ctx *c, int level, const double *u_coarse, double *u_fine);

/* u_0 = A_0^+ f_0, async: minimum Euclidean norm solution on level 0
 * (Algorithm 1, coarse grid solution), by projecting f_0 onto the range of
 * A_0 and fast diagonalization with the global periodic 1D eigenpairs. */
int sipg_coarse_solve(sipg_ctx *c, const double *f0, double *u0);

/* One multigrid V-cycle (Algorithm 1) in FP64 from the top-level value u for
 * the right side f, in place on u, async. */
int sipg_vcycle(sipg_ctx *c, double *u, const double *f);

/* z = B r: one V-cycle started from zero, in the preconditioner precision of
 * the context (FP64, or FP32 with the coarse solve in FP64), async.  This is
 * the preconditioner of sipg_pcg_solve. */
int sipg_precond(sipg_ctx *c, const double *r, double *z);

/* The solvers and the singular periodic problem.  A has the constants as
 * its null space (Sec. 2; Sec. 3.2, where Algorithm 1 uses the pseudo-inverse
 * A_0^+ on the coarse level), so A u = f is solvable only for f orthogonal
 * to the constants.  sipg_mg_solve and sipg_pcg_solve therefore solve
 * A u = f - mean(f) 1 (the Euclidean projection of f onto the range of A,
 * in a copy: f itself is not modified; sipg_rhs_mean returns the mean
 * removed) and return, on SIPG_OK, the solution of zero Euclidean mean, the
 * minimum-norm one.  Residual norms and rtol refer to the projected f. */

/* Multigrid solve: repeats V-cycles from the value in u until
 * ||f - A u||_2 <= rtol ||f - A u_start||_2 (f projected, see above).  On
 * return *ncyc holds the cycles run and *relres the final relative residual;
 * u has zero mean.  SIPG_ENOCONV if maxcyc cycles do not reach rtol (u holds
 * the last iterate, mean removed).  Synchronizes. */
int sipg_mg_solve(sipg_ctx *c, double *u, const double *f, double rtol, int maxcyc,
                  int *ncyc, double *relres);

/* Flexible (inexact preconditioned) CG (Sec. 3.2) with one V-cycle from zero
 * as preconditioner, FP64 outer iteration, starting from the value in u,
 * until the residual of the projected f satisfies ||r||_2 <= rtol ||r_0||_2,
 * confirmed by a recomputed FP64 residual of the iterate with its mean
 * removed.  *iters: operator applications in the loop.  SIPG_ENOCONV /
 * SIPG_EBREAKDOWN leave the last iterate in u (its mean not removed).
 * Allocates nothing (see sipg_footprint).  Synchronizes. */
int sipg_pcg_solve(sipg_ctx *c, double *u, const double *f, double rtol, int maxit,
                   int *iters, double *relres);

/* Euclidean mean of f removed by the last sipg_mg_solve / sipg_pcg_solve
 * (0 before any solve). */
int sipg_rhs_mean(const sipg_ctx *c, double *mean);

/* Residual norms of the last mg/pcg solve (index 0 = start); copies at most
 * cap values to the HOST array out and sets *n to the number available. */
int sipg_residual_history(const sipg_ctx *c, double *out, int cap, int *n);

/* Kernels of the hot path that sipg_time_kernel can time in isolation. */
typedef enum {
  SIPG_KERNEL_RESIDUAL = 0,        /* r = f - A_l u (operator apply, eq. (A))          */
  SIPG_KERNEL_SCHWARZ_SOLVE = 1,   /* the local fast-diagonalization solves of all
                                      subdomains (writes the per-subdomain corrections) */
  SIPG_KERNEL_SCHWARZ_ASSEMBLE = 2,/* u += sum of the weighted corrections             */
  SIPG_KERNEL_RESTRICT = 3,        /* f_{l-1} = I_l^T (f_l - A_l u_l), fused           */
  SIPG_KERNEL_PROLONG = 4          /* u_l += I_l u_{l-1}                                */
} sipg_kernel;

/* Measurement support: enqueues `reps` back-to-back launches of one kernel of
 * the hot path on level l (>= 1) of the context, in precision bits (64, or 32
 * for an FP32-preconditioner context), on the context stream, bracketed by two
 * HIP events recorded on that same stream, and returns the mean duration of
 * one launch in *ms.  The kernels run on the context's internal work vectors,
 * whose contents are overwritten (set to a fixed pattern first).
 * Synchronizes. */
int sipg_time_kernel(sipg_ctx *c, int kernel, int level, int bits, int reps, double *ms);

/* Autotuner.  For every level >= 1 of the context (FP64, and FP32 when
 * precond_bits is 32 or 16) times each candidate launch shape of the
 * operator kernel (elements per workgroup: powers of two up to the most that
 * fit 256 threads) and of the compile-time-shape local-solve kernel
 * (subdomains per workgroup, 1 up to the most its LDS tile allows) with
 * `reps` launches between HIP events on the context stream, and keeps the
 * fastest for all later launches of the context.  Choices are cached for the
 * process by (precision, order, subdomain shape, element count), so later
 * contexts of the same shape take them without timing.  Every element and
 * subdomain is computed as before; only the partition of the fused p.Ap and
 * residual-norm partial sums follows the new workgroup count.  Overwrites
 * the context's internal work vectors; drops a captured preconditioner graph
 * (captured again on its next use).  Synchronizes.  reps in 1..1000. */
int sipg_autotune(sipg_ctx *c, int reps);
/* Launch shapes in use on level `level` (>= 1, or -1 for the top) in
 * precision `bits` (64 or 32): elements per workgroup of the operator kernel
 * and subdomains per workgroup of the local-solve kernel; 0 = the built-in
 * default (not tuned, or the level has no such kernel). */
int sipg_tuning(const sipg_ctx *c, int level, int bits, int *apply_epb, int *schwarz_spb);
/* Sets the launch shapes of level `level` (>= 1, or -1 for the top) in
 * precision `bits` (64, or 32 for a context whose preconditioner is not
 * FP64): apply_epb elements per operator workgroup (0 = default, else
 * 1..sipg_tuning_limits' first value) and schwarz_spb subdomains per
 * local-solve workgroup (0 = default, else 1..its second value; only the
 * compile-time-shape local solves take it).  The computed values do not
 * depend on the shapes (only the partition of the fused partial sums does).
 * Drops a captured preconditioner graph.  For restoring shapes tuned
 * earlier (e.g. from a tuning cache); EINVAL for values out of range. */
int sipg_set_tuning(sipg_ctx *c, int level, int bits, int apply_epb, int schwarz_spb);
/* Largest values sipg_set_tuning accepts on that level (0 = the level has
 * no choice of that shape). */
int sipg_tuning_limits(const sipg_ctx *c, int level, int bits, int *max_apply_epb, int *max_schwarz_spb);
/* The process-wide tuning cache (the choices sipg_autotune made, keyed by
 * precision, order, subdomain shape, element count and local-solve kind)
 * as a JSON file: saved to `path` (written to path.tmp, then renamed), or
 * merged from such a file (nloaded: entries read, may be null).  Later
 * sipg_autotune calls and served requests take cached choices without
 * timing.  EINVAL for an unreadable or malformed file (then nothing is
 * merged).  The serving loop loads the file named by the environment
 * variable SIPG_TUNING_CACHE when it is created. */
int sipg_tuning_cache_save(const char *path);
int sipg_tuning_cache_load(const char *path, int *nloaded);

/* Context options. */
typedef enum {
  SIPG_OPT_GRAPH = 0,       /* value 1: capture the flexible-CG preconditioner V-cycle into a
                               HIP graph on its first use and replay it afterwards (needs a
                               non-NULL stream at sipg_setup; kernel nodes only) */
  SIPG_OPT_TRACE_KERNEL = 1,/* value k in SIPG_KERNEL_RESIDUAL..SIPG_KERNEL_PROLONG: from now
                               on every launch of that kernel on the top level in the
                               preconditioner's precision (FP64 for precond_bits 64, FP32
                               for 32 and 16; inside sipg_mg_solve, sipg_pcg_solve,
                               sipg_vcycle, ...), outside graph capture, is bracketed by a
                               pair of HIP events on the context's stream (at most 1024
                               launches are kept; later ones are not timed); -1 stops.
                               Setting it drops the launches recorded so far.  Allocates
                               the events when first set (not inside the solves). */
  SIPG_OPT_WIDE_PLANES = 2  /* value 1..16: the local solves of subdomains too large for one
                               workgroup's LDS process that many 2D planes per wave (matrix-core
                               kernels) or per workgroup (vector plane kernels); 0 (default):
                               chosen from the mesh size.  Results do not depend on it (a launch
                               shape only).  Drops a captured preconditioner graph. */
} sipg_option;
int sipg_set_option(sipg_ctx *c, int option, int value);
/* Launch durations recorded under SIPG_OPT_TRACE_KERNEL: waits for the last
 * recorded event, returns their count and mean duration in milliseconds
 * (*mean_ms = 0 when none), and drops them (tracing stays on). */
int sipg_traced_kernel_ms(sipg_ctx *c, double *mean_ms, int *count);

/* ---- serving: continuous batching of heterogeneous solves ---------------
 * A server accepts solves of any mesh, order and aspect ratio (each a
 * sipg_params plus a Fourier right-hand side as in sipg_rhs_fourier) and runs
 * them with the flexible CG of sipg_pcg_solve.  Requests wait in a FIFO queue
 * and are admitted when one of max_active slots is free and their device
 * footprint (sipg_footprint plus the solution and right-hand side vectors)
 * fits the memory budget.  Each admitted request owns a context, a stream and
 * a graph-captured preconditioner; its steps are enqueued as soon as its
 * previous step completes, so admitted requests run concurrently on the
 * device.  A request's result is bitwise the one sipg_pcg_solve gives alone.
 * The server is not thread safe: one host thread drives it. */
typedef struct sipg_server sipg_server;
typedef enum { SIPG_REQ_QUEUED = 0, SIPG_REQ_ACTIVE = 1, SIPG_REQ_DONE = 2, SIPG_REQ_FAILED = 3 } sipg_req_state;

/* memory_budget: device bytes the server may hold for requests (> 0). */
int sipg_server_create(size_t memory_budget, int max_active, sipg_server **out);

/* Queues a solve to rel. residual rtol within maxit iterations; k/phi/amp are
 * HOST arrays as in sipg_rhs_fourier (copied).  *id identifies the request.
 * SIPG_EINVAL for invalid parameters, SIPG_ENOMEM when the request's footprint
 * (sipg_footprint plus its two vectors) exceeds the whole memory budget, so
 * that it could never be admitted (nothing is queued in either case).  An
 * admitted request's solution stays reserved in the budget until it is
 * fetched: a client that never fetches can keep later requests queued. */
int sipg_server_submit(sipg_server *s, const sipg_params *p, int nmodes, const int32_t *k, const double *phi,
                       const double *amp, double rtol, int maxit, int64_t *id);

/* Admits what fits and advances every request whose last step completed;
 * returns once at least one request finished (done or failed), or after
 * wait_ms milliseconds, or when nothing is left.  Outputs may be NULL. */
int sipg_server_progress(sipg_server *s, int wait_ms, int *nactive, int *nqueued, int *ncompleted);

/* State (sipg_req_state), iterations, final relative residual, times[3] =
 * (submitted, admitted, finished) in seconds since the server was created,
 * and unknowns of a request.  Outputs may be NULL.  For a failed request the
 * reason is in sipg_last_error(). */
int sipg_server_status(sipg_server *s, int64_t id, int *state, int *iters, double *relres, double times[3],
                       int64_t *ndof);

/* Copies the solution of a finished request into the DEVICE vector u (its
 * unknowns, element-major) on hip_stream, synchronizes that stream, and frees
 * the request's memory. */
int sipg_server_fetch(sipg_server *s, int64_t id, double *u, void *hip_stream);

/* Server options.  SIPG_SERVER_FUSE_APPLY (default 1): when several active
 * requests of the same order, the same operator launch shape and a similar
 * size (unknowns within a factor of 8) are ready for a flexible-CG iteration
 * at the same time, their outer operator applications q = A p (with the p.q
 * partial sums) run as one launch over all of them (at most 8), on a stream
 * of the server (one per such class of requests) that waits for each
 * member's preconditioner; the rest of the members' steps follows on that
 * stream, and members stay in phase from step to step.  Every member computes exactly what
 * it computes alone.  0: every request steps on its own stream only. */
/* SIPG_SERVER_FUSE_SMOOTH (default 1): within such a group, the members
 * whose preconditioners have the same signature (precision, level orders,
 * subdomain shapes and smoothing counts, every level on a compile-time
 * local-solve shape) run their preconditioner V-cycles as one cohort on the
 * group's stream: level by level, the Schwarz local solves of all members
 * in one launch and their assemblies in one launch, the residuals,
 * transfers and coarse solves per member.  Every member again computes
 * exactly what it computes alone.  0: each member's V-cycle on its own
 * stream.
 * SIPG_SERVER_TUNE: launch shapes of admitted requests.  0 (the default):
 * the built-in defaults; 1 (the default when SIPG_TUNING_CACHE names a cache
 * file, which sipg_server_create then loads): the shapes the process-wide
 * tuning cache holds for the request's levels (see sipg_tuning_cache_load;
 * no timing); 2: sipg_autotune at admission (shapes already cached are
 * taken without timing), and at sipg_server_destroy the cache is saved to
 * the file named by SIPG_TUNING_CACHE, if set.  A served result equals,
 * bitwise, the same solve run alone with the same launch shapes (the
 * operator's launch shape sets the partition of the flexible-CG dot
 * products). */
typedef enum { SIPG_SERVER_FUSE_APPLY = 0, SIPG_SERVER_FUSE_SMOOTH = 1, SIPG_SERVER_TUNE = 2 } sipg_server_option;
int sipg_server_set_option(sipg_server *s, int option, int value);

/* Fused operator launches so far and the requests they served. */
int sipg_server_stats(const sipg_server *s, int64_t *fused_launches, int64_t *fused_requests);
/* Cohort V-cycles (SIPG_SERVER_FUSE_SMOOTH) so far and the requests they served. */
int sipg_server_smooth_stats(const sipg_server *s, int64_t *cohort_cycles, int64_t *cohort_requests);

/* Waits for the device and frees everything the server holds. */
int sipg_server_destroy(sipg_server *s);

/* Message of the last failed call on this thread ("" if none). */
const char *sipg_last_error(void);

/* ---- host-only table queries (no device needed; for verification) ------ */
typedef enum {
  SIPG_TAB_NODES = 0,      /* GLL nodes xi (n)                                 */
  SIPG_TAB_WEIGHTS = 1,    /* GLL weights (n)                                  */
  SIPG_TAB_DERIV = 2,      /* D[i][j] = phi_j'(xi_i) (n x n)                   */
  SIPG_TAB_MASS = 3,       /* element mass diagonal (h/2) w (n)                */
  SIPG_TAB_LDIAG = 4,      /* element diagonal block of L_d (n x n)            */
  SIPG_TAB_LUPPER = 5,     /* coupling block L_{e,e+1} of L_d (n x n)          */
  SIPG_TAB_OVERLAP = 6,    /* N_O (1 value)                                    */
  SIPG_TAB_SUB_L = 7,      /* restricted L_s (m x m)                           */
  SIPG_TAB_SUB_M = 8,      /* restricted M_s (m)                               */
  SIPG_TAB_SUB_LAM = 9,    /* generalized eigenvalues of (L_s, M_s), ascending */
  SIPG_TAB_SUB_S = 10,     /* eigenvectors S (m x m, column j = pair j)        */
  SIPG_TAB_SUB_W = 11,     /* 1D hat weights (m)                               */
  SIPG_TAB_INTERP = 12,    /* J (n_l x n_{l-1}) from level l-1 to level l      */
  SIPG_TAB_COARSE_LAM = 13,/* level-0 global eigenvalues (2 ne), zero mode = 0 */
  SIPG_TAB_COARSE_S = 14,  /* level-0 global eigenvectors (2ne x 2ne)          */
  SIPG_TAB_SUB_LAM_EO = 15,/* the pairs of (L_s, M_s) split by the reversal     */
  SIPG_TAB_SUB_S_EO = 16   /* a -> m-1-a: m - m/2 even then m/2 odd (m, m x m) */
} sipg_table;

/* Copies table `which` of direction dir (0..2) on level `level` into the HOST
 * array out (row-major), at most cap values; *count receives the table size.
 * Computed on the host from *p alone. */
int sipg_host_table(const sipg_params *p, int level, int dir, int which, double *out,
                    int cap, int *count);

#ifdef __cplusplus
}
#endif

#endif /* SIPG_MG_H */
