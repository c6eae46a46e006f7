// Internal interface between the solver context (sipg_api.cpp) and the serving
// loop (serving.cpp).  Every fcg_* call only enqueues work on the context's
// stream; the scalars it produces are written by its last reduction kernel
// to the context's pinned, device-mapped host mirror (indices FcgScalar) and
// are valid once the stream has passed that point.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "kernels.h"
#include "sipg_mg.h"

namespace sipg {
namespace detail {

// b projected onto 1^perp into the context (its mean in FS_MEAN), then
// r = b - A x and ||r||^2 (FS_RR)
void fcg_start(sipg_ctx *c, double *x, const double *b);
// z = B r, rz = r.z, p = z
void fcg_first_precond(sipg_ctx *c);
// q = A p, p.q (FS_PQ), r -= alpha q, ||r||^2 (FS_RR); the update
// x += alpha p is deferred to the next call that is given x
void fcg_apply_update(sipg_ctx *c);
// fcg_apply_update in two parts, for launching the operators of several
// contexts together: the operator launch q = A p with its p.q partial sums
// (returned as a launch description; false when the order has no
// compile-time operator kernel), then the rest of the step enqueued on
// stream st (p.q, r -= alpha q, ||r||^2).  fcg_apply_launch(c, &a) followed
// by launch_apply_segments over such descriptions and fcg_after_apply(c, st)
// computes exactly what fcg_apply_update does.
bool fcg_apply_launch(sipg_ctx *c, sipg::ApplyLaunch<double> *a);
void fcg_after_apply(sipg_ctx *c, hipStream_t st);
// fcg_after_apply of k contexts (k <= kMaxApplySegments) with one launch per
// kernel instead of one per context
void fcg_after_apply_batched(sipg_ctx *const *cs, int k, hipStream_t st);
// x += alpha p if pending, x -= mean(x), then ||b - A x||^2 (FS_RR) with the
// projected b of fcg_start, the true residual kept in q
void fcg_confirm(sipg_ctx *c, double *x);
// r = true residual, q = A p again
void fcg_restart_from_true(sipg_ctx *c);
// z = B r, beta = -alpha (z.q) / rz, rz = r.z, x += alpha p if pending, p = z + beta p
void fcg_precond_update(sipg_ctx *c, double *x);

// The preconditioner signature of a context: contexts with equal, non-empty
// signatures (same precision, level count, orders, subdomain shapes and
// smoothing counts, every level on the compile-time local-solve kernels)
// can run their V-cycles as one cohort.  Empty when the context cannot.
std::vector<int> precond_signature(const sipg_ctx *c);
// fcg_precond_update of k <= kMaxApplySegments contexts with equal
// signatures, all enqueued on stream st: the V-cycles level by level, each
// step of all k in one segmented launch (local solves, assemblies,
// residuals, restrictions, prolongations; the coarse solves per context),
// then every context's CG update.  Each context computes exactly what
// fcg_precond_update computes for it.  graph: the V-cycles captured earlier
// by capture_cohort_precond for the same contexts in the same order (null:
// launched directly).
void fcg_precond_update_cohort(sipg_ctx *const *cs, double *const *xs, int k, hipStream_t st,
                               hipGraphExec_t graph);
// The cohort's V-cycles captured into an executable graph on stream st
// (null when the capture fails; nothing is left enqueued then).
hipGraphExec_t capture_cohort_precond(sipg_ctx *const *cs, int k, hipStream_t st);
// Takes the launch shapes the process-wide tuning cache holds for the
// context's levels (no timing); returns how many levels took one.
int apply_cached_tuning(sipg_ctx *c);

const double *host_scalars(const sipg_ctx *c);
hipStream_t ctx_stream(const sipg_ctx *c);
void enable_graph(sipg_ctx *c, bool on);
int64_t ctx_ndof(const sipg_ctx *c);
size_t ctx_bytes(const sipg_ctx *c);
std::string last_error();
void set_error(const std::string &m);

}  // namespace detail
}  // namespace sipg
