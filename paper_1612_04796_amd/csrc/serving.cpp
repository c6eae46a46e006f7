// Serving loop: continuous batching of heterogeneous Poisson solves.
//
// Requests (any mesh, order and aspect ratio) enter a FIFO queue.  A request
// is admitted when an active slot is free and its device footprint (context
// plus solution and right-hand side) fits the memory budget; it then gets its
// own context (hierarchy, tables, Krylov vectors resident in HBM), its own
// stream and a HIP-graph-captured preconditioner V-cycle.  The loop is
// event driven: each active request has at most one flexible-CG step in
// flight, followed by an event; whenever a request's event has completed the
// loop reads its scalars, decides (converged / breakdown / next step) and
// enqueues the next step at once.  Requests therefore never wait for one
// another: small solves finish while large ones are still running, their
// kernels overlap on the device, and new requests are admitted as slots and
// memory free up.  Each request's kernel sequence is exactly the one of
// sipg_pcg_solve, so its result does not depend on what else is running.
//
// Same-order batching: the requests that become ready for a flexible-CG
// iteration in the same pass are grouped by order, operator launch shape and
// size class (unknowns within a factor of 8).  A group of two or more runs
// its preconditioners on the members' own streams, then one operator launch
// q = A p over all members (launch_apply_segments, each member's workgroups
// computing exactly what its own launch would) on a stream of the key that
// waits for every member, followed by the members' remaining steps (one
// launch per kernel for all of them) on that stream.  Within such a group,
// members whose preconditioners have the same signature (precision, orders,
// subdomain shapes, smoothing counts) run their V-cycles as one cohort on
// that stream: level by level, the local solves and the assembly of all of
// them in one launch each, the other steps per member.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "sipg_mg.h"
#include "solver_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

enum Phase { PH_START = 0, PH_ITER = 1, PH_CONFIRM = 2 };

// batching key: order (nodes per direction), elements per operator
// workgroup, size class (unknowns in [8^k, 8^(k+1))), precision of the
// operator's input p (1: single)
using BatchKey = std::tuple<int, int, int, int>;

struct Request {
  int64_t id = 0;
  sipg_params prm{};
  std::vector<int32_t> k;
  std::vector<double> phi, amp;
  double rtol = 1e-10;
  int maxit = 100;
  int state = SIPG_REQ_QUEUED;
  int phase = PH_START;
  sipg_ctx *ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  double *x = nullptr, *b = nullptr;
  size_t bytes = 0;
  int64_t ndof = 0;
  int iters = 0;
  double r0 = 0.0, relres = 1.0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::string err;
};

}  // namespace

struct sipg_server {
  size_t budget = 0, used = 0;
  int max_active = 1;
  bool fuse = true;
  // cohorts of equal preconditioner signature within a batched group run
  // their V-cycles together (segmented local solves and assemblies)
  bool fuse_smooth = true;
  // launch shapes of admitted contexts: 0 built-in, 1 the process-wide
  // tuning cache, 2 autotuned at admission (cached shapes without timing);
  // set at creation (1 when a tuning cache file is configured)
  int tune = 0;
  int64_t smooth_cycles = 0, smooth_requests = 0;
  // captured cohort V-cycles by member contexts (in cohort order); an entry
  // is dropped when one of its members leaves.  A null graph: capture failed,
  // launched directly.
  std::map<std::vector<sipg_ctx *>, hipGraphExec_t> cohort_graphs;
  // per batching key: the stream of its batched launches and joins (created
  // on first use; one per key, so cohorts of different keys never wait for
  // each other)
  std::map<BatchKey, hipStream_t> fuse_streams;
  int64_t fused_launches = 0, fused_requests = 0;
  Clock::time_point t0 = Clock::now();
  int64_t next_id = 1;
  std::deque<Request *> queue;
  std::vector<Request *> active;
  std::map<int64_t, std::unique_ptr<Request>> all;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

int fail(int code, const std::string &msg) {
  sipg::detail::set_error(msg);
  return code;
}

// Memory is accounted by reservation: an admitted request reserves its
// footprint estimate plus its two vectors (r->bytes); the solution vector stays
// reserved until it is fetched.
void unreserve(sipg_server *s, size_t b) {
  b = std::min(b, s->used);
  s->used -= b;
}

// drops the captured cohort V-cycles that use the context (their launches
// completed before the member's last step event)
void drop_cohort_graphs(sipg_server *s, const sipg_ctx *c) {
  for (auto it = s->cohort_graphs.begin(); it != s->cohort_graphs.end();) {
    if (std::find(it->first.begin(), it->first.end(), c) != it->first.end()) {
      if (it->second) (void)hipGraphExecDestroy(it->second);
      it = s->cohort_graphs.erase(it);
    } else {
      ++it;
    }
  }
}

void release_compute(sipg_server *s, Request *r) {
  if (r->ctx) {
    drop_cohort_graphs(s, r->ctx);
    sipg_destroy(r->ctx);
    r->ctx = nullptr;
  }
  if (r->b) {
    (void)hipFree(r->b);
    r->b = nullptr;
  }
  if (r->bytes) {
    const size_t keep = r->x ? (size_t)r->ndof * sizeof(double) : 0;
    unreserve(s, r->bytes - keep);
    r->bytes = keep;
  }
  if (r->ev) {
    (void)hipEventDestroy(r->ev);
    r->ev = nullptr;
  }
  if (r->stream) {
    (void)hipStreamDestroy(r->stream);
    r->stream = nullptr;
  }
}

void release_all(sipg_server *s, Request *r) {
  release_compute(s, r);
  if (r->x) {
    (void)hipFree(r->x);
    r->x = nullptr;
  }
  unreserve(s, r->bytes);
  r->bytes = 0;
}

void finish(sipg_server *s, Request *r, int state, const std::string &err = "") {
  r->state = state;
  r->t_done = s->now();
  r->err = err;
  if (state == SIPG_REQ_DONE) release_compute(s, r);
  else release_all(s, r);
}

// Admits the request: context, stream, vectors, right-hand side, first step.
bool admit(sipg_server *s, Request *r) {
  size_t fp = 0;
  if (sipg_footprint(&r->prm, &fp) != SIPG_OK) {
    finish(s, r, SIPG_REQ_FAILED, sipg_last_error());
    return true;
  }
  int64_t E = (int64_t)r->prm.ne[0] * r->prm.ne[1] * r->prm.ne[2];
  int64_t n = r->prm.P + 1;
  r->ndof = E * n * n * n;
  const size_t need = fp + 2 * (size_t)r->ndof * sizeof(double);
  if (s->used + need > s->budget) return false;  // wait for memory
  s->used += need;
  r->bytes = need;
  r->t_admit = s->now();
  if (hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
    finish(s, r, SIPG_REQ_FAILED, "stream or event creation failed");
    return true;
  }
  if (sipg_setup(&r->prm, r->stream, &r->ctx) != SIPG_OK) {
    finish(s, r, SIPG_REQ_FAILED, sipg_last_error());
    return true;
  }
  if (s->tune == 2) {
    if (sipg_autotune(r->ctx, 3) != SIPG_OK) {
      finish(s, r, SIPG_REQ_FAILED, sipg_last_error());
      return true;
    }
  } else if (s->tune == 1) {
    sipg::detail::apply_cached_tuning(r->ctx);
  }
  if (hipMalloc(&r->x, r->ndof * sizeof(double)) != hipSuccess) {
    finish(s, r, SIPG_REQ_FAILED, "out of device memory");
    return true;
  }
  if (hipMalloc(&r->b, r->ndof * sizeof(double)) != hipSuccess) {
    finish(s, r, SIPG_REQ_FAILED, "out of device memory");
    return true;
  }
  if (sipg_rhs_fourier(r->ctx, (int)r->amp.size(), r->k.data(), r->phi.data(), r->amp.data(), r->b) != SIPG_OK) {
    finish(s, r, SIPG_REQ_FAILED, sipg_last_error());
    return true;
  }
  sipg::detail::enable_graph(r->ctx, true);
  // x = 0 (a fill kernel on the request's stream)
  if (sipg::launch_fill<double>(r->x, r->ndof, 0.0, r->stream) != hipSuccess) {
    finish(s, r, SIPG_REQ_FAILED, "fill failed");
    return true;
  }
  sipg::detail::fcg_start(r->ctx, r->x, r->b);
  (void)hipEventRecord(r->ev, r->stream);
  r->state = SIPG_REQ_ACTIVE;
  r->phase = PH_START;
  s->active.push_back(r);
  return true;
}

enum Advance { ADV_LEFT = 0, ADV_STEPPED = 1, ADV_ITERATE = 2 };

// The request's last step has completed: decide and enqueue the next one.
// ADV_LEFT: the request left the active set; ADV_ITERATE: it needs a plain
// flexible-CG iteration, which the caller enqueues (alone or batched).
int advance(sipg_server *s, Request *r) {
  const double *hs = sipg::detail::host_scalars(r->ctx);
  try {
    if (r->phase == PH_START) {
      r->r0 = std::sqrt(hs[2]);
      if (!std::isfinite(r->r0)) {
        finish(s, r, SIPG_REQ_FAILED, "initial residual is not finite");
        return ADV_LEFT;
      }
      if (r->r0 == 0.0) {
        r->relres = 0.0;
        finish(s, r, SIPG_REQ_DONE);
        return ADV_LEFT;
      }
      sipg::detail::fcg_first_precond(r->ctx);
      sipg::detail::fcg_apply_update(r->ctx);
      r->iters = 1;
      r->phase = PH_ITER;
    } else if (r->phase == PH_ITER) {
      const double pq = hs[1], rn = std::sqrt(hs[2]);
      if (!(pq > 0.0) || !std::isfinite(pq)) {
        finish(s, r, SIPG_REQ_FAILED, "flexible CG breakdown");
        return ADV_LEFT;
      }
      if (!std::isfinite(rn)) {
        finish(s, r, SIPG_REQ_FAILED, "residual norm is not finite");
        return ADV_LEFT;
      }
      r->relres = rn / r->r0;
      if (rn <= r->rtol * r->r0) {
        sipg::detail::fcg_confirm(r->ctx, r->x);
        r->phase = PH_CONFIRM;
      } else if (r->iters >= r->maxit) {
        finish(s, r, SIPG_REQ_FAILED, "tolerance not reached");
        return ADV_LEFT;
      } else {
        return ADV_ITERATE;
      }
    } else {  // PH_CONFIRM
      const double rt = std::sqrt(hs[2]);
      if (rt <= r->rtol * r->r0) {
        r->relres = rt / r->r0;
        finish(s, r, SIPG_REQ_DONE);
        return ADV_LEFT;
      }
      if (r->iters >= r->maxit) {
        finish(s, r, SIPG_REQ_FAILED, "tolerance not reached");
        return ADV_LEFT;
      }
      sipg::detail::fcg_restart_from_true(r->ctx);
      sipg::detail::fcg_precond_update(r->ctx, r->x);
      sipg::detail::fcg_apply_update(r->ctx);
      r->iters += 1;
      r->phase = PH_ITER;
    }
  } catch (const std::exception &e) {
    finish(s, r, SIPG_REQ_FAILED, e.what());
    return ADV_LEFT;
  }
  if (hipEventRecord(r->ev, r->stream) != hipSuccess) {
    finish(s, r, SIPG_REQ_FAILED, "event record failed");
    return ADV_LEFT;
  }
  return ADV_STEPPED;
}

// One plain iteration of a request on its own stream.
bool iterate_alone(sipg_server *s, Request *r) {
  try {
    sipg::detail::fcg_precond_update(r->ctx, r->x);
    sipg::detail::fcg_apply_update(r->ctx);
  } catch (const std::exception &e) {
    finish(s, r, SIPG_REQ_FAILED, e.what());
    return false;
  }
  r->iters += 1;
  if (hipEventRecord(r->ev, r->stream) != hipSuccess) {
    finish(s, r, SIPG_REQ_FAILED, "event record failed");
    return false;
  }
  return true;
}

// One iteration of every member of a group with one operator launch; on a
// failure the members not yet enqueued fall back to iterate_alone.  Returns
// the members that left the active set.
std::vector<Request *> iterate_batched(sipg_server *s, hipStream_t fs, const std::vector<Request *> &g,
                                       const std::vector<sipg::ApplyLaunch<double>> &a) {
  std::vector<Request *> left;
  bool ok = true;
  try {
    // members of equal preconditioner signature: one cohort V-cycle on fs
    std::map<std::vector<int>, std::vector<Request *>> cohorts;
    for (Request *r : g) {
      std::vector<int> sig;
      if (s->fuse_smooth) sig = sipg::detail::precond_signature(r->ctx);
      cohorts[sig].push_back(r);
    }
    for (auto &kv : cohorts) {
      const std::vector<Request *> &m = kv.second;
      if (kv.first.empty() || m.size() < 2) {
        for (Request *r : m) {
          sipg::detail::fcg_precond_update(r->ctx, r->x);
          ok = ok && hipEventRecord(r->ev, r->stream) == hipSuccess &&
               hipStreamWaitEvent(fs, r->ev, 0) == hipSuccess;
        }
        continue;
      }
      std::vector<sipg_ctx *> cs;
      std::vector<double *> xs;
      for (Request *r : m) {
        ok = ok && hipStreamWaitEvent(fs, r->ev, 0) == hipSuccess;
        cs.push_back(r->ctx);
        xs.push_back(r->x);
      }
      auto git = s->cohort_graphs.find(cs);
      if (git == s->cohort_graphs.end()) {
        if (s->cohort_graphs.size() >= 64) {  // bounded: start over
          for (auto &kv2 : s->cohort_graphs)
            if (kv2.second) (void)hipGraphExecDestroy(kv2.second);
          s->cohort_graphs.clear();
        }
        git = s->cohort_graphs.emplace(cs, sipg::detail::capture_cohort_precond(cs.data(), (int)cs.size(), fs)).first;
      }
      sipg::detail::fcg_precond_update_cohort(cs.data(), xs.data(), (int)cs.size(), fs, git->second);
      s->smooth_cycles += 1;
      s->smooth_requests += (int64_t)cs.size();
    }
    ok = ok && sipg::launch_apply_segments<double>(a.data(), (int)a.size(), fs) == hipSuccess;
    if (ok) {
      std::vector<sipg_ctx *> cs;
      for (Request *r : g) cs.push_back(r->ctx);
      sipg::detail::fcg_after_apply_batched(cs.data(), (int)cs.size(), fs);
    }
  } catch (const std::exception &e) {
    sipg::detail::set_error(e.what());
    ok = false;
  }
  for (Request *r : g) {
    if (!ok) {
      finish(s, r, SIPG_REQ_FAILED, "batched operator launch failed: " + sipg::detail::last_error());
      left.push_back(r);
      continue;
    }
    r->iters += 1;
    if (hipEventRecord(r->ev, fs) != hipSuccess) {
      finish(s, r, SIPG_REQ_FAILED, "event record failed");
      left.push_back(r);
    }
  }
  if (ok) {
    s->fused_launches += 1;
    s->fused_requests += (int64_t)g.size();
  }
  return left;
}

// The batching key of a request and its operator launch; false when its
// operator cannot be batched or batching is off.
bool batch_key(sipg_server *s, Request *r, BatchKey *key, sipg::ApplyLaunch<double> *a) {
  if (!s->fuse || !sipg::detail::fcg_apply_launch(r->ctx, a)) return false;
  int cls = 0;
  while ((r->ndof >> (3 * (cls + 1))) > 0) ++cls;
  *key = std::make_tuple(a->n, a->epb, cls, a->u32 ? 1 : 0);
  return true;
}

// the stream of a batching key (nullptr if it cannot be created)
hipStream_t key_stream(sipg_server *s, const BatchKey &key) {
  auto it = s->fuse_streams.find(key);
  if (it != s->fuse_streams.end()) return it->second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
  s->fuse_streams[key] = st;
  return st;
}

// Keeps batchable requests that stepped in the same pass in phase: each one's
// step-complete event is re-recorded on its key's stream after all of their
// steps, so they become ready together and their next iterations batch.
void join_cohorts(sipg_server *s, const std::vector<Request *> &stepped) {
  std::map<BatchKey, std::vector<Request *>> groups;
  for (Request *r : stepped) {
    BatchKey key;
    sipg::ApplyLaunch<double> a{};
    if (r->state == SIPG_REQ_ACTIVE && batch_key(s, r, &key, &a)) groups[key].push_back(r);
  }
  for (auto &kv : groups) {
    const std::vector<Request *> &g = kv.second;
    if (g.size() < 2) continue;
    hipStream_t fs = key_stream(s, kv.first);
    if (!fs) continue;
    for (Request *r : g) (void)hipStreamWaitEvent(fs, r->ev, 0);
    for (Request *r : g) (void)hipEventRecord(r->ev, fs);
  }
}

// Enqueues the plain iterations: batched where two or more requests share a
// key, alone otherwise.  Returns the requests that left the active set.
std::vector<Request *> iterate(sipg_server *s, const std::vector<Request *> &ready) {
  std::vector<Request *> left;
  std::map<BatchKey, std::vector<std::pair<Request *, sipg::ApplyLaunch<double>>>> groups;
  for (Request *r : ready) {
    sipg::ApplyLaunch<double> a{};
    BatchKey key;
    if (batch_key(s, r, &key, &a)) {
      groups[key].push_back({r, a});
    } else if (!iterate_alone(s, r)) {
      left.push_back(r);
    }
  }
  for (auto &kv : groups) {
    auto &v = kv.second;
    for (size_t i0 = 0; i0 < v.size(); i0 += sipg::kMaxApplySegments) {
      const size_t i1 = std::min(v.size(), i0 + sipg::kMaxApplySegments);
      hipStream_t fs = i1 - i0 > 1 ? key_stream(s, kv.first) : nullptr;
      if (!fs) {
        for (size_t i = i0; i < i1; ++i)
          if (!iterate_alone(s, v[i].first)) left.push_back(v[i].first);
        continue;
      }
      std::vector<Request *> g;
      std::vector<sipg::ApplyLaunch<double>> a;
      for (size_t i = i0; i < i1; ++i) {
        g.push_back(v[i].first);
        a.push_back(v[i].second);
      }
      for (Request *r : iterate_batched(s, fs, g, a)) left.push_back(r);
    }
  }
  return left;
}

}  // namespace

extern "C" {

int sipg_server_create(size_t memory_budget, int max_active, sipg_server **out) {
  if (!out || memory_budget == 0 || max_active < 1) return fail(SIPG_EINVAL, "need budget > 0 and max_active >= 1");
  sipg_server *s = new (std::nothrow) sipg_server();
  if (!s) return fail(SIPG_ENOMEM, "host allocation failed");
  s->budget = memory_budget;
  s->max_active = max_active;
  // a tuning cache saved earlier (a missing or unreadable file is ignored:
  // the requests then run with the built-in shapes)
  if (const char *path = std::getenv("SIPG_TUNING_CACHE")) {
    (void)sipg_tuning_cache_load(path, nullptr);
    s->tune = 1;
  }
  *out = s;
  return SIPG_OK;
}

int sipg_server_submit(sipg_server *s, const sipg_params *p, int nmodes, const int32_t *k, const double *phi,
                       const double *amp, double rtol, int maxit, int64_t *id) {
  if (!s || !p || !k || !phi || !amp || !id) return fail(SIPG_EINVAL, "null argument");
  if (nmodes < 1 || nmodes > 64) return fail(SIPG_EINVAL, "nmodes must be in 1..64");
  if (!(rtol > 0.0) || maxit < 1) return fail(SIPG_EINVAL, "need rtol > 0 and maxit >= 1");
  size_t fp = 0;
  int rc = sipg_footprint(p, &fp);  // validates the parameters
  if (rc != SIPG_OK) return rc;
  // a request that could never be admitted would block the FIFO for good
  const int64_t n = (int64_t)p->P + 1;
  const size_t need = fp + 2 * (size_t)((int64_t)p->ne[0] * p->ne[1] * p->ne[2] * n * n * n) * sizeof(double);
  if (need > s->budget)
    return fail(SIPG_ENOMEM, "request needs " + std::to_string(need) + " device bytes, more than the server's budget of " +
                                 std::to_string(s->budget));
  auto r = std::make_unique<Request>();
  r->id = s->next_id++;
  r->prm = *p;
  r->k.assign(k, k + 3 * nmodes);
  r->phi.assign(phi, phi + 3 * nmodes);
  r->amp.assign(amp, amp + nmodes);
  r->rtol = rtol;
  r->maxit = maxit;
  r->t_submit = s->now();
  *id = r->id;
  s->queue.push_back(r.get());
  s->all[r->id] = std::move(r);
  return SIPG_OK;
}

int sipg_server_progress(sipg_server *s, int wait_ms, int *nactive, int *nqueued, int *ncompleted) {
  if (!s) return fail(SIPG_EINVAL, "null server");
  int done = 0;
  const double deadline = s->now() + std::max(0, wait_ms) * 1e-3;
  for (;;) {
    // admission, first come first served, while slots and memory allow
    std::vector<Request *> stepped;
    while (!s->queue.empty() && (int)s->active.size() < s->max_active) {
      Request *r = s->queue.front();
      if (!admit(s, r)) break;
      s->queue.pop_front();
      if (r->state != SIPG_REQ_ACTIVE) ++done;
      else stepped.push_back(r);
    }
    // advance every request whose step has completed; plain iterations are
    // collected and enqueued together (batched where they share an order)
    std::vector<Request *> ready;
    for (size_t i = 0; i < s->active.size();) {
      Request *r = s->active[i];
      const hipError_t q = hipEventQuery(r->ev);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      const int a = (q == hipSuccess) ? advance(s, r) : (finish(s, r, SIPG_REQ_FAILED, hipGetErrorString(q)), ADV_LEFT);
      if (a == ADV_LEFT) {
        ++done;
        s->active.erase(s->active.begin() + i);
      } else {
        if (a == ADV_ITERATE) ready.push_back(r);
        else stepped.push_back(r);
        ++i;
      }
    }
    if (!ready.empty()) {
      const std::vector<Request *> left = iterate(s, ready);
      for (Request *r : left) {
        ++done;
        s->active.erase(std::find(s->active.begin(), s->active.end(), r));
      }
      for (Request *r : ready)
        if (std::find(left.begin(), left.end(), r) == left.end()) stepped.push_back(r);
    }
    join_cohorts(s, stepped);
    if (done > 0 || s->now() >= deadline || (s->active.empty() && s->queue.empty())) break;
    std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  if (nactive) *nactive = (int)s->active.size();
  if (nqueued) *nqueued = (int)s->queue.size();
  if (ncompleted) *ncompleted = done;
  return SIPG_OK;
}

int sipg_server_status(sipg_server *s, int64_t id, int *state, int *iters, double *relres, double times[3],
                       int64_t *ndof) {
  if (!s) return fail(SIPG_EINVAL, "null server");
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(SIPG_EINVAL, "unknown request id");
  const Request *r = it->second.get();
  if (state) *state = r->state;
  if (iters) *iters = r->iters;
  if (relres) *relres = r->relres;
  if (times) {
    times[0] = r->t_submit;
    times[1] = r->t_admit;
    times[2] = r->t_done;
  }
  if (ndof) {
    const int64_t E = (int64_t)r->prm.ne[0] * r->prm.ne[1] * r->prm.ne[2];
    const int64_t n = r->prm.P + 1;
    *ndof = E * n * n * n;
  }
  if (r->state == SIPG_REQ_FAILED) sipg::detail::set_error(r->err);
  return SIPG_OK;
}

int sipg_server_fetch(sipg_server *s, int64_t id, double *u, void *hip_stream) {
  if (!s || !u) return fail(SIPG_EINVAL, "null argument");
  auto it = s->all.find(id);
  if (it == s->all.end()) return fail(SIPG_EINVAL, "unknown request id");
  Request *r = it->second.get();
  if (r->state != SIPG_REQ_DONE || !r->x) return fail(SIPG_EINVAL, "request has no result");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (hipMemcpyAsync(u, r->x, r->ndof * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(SIPG_EHIP, "result copy failed");
  release_all(s, r);
  return SIPG_OK;
}

int sipg_server_set_option(sipg_server *s, int option, int value) {
  if (!s) return fail(SIPG_EINVAL, "null server");
  if (option == SIPG_SERVER_FUSE_APPLY) {
    s->fuse = value != 0;
  } else if (option == SIPG_SERVER_FUSE_SMOOTH) {
    s->fuse_smooth = value != 0;
  } else if (option == SIPG_SERVER_TUNE) {
    if (value < 0 || value > 2) return fail(SIPG_EINVAL, "tuning mode must be 0, 1 or 2");
    s->tune = value;
  } else {
    return fail(SIPG_EINVAL, "unknown server option");
  }
  return SIPG_OK;
}

int sipg_server_smooth_stats(const sipg_server *s, int64_t *cohort_cycles, int64_t *cohort_requests) {
  if (!s) return fail(SIPG_EINVAL, "null server");
  if (cohort_cycles) *cohort_cycles = s->smooth_cycles;
  if (cohort_requests) *cohort_requests = s->smooth_requests;
  return SIPG_OK;
}

int sipg_server_stats(const sipg_server *s, int64_t *fused_launches, int64_t *fused_requests) {
  if (!s) return fail(SIPG_EINVAL, "null server");
  if (fused_launches) *fused_launches = s->fused_launches;
  if (fused_requests) *fused_requests = s->fused_requests;
  return SIPG_OK;
}

int sipg_server_destroy(sipg_server *s) {
  if (!s) return SIPG_OK;
  (void)hipDeviceSynchronize();
  for (auto &kv : s->all) release_all(s, kv.second.get());
  for (auto &kv : s->cohort_graphs)
    if (kv.second) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : s->fuse_streams) (void)hipStreamDestroy(kv.second);
  // shapes timed at admission are kept for later processes
  if (s->tune == 2)
    if (const char *path = std::getenv("SIPG_TUNING_CACHE")) (void)sipg_tuning_cache_save(path);
  delete s;
  return SIPG_OK;
}

}  // extern "C"
