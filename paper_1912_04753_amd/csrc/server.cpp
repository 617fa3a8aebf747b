// Request server of the ripk C ABI: continuous batching of K / envelope
// requests of uneven size on one device.
//
// A server owns `slots` worker threads.  Each slot has its own HIP stream
// (non-blocking, default priority) and keeps one device workspace (a plan
// sized by capacities) that it rebinds to every request it can hold.
//
// Admission (ripk_server_desc.admission) is first come first served, or by
// size: each request's work is estimated at submit as (m + 1) (n^2 f + 64 n),
// f the share of a uniform set's ordered pairs within the thresholds (about
// the in-range pairs of the observed set and each CSR simulation).  Requests
// above large_work are large; a free slot takes a request that has waited
// longer than age_ms first (oldest first), then the oldest large request while
// fewer than max_large run, then the smallest waiting request that is not
// large, so that small requests do not queue behind large ones.  A request is
// admitted by an idle slot when its device footprint fits the server's HBM
// budget: the slot's own workspace if large enough, else a grown one, after
// releasing idle slots' workspaces when the budget is short (freed outside
// the lock).
//
// Admitted requests run concurrently on their slots' streams.  A persistent
// pair kernel holds every compute unit it gets until it ends; with
// device_share < 1 a pair launch keeps that share of its workgroups while
// more than one slot is busy (a count in host memory that the kernel reads),
// leaving the rest to the other streams, and with slice_ms long pair launches
// are cut into slices, so that the other requests' kernels start between
// them and the share is taken afresh.
// Each request is an observed K (Eq. 2-4) plus, when m > 0, its m CSR
// simulations and envelopes (Sec. 3); results are exact integer sums, so they
// are the same whatever else shares the device.
#include <hip/hip_runtime.h>
#include <time.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/ripk.h"
#include "ripk_internal.h"

using namespace ripk;

namespace {

constexpr int kMaxSlots = 16;
constexpr double kLargeWorkDefault = 2e10;  // pair evaluations of a large request (~30 ms)

double mono_now() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

struct Request {
  uint64_t ticket = 0;
  ripk_plan_desc desc{};
  Caps caps{};
  int64_t n = 0, n_centres = 0;
  double work = 0;  // estimated pair evaluations (admission order)
  int32_t m = 0;
  uint32_t flags = 0;
  uint64_t seed = 0;
  std::vector<int32_t> xyt;  // x | y | t, n each
  std::vector<int32_t> poly; // the descriptor's polygon (desc.poly points here)
  std::vector<double> lam;   // intensities (inhomogeneous plans)
  // results
  bool done = false;
  ripk_status status = RIPK_PENDING;
  std::string msg;
  int32_t slot = -1;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int64_t n_in = 0;
  std::vector<uint64_t> C, C_sims;
  std::vector<double> W, K, L, env, W_sims, K_sims;
};

struct Slot {
  std::thread th;
  hipStream_t stream = nullptr;
  ripk_plan_s *plan = nullptr;
  int64_t bytes = 0;           // device bytes of `plan`
  bool busy = false;
  uint64_t seen_epoch = 0;
  int32_t *stage = nullptr;    // pinned host staging for points
  int64_t stage_cap = 0;       // int32 elements
};

}  // namespace

struct ripk_server_s {
  ripk_server_desc desc{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  uint64_t epoch = 1;  // bumped on every submit and completion
  int64_t used = 0;    // device bytes held by slot workspaces
  bool stop = false;
  int32_t *busy_word = nullptr;  // busy slots, in host memory the pair kernels read
  int busy = 0;
  int large_running = 0;
  Slot slots[kMaxSlots];
};

namespace {

bool is_large(const ripk_server_s *sv, const Request *r) {
  const double lw = sv->desc.large_work > 0 ? sv->desc.large_work : kLargeWorkDefault;
  return sv->desc.admission == RIPK_ADMIT_SIZE && r->work > lw;
}

// The next request for a free slot (see the admission orders above).
std::deque<Request *>::iterator pick(ripk_server_s *sv) {
  if (sv->desc.admission != RIPK_ADMIT_SIZE) return sv->queue.begin();
  const double now = mono_now();
  const double age = sv->desc.age_ms * 1e-3;
  auto best = sv->queue.end(), large = sv->queue.end();
  for (auto it = sv->queue.begin(); it != sv->queue.end(); ++it) {
    if (age > 0 && now - (*it)->t_submit > age) return it;  // queue order: the oldest
    if (is_large(sv, *it)) {
      if (large == sv->queue.end()) large = it;
      continue;
    }
    if (best == sv->queue.end() || (*it)->work < (*best)->work) best = it;
  }
  if (large != sv->queue.end() &&
      (sv->desc.max_large <= 0 || sv->large_running < sv->desc.max_large))
    return large;
  return best;
}

// Picks a request for slot k if its footprint fits; sets *target to the
// capacities the slot must (re)allocate, or leaves it empty for reuse.  Called
// with the server lock held; idle slots' workspaces that must go to make room
// are detached into *release (freed by the caller without the lock).
Request *try_admit(ripk_server_s *sv, int k, Caps *target, bool *realloc,
                   std::vector<ripk_plan_s *> *release) {
  if (sv->queue.empty()) return nullptr;
  Slot &me = sv->slots[k];
  const auto it = pick(sv);
  if (it == sv->queue.end()) return nullptr;
  Request *r = *it;
  *realloc = false;
  if (me.plan && caps_fit(plan_caps(me.plan), r->caps)) {
    sv->queue.erase(it);
    return r;
  }
  const int64_t budget = sv->desc.hbm_budget_bytes;
  int64_t others = sv->used - me.bytes;
  if (me.plan) {
    const Caps grow = caps_max(plan_caps(me.plan), r->caps);
    if (others + caps_bytes(grow) <= budget) {
      *target = grow;
      *realloc = true;
      sv->queue.erase(it);
      return r;
    }
  }
  if (others + caps_bytes(r->caps) > budget) {
    // release idle slots' workspaces (no work of theirs is in flight)
    for (int j = 0; j < sv->desc.slots; ++j) {
      Slot &o = sv->slots[j];
      if (j == k || o.busy || !o.plan) continue;
      release->push_back(o.plan);
      o.plan = nullptr;
      sv->used -= o.bytes;
      o.bytes = 0;
    }
    others = sv->used - me.bytes;
    if (others + caps_bytes(r->caps) > budget) return nullptr;  // wait for a running request
  }
  *target = r->caps;
  *realloc = true;
  sv->queue.erase(it);
  return r;
}

ripk_status ensure_stage(Slot &s, int64_t elems) {
  if (s.stage_cap >= elems) return RIPK_OK;
  if (s.stage) (void)hipHostFree(s.stage);
  s.stage = nullptr;
  s.stage_cap = 0;
  const int64_t cap = std::max<int64_t>(elems, 3 << 16);
  if (hipHostMalloc((void **)&s.stage, sizeof(int32_t) * cap, hipHostMallocDefault) != hipSuccess) {
    s.stage = nullptr;
    return set_error(RIPK_ENOMEM, "pinned staging allocation failed");
  }
  s.stage_cap = cap;
  return RIPK_OK;
}

// Evaluates one admitted request on slot s (no server lock held).
ripk_status run_request(Slot &s, Request *r) {
  ripk_status st = plan_bind(s.plan, &r->desc, s.stream);
  if (st != RIPK_OK) return st;
  const int64_t n = r->n;
  st = ensure_stage(s, 3 * n);
  if (st != RIPK_OK) return st;
  std::copy(r->xyt.begin(), r->xyt.end(), s.stage);
  const size_t NB = (size_t)r->desc.n_s * (size_t)r->desc.n_t;
  r->C.assign(NB, 0);
  r->W.assign(NB, 0.0);
  r->K.assign(NB, 0.0);
  r->L.assign(NB, 0.0);
  ripk_points pts{s.stage, s.stage + n, s.stage + 2 * n, n, r->n_centres, 0,
                  r->lam.empty() ? nullptr : r->lam.data()};
  ripk_K_out ko{r->C.data(), r->W.data(), r->K.data(), r->L.data()};
  // CSR simulations of every point (or of two types): the observed set and
  // the simulations in one launch
  const bool one_launch =
      r->m > 0 && r->desc.sim_method == RIPK_SIM_CSR &&
      ((r->desc.flags & RIPK_PLAN_CROSS) || r->n_centres == 0 || r->n_centres == n);
  ripk_stats stats;
  if (!one_launch) {
    st = ripk_compute_K(s.plan, &pts, s.stream, &ko);
    if (st != RIPK_OK) return st;
    ripk_plan_stats(s.plan, &stats);
    r->n_in = stats.n_in;
  }
  if (r->m > 0) {
    r->env.assign(5 * NB, 0.0);
    ripk_env_out eo{};
    eo.K_lo = r->env.data();
    eo.K_hi = eo.K_lo + NB;
    eo.L_lo = eo.K_hi + NB;
    eo.L_hi = eo.L_lo + NB;
    eo.dL_hi = eo.L_hi + NB;
    if (r->flags & RIPK_REQ_KEEP_SIMS) {
      r->C_sims.assign(NB * r->m, 0);
      r->W_sims.assign(NB * r->m, 0.0);
      r->K_sims.assign(NB * r->m, 0.0);
      eo.C_sims = r->C_sims.data();
      eo.W_sims = r->W_sims.data();
      eo.K_sims = r->K_sims.data();
    }
    if (one_launch) {
      st = ripk_compute_K_envelope(s.plan, &pts, r->m, r->seed, s.stream, &ko, &eo);
      if (st != RIPK_OK) return st;
      ripk_plan_stats(s.plan, &stats);
      r->n_in = stats.n_in;
    } else {
      st = ripk_simulate_envelope(s.plan, n, r->m, r->seed, r->L.data(), s.stream, &eo);
      if (st != RIPK_OK) return st;
      ripk_plan_stats(s.plan, &stats);
      r->n_in += stats.n_in;
    }
  }
  return RIPK_OK;
}

void slot_main(ripk_server_s *sv, int k) {
  Slot &me = sv->slots[k];
  (void)hipSetDevice(sv->desc.device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    sv->cv_work.wait(lk, [&] { return sv->stop || (!sv->queue.empty() && me.seen_epoch != sv->epoch); });
    if (sv->stop) break;
    me.seen_epoch = sv->epoch;
    Caps target;
    bool realloc = false;
    std::vector<ripk_plan_s *> release;
    Request *r = try_admit(sv, k, &target, &realloc, &release);
    if (!release.empty()) {
      lk.unlock();
      for (ripk_plan_s *pl : release) plan_free(pl);
      lk.lock();
    }
    if (!r) continue;
    me.busy = true;
    const bool large = is_large(sv, r);
    sv->large_running += large ? 1 : 0;
    __atomic_store_n(sv->busy_word, ++sv->busy, __ATOMIC_RELEASE);
    r->slot = k;
    r->t_admit = mono_now();
    ripk_plan_s *old = nullptr;
    if (realloc) {
      old = me.plan;
      me.plan = nullptr;
      sv->used += caps_bytes(target) - me.bytes;  // reserve before allocating
      me.bytes = caps_bytes(target);
    }
    lk.unlock();

    ripk_status st = RIPK_OK;
    if (realloc) {
      if (old) plan_free(old);
      st = plan_create(sv->desc.device, target, &me.plan);
      if (st == RIPK_OK && (sv->desc.device_share > 0.f || sv->desc.slice_ms > 0.f))
        plan_set_sharing(me.plan, sv->desc.device_share > 0.f ? sv->busy_word : nullptr,
                         sv->desc.device_share > 0.f ? sv->desc.device_share : 1.0,
                         1e3 * (double)sv->desc.slice_ms);
    }
    if (st == RIPK_OK) st = run_request(me, r);
    std::string msg = st == RIPK_OK ? std::string() : std::string(ripk_last_error());

    lk.lock();
    if (realloc && !me.plan) {
      sv->used -= me.bytes;
      me.bytes = 0;
    }
    r->status = st;
    r->msg = msg;
    r->t_done = mono_now();
    r->done = true;
    me.busy = false;
    sv->large_running -= large ? 1 : 0;
    __atomic_store_n(sv->busy_word, --sv->busy, __ATOMIC_RELEASE);
    ++sv->epoch;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

void copy_out(const Request *r, ripk_result *out) {
  const size_t NB = (size_t)r->desc.n_s * (size_t)r->desc.n_t;
  auto cp = [&](void *dst, const void *src, size_t bytes) {
    if (dst && src && bytes) std::memcpy(dst, src, bytes);
  };
  if (r->status == RIPK_OK) {
    cp(out->k.C, r->C.data(), 8 * NB);
    cp(out->k.W, r->W.data(), 8 * NB);
    cp(out->k.K, r->K.data(), 8 * NB);
    cp(out->k.L, r->L.data(), 8 * NB);
    if (r->m > 0) {
      double *rows[5] = {out->env.K_lo, out->env.K_hi, out->env.L_lo, out->env.L_hi, out->env.dL_hi};
      for (int i = 0; i < 5; ++i) cp(rows[i], r->env.data() + i * NB, 8 * NB);
      if (r->flags & RIPK_REQ_KEEP_SIMS) {
        cp(out->env.C_sims, r->C_sims.data(), 8 * NB * r->m);
        cp(out->env.W_sims, r->W_sims.data(), 8 * NB * r->m);
        cp(out->env.K_sims, r->K_sims.data(), 8 * NB * r->m);
      }
    }
  }
  out->status = r->status;
  out->slot = r->slot;
  out->t_submit = r->t_submit;
  out->t_admit = r->t_admit;
  out->t_done = r->t_done;
  out->n_in = r->n_in;
}

}  // namespace

extern "C" {

ripk_status ripk_server_create(const ripk_server_desc *desc, ripk_server_t *out) {
  if (!desc || !out) return set_error(RIPK_EINVAL, "null descriptor or output handle");
  *out = nullptr;
  if (desc->slots < 1 || desc->slots > kMaxSlots) return set_error(RIPK_EINVAL, "slots must be in [1, 16]");
  if (desc->queue_cap < 1) return set_error(RIPK_EINVAL, "queue_cap must be >= 1");
  if (desc->hbm_budget_bytes < 1) return set_error(RIPK_EINVAL, "hbm_budget_bytes must be >= 1");
  if (desc->admission > RIPK_ADMIT_SIZE) return set_error(RIPK_EINVAL, "unknown admission order");
  if (!(desc->large_work >= 0) || !(desc->age_ms >= 0) || desc->max_large < 0 ||
      !(desc->device_share >= 0.f && desc->device_share <= 1.f) || !(desc->slice_ms >= 0.f) ||
      desc->reserved != 0)
    return set_error(RIPK_EINVAL,
                     "bad admission or sharing parameters (large_work, age_ms, max_large >= 0; "
                     "device_share in [0, 1]; slice_ms >= 0; reserved 0)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return set_error(RIPK_EDEVICE, "no HIP device available");
  if (desc->device < 0 || desc->device >= ndev) return set_error(RIPK_EINVAL, "device out of range");
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(desc->device);
  ripk_server_s *sv = new ripk_server_s();
  sv->desc = *desc;
  ripk_status st = RIPK_OK;
  if (hipHostMalloc((void **)&sv->busy_word, sizeof(int32_t), hipHostMallocCoherent) != hipSuccess) {
    sv->busy_word = nullptr;
    st = set_error(RIPK_ENOMEM, "pinned allocation failed");
  } else {
    *sv->busy_word = 0;
  }
  for (int k = 0; k < desc->slots && st == RIPK_OK; ++k)
    if (hipStreamCreateWithFlags(&sv->slots[k].stream, hipStreamNonBlocking) != hipSuccess) {
      st = set_error(RIPK_EDEVICE, "stream creation failed");
      break;
    }
  (void)hipSetDevice(prev);
  if (st != RIPK_OK) {
    for (int k = 0; k < desc->slots; ++k)
      if (sv->slots[k].stream) (void)hipStreamDestroy(sv->slots[k].stream);
    if (sv->busy_word) (void)hipHostFree(sv->busy_word);
    delete sv;
    return st;
  }
  for (int k = 0; k < desc->slots; ++k) sv->slots[k].th = std::thread(slot_main, sv, k);
  *out = sv;
  return RIPK_OK;
}

void ripk_server_destroy(ripk_server_t sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    for (Request *r : sv->queue) {
      r->status = RIPK_ECANCELED;
      r->msg = "cancelled by server shutdown";
      r->done = true;
    }
    sv->queue.clear();
    sv->cv_work.notify_all();
    sv->cv_done.notify_all();
  }
  for (int k = 0; k < sv->desc.slots; ++k)
    if (sv->slots[k].th.joinable()) sv->slots[k].th.join();  // in-flight requests finish
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(sv->desc.device);
  for (int k = 0; k < sv->desc.slots; ++k) {
    Slot &s = sv->slots[k];
    if (s.plan) plan_free(s.plan);
    if (s.stage) (void)hipHostFree(s.stage);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  if (sv->busy_word) (void)hipHostFree(sv->busy_word);
  (void)hipSetDevice(prev);
  for (auto &kv : sv->all) delete kv.second;
  delete sv;
}

ripk_status ripk_submit(ripk_server_t sv, const ripk_request *req, uint64_t *ticket) {
  if (!sv || !req || !ticket) return set_error(RIPK_EINVAL, "null server, request or ticket");
  const ripk_points &p = req->pts;
  if (p.on_device) return set_error(RIPK_EINVAL, "the server takes host points (on_device = 0)");
  if (!p.x || !p.y || !p.t) return set_error(RIPK_EINVAL, "null coordinate array");
  if (p.n < 2) return set_error(RIPK_EINVAL, "need n >= 2 points");
  if (p.n_centres < 0 || p.n_centres > p.n) return set_error(RIPK_EINVAL, "n_centres must be in [0, n]");
  if (req->m < 0) return set_error(RIPK_EINVAL, "m must be >= 0");
  if (req->flags & ~RIPK_REQ_KEEP_SIMS) return set_error(RIPK_EINVAL, "unknown request flags");
  Request *r = new Request();
  r->desc = req->plan;
  r->desc.n_max = p.n;
  r->desc.m_max = req->m;
  r->desc.device = sv->desc.device;
  if (req->plan.poly_n > 0 && req->plan.poly) {
    r->poly.assign(req->plan.poly, req->plan.poly + 2 * (size_t)std::min(req->plan.poly_n, kMaxPoly));
    r->desc.poly = r->poly.data();
  }
  ripk_status st = plan_validate(&r->desc, &r->caps);
  if (st != RIPK_OK) {
    delete r;
    return st;
  }
  if (caps_bytes(r->caps) > sv->desc.hbm_budget_bytes) {
    delete r;
    return set_error(RIPK_E2BIG, "request footprint exceeds the server's HBM budget");
  }
  r->n = p.n;
  r->n_centres = p.n_centres;
  {
    // in-range share of a uniform set's ordered pairs (Sec. 3 thresholds)
    const double A = (double)(r->desc.x1 - r->desc.x0) * (double)(r->desc.y1 - r->desc.y0);
    const double D = (double)(r->desc.t1 - r->desc.t0);
    const double f = std::min(1.0, 3.141592653589793 * (double)r->desc.s_max * r->desc.s_max / A) *
                     std::min(1.0, 2.0 * (double)r->desc.t_max / D);
    r->work = (double)(req->m + 1) * ((double)p.n * (double)p.n * f + 64.0 * (double)p.n);
  }
  r->m = req->m;
  r->flags = req->flags;
  r->seed = req->seed;
  r->xyt.resize(3 * (size_t)p.n);
  std::copy(p.x, p.x + p.n, r->xyt.begin());
  std::copy(p.y, p.y + p.n, r->xyt.begin() + p.n);
  std::copy(p.t, p.t + p.n, r->xyt.begin() + 2 * p.n);
  if (p.lambda) r->lam.assign(p.lambda, p.lambda + p.n);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) {
    delete r;
    return set_error(RIPK_ECANCELED, "server is shutting down");
  }
  if ((int64_t)sv->queue.size() >= sv->desc.queue_cap) {
    delete r;
    return set_error(RIPK_EAGAIN, "request queue is full");
  }
  r->ticket = sv->next_ticket++;
  r->t_submit = mono_now();
  sv->queue.push_back(r);
  sv->all[r->ticket] = r;
  ++sv->epoch;
  sv->cv_work.notify_all();
  *ticket = r->ticket;
  return RIPK_OK;
}

ripk_status ripk_poll(ripk_server_t sv, uint64_t ticket, ripk_result *out, int32_t timeout_ms) {
  if (!sv || !out) return set_error(RIPK_EINVAL, "null server or result");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return set_error(RIPK_ENOTFOUND, "unknown ticket");
  Request *r = it->second;
  if (!r->done) {
    if (timeout_ms < 0)
      sv->cv_done.wait(lk, [&] { return r->done; });
    else if (timeout_ms > 0)
      sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return r->done; });
  }
  if (!r->done) {
    out->status = RIPK_PENDING;
    return RIPK_PENDING;
  }
  sv->all.erase(it);
  lk.unlock();
  copy_out(r, out);
  const ripk_status st = r->status;
  if (st != RIPK_OK) set_error(st, r->msg.c_str());
  delete r;
  return st;
}

ripk_status ripk_server_status(ripk_server_t sv, ripk_server_state *out) {
  if (!sv || !out) return set_error(RIPK_EINVAL, "null server or output");
  std::lock_guard<std::mutex> lk(sv->mu);
  out->queued = (int64_t)sv->queue.size();
  int busy = 0;
  for (int k = 0; k < sv->desc.slots; ++k) busy += sv->slots[k].busy ? 1 : 0;
  out->busy_slots = busy;
  out->device_bytes = sv->used;
  out->unpolled = (int64_t)sv->all.size();
  return RIPK_OK;
}

}  // extern "C"
