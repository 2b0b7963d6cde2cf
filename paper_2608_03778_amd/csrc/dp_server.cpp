// Serving layer: continuous batching of forward / gradient queries against
// device-resident compiled designs.
//
// Optimizer clients submit queries (a design id, their own PI probabilities
// and per-gate size factors) and return at once.  A scheduler thread:
//   * admits pending queries into idle lanes of their design, oldest first,
//     as long as the lanes' device memory stays inside the HBM budget
//     (a lane is an eval of `capacity` columns with its own stream);
//   * launches the lanes it filled in one pass as one device step: the lanes
//     of all designs in the step share one launch per level index (merged
//     level launches), then each lane's finalize and power, then shared
//     reverse levels for the lanes that want gradients (column b of a lane
//     = query b).  Steps run concurrently on their own streams while new
//     queries keep arriving; under load, queries that waited for a free
//     step are batched across designs into the next one;
//   * polls step completion events, copies results to the queries' buffers
//     and timestamps them.
// A query's result does not depend on the batch it rides in: every column
// of a sweep is computed independently and reduced in a fixed order.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "dp_eval.h"

using dp::fail;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t ticket = 0;
  int32_t design = 0, kind = 0;
  const float *p = nullptr, *size = nullptr;
  float *out_power = nullptr, *out_dpi = nullptr;
  Clock::time_point t_submit, t_done;
  bool done = false;
  dp_status status = DP_OK;
  std::string error;  // why status is not DP_OK
};

struct DesignEntry {
  dp_design *d = nullptr;
  dp_params prm{};
  dp::DevBuf cap_int, beta_int;
  bool frozen = false;
};

struct Lane {
  dp_eval *ev = nullptr;
  int32_t design = 0, capacity = 0;
  hipStream_t stream = nullptr;
  bool busy = false;
  std::vector<Request *> batch;
  float *pin_p = nullptr, *pin_size = nullptr, *pin_power = nullptr, *pin_dpi = nullptr;
  size_t bytes = 0;
};

// One device step in flight: its stream, completion event, the merged
// launches' table scratch and the lanes it carries.
struct Step {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  dp::StepScratch scratch;
  std::vector<Lane *> lanes;
  bool busy = false;
};

}  // namespace

struct dp_server {
  dp_ctx *ctx = nullptr;
  size_t budget = 0;
  int32_t max_batch = 64, max_inflight = 8;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> reqs;
  std::vector<DesignEntry *> designs;
  std::vector<Lane *> lanes;
  std::vector<Step *> steps;
  size_t used = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  dp_server_stats st{};
  Clock::time_point busy_since;
  int32_t inflight = 0;
  std::string thread_error;
};

namespace {

void destroy_lane(Lane *l) {
  if (l->stream) (void)hipStreamSynchronize(l->stream);
  dp_eval_destroy(l->ev);
  if (l->stream) (void)hipStreamDestroy(l->stream);
  (void)hipHostFree(l->pin_p);
  (void)hipHostFree(l->pin_size);
  (void)hipHostFree(l->pin_power);
  (void)hipHostFree(l->pin_dpi);
  delete l;
}

// Create a lane for `design` holding up to `cap` columns (caller holds mu).
Lane *make_lane(dp_server *s, int32_t design, int32_t cap) {
  DesignEntry *de = s->designs[design];
  auto *l = new Lane();
  l->design = design;
  l->capacity = cap;
  const dp_design *d = de->d;
  bool ok = hipStreamCreateWithFlags(&l->stream, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc((void **)&l->pin_p, std::max<size_t>((size_t)cap * d->n_pi * 4, 16)) == hipSuccess &&
            hipHostMalloc((void **)&l->pin_size, std::max<size_t>((size_t)cap * d->n_gates * 4, 16)) == hipSuccess &&
            hipHostMalloc((void **)&l->pin_power, (size_t)cap * 4) == hipSuccess &&
            hipHostMalloc((void **)&l->pin_dpi, std::max<size_t>((size_t)cap * d->n_pi * 4, 16)) == hipSuccess;
  if (ok)
    ok = dp::lane_create(de->d, cap, &de->prm, l->stream, de->cap_int.as<float>(),
                         de->frozen ? de->beta_int.as<float>() : nullptr, &l->ev) == DP_OK;
  if (!ok) {
    (void)hipGetLastError();
    destroy_lane(l);
    return nullptr;
  }
  l->bytes = dp::lane_bytes(d, cap);
  s->lanes.push_back(l);
  s->used += l->bytes;
  s->st.lanes_created++;
  s->st.peak_slot_bytes = std::max<int64_t>(s->st.peak_slot_bytes, (int64_t)s->used);
  return l;
}

// Free idle lanes of other designs until `need` bytes fit (caller holds mu).
bool make_room(dp_server *s, size_t need, int32_t keep_design) {
  for (size_t i = 0; i < s->lanes.size() && s->used + need > s->budget;) {
    Lane *l = s->lanes[i];
    if (!l->busy && l->design != keep_design) {
      s->used -= l->bytes;
      s->st.lanes_freed++;
      destroy_lane(l);
      s->lanes.erase(s->lanes.begin() + i);
    } else {
      ++i;
    }
  }
  return s->used + need <= s->budget;
}

// Copy a lane's queries into its pinned staging (sizes validated here, off
// the submitting thread); returns whether any query brought sizes.
bool stage_lane(dp_server *s, Lane *l) {
  const dp_design *d = s->designs[l->design]->d;
  const int32_t n = (int32_t)l->batch.size();
  bool any_size = false;
  for (int32_t b = 0; b < n; ++b) {
    Request *r = l->batch[b];
    std::memcpy(l->pin_p + (size_t)b * d->n_pi, r->p, (size_t)d->n_pi * 4);
    any_size |= r->size != nullptr;
  }
  if (any_size)
    for (int32_t b = 0; b < n; ++b) {
      float *dst = l->pin_size + (size_t)b * d->n_gates;
      const float *src = l->batch[b]->size;
      if (!src) {
        std::fill(dst, dst + d->n_gates, 1.0f);
        continue;
      }
      bool ok = true;
      for (int32_t g = 0; g < d->n_gates; ++g) {
        const float v = src[g];
        ok &= (v >= 0.0f) & (v <= 3.0e38f);
        dst[g] = v;
      }
      if (!ok) {
        l->batch[b]->status = DP_E_INVALID;
        std::fill(dst, dst + d->n_gates, 1.0f);
      }
    }
  return any_size;
}

// An idle step, created while fewer than max_inflight exist (caller holds mu).
Step *idle_step(dp_server *s) {
  for (Step *st : s->steps)
    if (!st->busy) return st;
  if ((int32_t)s->steps.size() >= s->max_inflight) return nullptr;
  auto *st = new Step();
  if (hipStreamCreateWithFlags(&st->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&st->done, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    if (st->stream) (void)hipStreamDestroy(st->stream);
    delete st;
    return nullptr;
  }
  s->steps.push_back(st);
  return st;
}

// Launch the filled lanes as one device step on `st` (caller holds mu).
void launch_step(dp_server *s, Step *st, const std::vector<Lane *> &ready) {
  std::vector<dp::LaneJob> jobs;
  for (Lane *l : ready) {
    const bool any_size = stage_lane(s, l);
    jobs.push_back({l->ev, (int32_t)l->batch.size(), l->pin_p, any_size ? l->pin_size : nullptr,
                    l->batch[0]->kind == DP_Q_FWD_BWD, l->pin_power, l->pin_dpi});
    l->busy = true;
  }
  dp_status rc = dp::lanes_run_merged(jobs.data(), (int32_t)jobs.size(), st->stream, &st->scratch);
  if (rc == DP_OK && hipEventRecord(st->done, st->stream) != hipSuccess)
    rc = fail(DP_E_HIP, "hipEventRecord failed");
  if (rc != DP_OK) {
    // the step did not go out whole: its queries fail with the reason (their
    // outputs are never read), after whatever was enqueued has drained
    const std::string why = dp_last_error();
    (void)hipStreamSynchronize(st->stream);
    (void)hipGetLastError();
    const auto now = Clock::now();
    for (Lane *l : ready) {
      for (Request *r : l->batch) {
        r->status = rc;
        r->error = "server step: " + why;
        r->t_done = now;
        r->done = true;
        s->st.completed++;
      }
      l->batch.clear();
      l->busy = false;
    }
    s->cv_done.notify_all();
    return;
  }
  st->lanes = ready;
  st->busy = true;
  if (s->inflight++ == 0) s->busy_since = Clock::now();
  s->st.max_inflight = std::max(s->st.max_inflight, s->inflight);
  s->st.device_steps++;
}

void finish_lane(dp_server *s, Lane *l, Clock::time_point now) {
  const dp_design *d = s->designs[l->design]->d;
  for (size_t b = 0; b < l->batch.size(); ++b) {
    Request *r = l->batch[b];
    if (r->out_power) *r->out_power = l->pin_power[b];
    if (r->out_dpi && r->kind == DP_Q_FWD_BWD)
      std::memcpy(r->out_dpi, l->pin_dpi + b * (size_t)d->n_pi, (size_t)d->n_pi * 4);
    r->t_done = now;
    r->done = true;
    s->st.completed++;
  }
  l->batch.clear();
  l->busy = false;
}

void finish_step(dp_server *s, Step *st) {
  const auto now = Clock::now();
  for (Lane *l : st->lanes) finish_lane(s, l, now);
  st->lanes.clear();
  st->busy = false;
  if (--s->inflight == 0)
    s->st.busy_s += std::chrono::duration<double>(now - s->busy_since).count();
}

// Admit pending queries into idle lanes, oldest first, and launch the lanes
// filled in this pass as one step (caller holds mu).
void admit(dp_server *s) {
  if (s->pending.empty()) return;
  Step *step = idle_step(s);
  if (!step) return;  // every step is in flight; queries wait and batch up
  std::vector<Lane *> ready;
  int32_t carried = 0;  // queries in this step: at most max_batch
  for (size_t i = 0; i < s->pending.size() && carried < s->max_batch;) {
    Request *r = s->pending[i];
    Lane *lane = nullptr;
    for (Lane *l : s->lanes)
      if (!l->busy && l->design == r->design) {
        lane = l;
        break;
      }
    if (!lane) {
      const dp_design *d = s->designs[r->design]->d;
      int32_t want = 0;  // queries of this design waiting
      for (Request *q : s->pending) want += q->design == r->design;
      int32_t cap = std::min(s->max_batch, std::max(want, 1));
      // round the capacity up to a power of two so lanes are reused
      int32_t c2 = 1;
      while (c2 < cap) c2 <<= 1;
      cap = std::min(c2, s->max_batch);
      while (cap > 1 && dp::lane_bytes(d, cap) > s->budget) cap >>= 1;
      // under memory pressure a smaller lane that fits what is free now is
      // preferred to freeing other designs' idle lanes: a lane costs
      // allocations to create, which freeing throws away
      const size_t free_now = s->used < s->budget ? s->budget - s->used : 0;
      int32_t fit = cap;
      while (fit > 1 && dp::lane_bytes(d, fit) > free_now) fit >>= 1;
      if (dp::lane_bytes(d, fit) <= free_now) cap = fit;
      const size_t need = dp::lane_bytes(d, cap);
      // other designs' idle lanes are freed only for a design that has no
      // lane at all; one that has (busy) lanes waits for them instead, so
      // designs do not free and recreate each other's lanes under load (a
      // lane's pinned staging alone takes a large design hundreds of ms)
      bool has_lane = false;
      for (Lane *l : s->lanes) has_lane |= l->design == r->design;
      if (s->used + need > s->budget && (has_lane || !make_room(s, need, r->design))) {
        s->st.memory_waits++;
        ++i;  // no memory now; a running lane will free some
        continue;
      }
      lane = make_lane(s, r->design, cap);
      if (!lane) {
        ++i;
        continue;
      }
    }
    // fill the lane with same-design, same-kind queries in arrival order
    for (size_t j = i; j < s->pending.size() && (int32_t)lane->batch.size() < lane->capacity &&
                       carried < s->max_batch;) {
      Request *q = s->pending[j];
      if (q->design == r->design && q->kind == r->kind) {
        lane->batch.push_back(q);
        s->pending.erase(s->pending.begin() + j);
        ++carried;
      } else {
        ++j;
      }
    }
    lane->busy = true;  // taken: not reused or freed while this pass goes on
    ready.push_back(lane);
  }
  if (!ready.empty()) launch_step(s, step, ready);
}

void scheduler(dp_server *s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool completed = false;
    for (Step *st : s->steps)
      if (st->busy && hipEventQuery(st->done) == hipSuccess) {
        finish_step(s, st);
        completed = true;
      }
    if (completed) s->cv_done.notify_all();
    admit(s);
    if (s->inflight == 0 && s->pending.empty()) {
      s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
    } else if (s->inflight == 0) {  // nothing could be admitted (allocation failed)
      s->cv_work.wait_for(lk, std::chrono::milliseconds(1));
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

// Scheduler threads still running when the process exits are stopped
// before the HIP runtime tears down (handlers registered later run first).
std::mutex g_live_mu;
std::vector<dp_server *> g_live;
std::once_flag g_atexit_once;

void stop_thread(dp_server *s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
}

void stop_all_at_exit() {
  std::lock_guard<std::mutex> g(g_live_mu);
  for (dp_server *s : g_live) stop_thread(s);
}

}  // namespace

extern "C" {

dp_status dp_server_create(dp_ctx *ctx, size_t hbm_budget_bytes, dp_server **out) {
  if (!ctx || !out) return fail(DP_E_INVALID, "dp_server_create: NULL argument");
  if (hbm_budget_bytes == 0) return fail(DP_E_INVALID, "dp_server_create: zero budget");
  std::call_once(g_atexit_once, [] { std::atexit(stop_all_at_exit); });
  auto *s = new dp_server();
  s->ctx = ctx;
  dp::ctx_retain(ctx);
  s->budget = hbm_budget_bytes;
  s->th = std::thread(scheduler, s);
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live.push_back(s);
  }
  *out = s;
  return DP_OK;
}

dp_status dp_server_configure(dp_server *s, int32_t max_batch, int32_t max_inflight) {
  if (!s || max_batch < 1 || max_inflight < 1)
    return fail(DP_E_INVALID, "dp_server_configure: need max_batch >= 1, max_inflight >= 1");
  std::lock_guard<std::mutex> g(s->mu);
  s->max_batch = max_batch;
  s->max_inflight = max_inflight;
  return DP_OK;
}

dp_status dp_server_add_design(dp_server *s, dp_design *d, const float *cap,
                               const dp_params *params, int32_t *design_id) {
  if (!s || !d || !cap || !params || !design_id)
    return fail(DP_E_INVALID, "dp_server_add_design: NULL argument");
  if (params->mode == DP_HYBRID)
    return fail(DP_E_UNSUPPORTED,
                "dp_server_add_design: queries run DP_MODELED or DP_FROZEN_BETA (beta is "
                "calibrated once here)");
  for (int32_t n = 0; n < d->n_nets; ++n)
    if (!(cap[n] >= 0.0f && cap[n] <= 3.0e38f))
      return fail(DP_E_INVALID, "dp_server_add_design: bad capacitance");
  auto *de = new DesignEntry();
  de->d = d;
  dp::design_retain(d);
  de->prm = *params;
  de->frozen = params->mode == DP_FROZEN_BETA;
  dp_status st = de->cap_int.alloc((size_t)d->n_nets * 4 + 16);
  if (st == DP_OK) {
    std::vector<float> ci(d->n_nets);
    for (int32_t n = 0; n < d->n_nets; ++n) ci[n] = cap[d->h_int2ext[n]];
    hipError_t e = hipMemcpy(de->cap_int.ptr, ci.data(), ci.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) st = fail(DP_E_HIP, std::string("dp_server_add_design: ") + hipGetErrorString(e));
  }
  if (st == DP_OK && de->frozen) {
    st = de->beta_int.alloc((size_t)d->n_nets * 4 + 16);
    if (st == DP_OK) st = dp::calibrate_beta(d, cap, params, 0.5f, de->beta_int.as<float>());
  }
  if (st != DP_OK) {
    delete de;
    dp::design_release(d);
    return st;
  }
  std::lock_guard<std::mutex> g(s->mu);
  *design_id = (int32_t)s->designs.size();
  s->designs.push_back(de);
  return DP_OK;
}

dp_status dp_submit(dp_server *s, const dp_query *q, uint64_t *ticket) {
  if (!s || !q || !ticket) return fail(DP_E_INVALID, "dp_submit: NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  if (q->design_id < 0 || q->design_id >= (int32_t)s->designs.size())
    return fail(DP_E_NOTFOUND, "dp_submit: unknown design id");
  if (q->kind != DP_Q_FWD && q->kind != DP_Q_FWD_BWD)
    return fail(DP_E_INVALID, "dp_submit: unknown query kind");
  const dp_design *d = s->designs[q->design_id]->d;
  if (dp::lane_bytes(d, 1) > s->budget)
    return fail(DP_E_BUDGET, "dp_submit: one query of this design exceeds the HBM budget");
  if (!s->thread_error.empty()) return fail(DP_E_HIP, "server: " + s->thread_error);
  lk.unlock();
  if (!q->pi_prob) return fail(DP_E_INVALID, "dp_submit: NULL pi_prob");
  for (int32_t i = 0; i < d->n_pi; ++i)
    if (!(q->pi_prob[i] >= 0.0f && q->pi_prob[i] <= 1.0f))
      return fail(DP_E_INVALID, "dp_submit: PI probability NaN or outside [0, 1]");
  auto *r = new Request();
  r->design = q->design_id;
  r->kind = q->kind;
  r->p = q->pi_prob;
  r->size = q->cap_scale;
  r->out_power = q->power;
  r->out_dpi = q->dpower_dpi;
  r->t_submit = Clock::now();
  lk.lock();
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->pending.push_back(r);
  s->st.submitted++;
  *ticket = r->ticket;
  lk.unlock();
  s->cv_work.notify_one();
  return DP_OK;
}

dp_status dp_poll(dp_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return fail(DP_E_INVALID, "dp_poll: NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(DP_E_NOTFOUND, "dp_poll: unknown ticket");
  *done = it->second->done ? 1 : 0;
  return DP_OK;
}

dp_status dp_wait(dp_server *s, uint64_t ticket, double *latency_s) {
  if (!s) return fail(DP_E_INVALID, "dp_wait: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(DP_E_NOTFOUND, "dp_wait: unknown ticket");
  Request *r = it->second;
  s->cv_done.wait(lk, [&] { return r->done || !s->thread_error.empty(); });
  if (!r->done) return fail(DP_E_HIP, "server: " + s->thread_error);
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  const dp_status st = r->status;
  const std::string why = r->error;
  s->reqs.erase(it);
  delete r;
  if (st != DP_OK)
    return fail(st, why.empty() ? "dp_wait: the query's cap_scale had a NaN or negative entry" : why);
  return DP_OK;
}

dp_status dp_server_get_stats(dp_server *s, dp_server_stats *out) {
  if (!s || !out) return fail(DP_E_INVALID, "dp_server_get_stats: NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  if (s->inflight > 0)
    out->busy_s += std::chrono::duration<double>(Clock::now() - s->busy_since).count();
  return DP_OK;
}

void dp_server_destroy(dp_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(g_live_mu);
    g_live.erase(std::remove(g_live.begin(), g_live.end(), s), g_live.end());
  }
  stop_thread(s);
  for (Step *st : s->steps) {
    (void)hipStreamSynchronize(st->stream);
    (void)hipEventDestroy(st->done);
    (void)hipStreamDestroy(st->stream);
    delete st;
  }
  for (Lane *l : s->lanes) destroy_lane(l);
  for (DesignEntry *de : s->designs) {
    dp_design *d = de->d;
    delete de;
    dp::design_release(d);
  }
  for (auto &kv : s->reqs) delete kv.second;
  dp::ctx_release(s->ctx);
  delete s;
}

}  // extern "C"
