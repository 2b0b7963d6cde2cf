// C-ABI entry points of libdiffpower: contexts, designs, evals, forward and
// reverse sweeps.  The serving layer lives in dp_server.cpp.
#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>

#include "dp_eval.h"

namespace dp {

static thread_local std::string g_err;

dp_status fail(dp_status st, const std::string &msg) {
  g_err = msg;
  return st;
}
void clear_error() { g_err.clear(); }

void ctx_retain(dp_ctx *c) { c->refs.fetch_add(1); }
void ctx_release(dp_ctx *c) {
  if (c->refs.fetch_sub(1) != 1) return;
  if (c->owned) {
    (void)hipStreamSynchronize(c->owned);
    (void)hipStreamDestroy(c->owned);
  }
  delete c;
}
void design_retain(dp_design *d) { d->refs.fetch_add(1); }
void design_release(dp_design *d) {
  if (d->refs.fetch_sub(1) != 1) return;
  dp_ctx *c = d->ctx;
  (void)hipStreamSynchronize(c->stream);
  delete d;
  ctx_release(c);
}

}  // namespace dp

using dp::DevBuf;
using dp::fail;

namespace {

constexpr int64_t kAutoWordBudget = 32ll << 30;  // bytes of simulation words in flight
// Largest forward sweep (kernel launches) captured into one HIP graph.  A graph
// pays off where a sweep is launch-bound; bigger sweeps run per level.
constexpr int64_t kMaxGraphLaunches = 1024;
const char *kVersion = "diffpower-mi355x 0.1 (gfx950)";
enum { SPAN_SIM = 0, SPAN_SP = 1, SPAN_BWD = 2, SPAN_STIM = 3 };

dp::GraphView view(const dp_design *d) { return dp::design_view(d); }
using dp::for_level_parts;
using dp::pairs_levels;

int32_t s_prime(const dp_eval *ev) { return (ev->S > 0 && !ev->paired_sizes) ? ev->S : 1; }
double kappa_of(const dp_params &p) { return p.energy_factor * p.vdd * p.vdd * p.fclk; }
int64_t n_words(const dp_params &p) { return p.n_sim / 64; }

dp_status check_params(const dp_params *p) {
  if (!p) return fail(DP_E_INVALID, "NULL params");
  if (p->mode < DP_MODELED || p->mode > DP_FROZEN_BETA)
    return fail(DP_E_INVALID, "params.mode must be DP_MODELED, DP_HYBRID or DP_FROZEN_BETA");
  if (p->beta_grad != DP_BETA_LOCAL && p->beta_grad != DP_BETA_STE)
    return fail(DP_E_INVALID, "params.beta_grad must be DP_BETA_LOCAL or DP_BETA_STE");
  if (!(p->beta_min > 0.0) || !(p->beta_max >= p->beta_min) || !std::isfinite(p->beta_max))
    return fail(DP_E_INVALID, "params: need 0 < beta_min <= beta_max < inf");
  const double k = kappa_of(*p);
  if (!std::isfinite(k) || k < 0.0) return fail(DP_E_INVALID, "params: bad vdd/fclk/energy_factor");
  if (p->mode == DP_HYBRID) {
    if (p->n_sim < 128 || p->n_sim % 64 != 0)
      return fail(DP_E_INVALID, "params.n_sim must be a multiple of 64 and >= 128 in DP_HYBRID");
    if (p->n_sim / 64 > (int64_t)INT32_MAX)
      return fail(DP_E_INVALID, "params.n_sim too large");
  }
  return DP_OK;
}

// Validate a float array (host or device) against [lo, hi] (NaN rejected).
dp_status check_values(dp_eval *ev, const float *v, int64_t n, float lo, float hi, int on_device,
                       const char *what) {
  if (!v) return fail(DP_E_INVALID, std::string(what) + ": NULL pointer");
  if (!on_device) {
    for (int64_t i = 0; i < n; ++i)
      if (!(v[i] >= lo && v[i] <= hi))
        return fail(DP_E_INVALID, std::string(what) + ": value " + std::to_string(v[i]) +
                                      " at index " + std::to_string(i) + " out of range");
    return DP_OK;
  }
  hipStream_t s = ev->stream();
  DP_TRY(ev->flag.alloc(sizeof(int32_t)));
  DP_HIP_TRY(dp::launch_fill_u32(ev->flag.as<uint32_t>(), 1, 0u, s));
  DP_HIP_TRY(dp::launch_check_range(v, n, lo, hi, ev->flag.as<int32_t>(), s));
  int32_t bad = 0;
  DP_HIP_TRY(hipMemcpyAsync(&bad, ev->flag.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  DP_HIP_TRY(hipStreamSynchronize(s));
  if (bad) return fail(DP_E_INVALID, std::string(what) + ": a value is NaN or out of range");
  return DP_OK;
}

// Copy a caller array into a device staging buffer (device-to-device when on_device).
dp_status stage_in(DevBuf &buf, const void *src, size_t bytes, int on_device, hipStream_t s) {
  DP_TRY(buf.alloc(std::max<size_t>(bytes, 16)));
  if (bytes)
    DP_HIP_TRY(hipMemcpyAsync(buf.ptr, src, bytes,
                              on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
  return DP_OK;
}

// --- profiling: events around launches, resolved after the stream drains
hipEvent_t take_event(dp_eval *ev) {
  if (ev->ev_used == ev->ev_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ev->ev_pool.push_back(e);
  }
  return ev->ev_pool[ev->ev_used++];
}

struct SpanGuard {
  dp_eval *ev;
  size_t a = 0;
  int kind;
  double bytes;
  bool on;
  int64_t launches;
  hipStream_t st;
  SpanGuard(dp_eval *e, int k, double b, bool enabled, int64_t n_launch,
            hipStream_t stream = nullptr)
      : ev(e), kind(k), bytes(b), on(enabled), launches(n_launch),
        st(stream ? stream : e->stream()) {
    if (on) {
      a = ev->ev_used;
      hipEvent_t x = take_event(ev);
      if (!x) { on = false; return; }
      (void)hipEventRecord(x, st);
    }
  }
  ~SpanGuard() {
    if (!on) return;
    size_t b = ev->ev_used;
    hipEvent_t x = take_event(ev);
    if (!x) return;
    (void)hipEventRecord(x, st);
    ev->spans.push_back({a, b, kind, bytes, launches});
  }
};

dp_status resolve_profile(dp_eval *ev) {
  if (ev->spans.empty()) {
    ev->ev_used = 0;
    return DP_OK;
  }
  DP_HIP_TRY(hipStreamSynchronize(ev->stream()));
  for (const auto &sp : ev->spans) {
    float ms = 0.0f;
    DP_HIP_TRY(hipEventElapsedTime(&ms, ev->ev_pool[sp.a], ev->ev_pool[sp.b]));
    switch (sp.kind) {
      case SPAN_SIM: ev->prof.sim_ms += ms; ev->prof.sim_launches += sp.launches; ev->prof.sim_bytes += sp.bytes; break;
      case SPAN_SP: ev->prof.sp_ms += ms; ev->prof.sp_launches += sp.launches; ev->prof.sp_bytes += sp.bytes; break;
      case SPAN_BWD: ev->prof.bwd_ms += ms; ev->prof.bwd_launches += sp.launches; ev->prof.bwd_bytes += sp.bytes; break;
      default: ev->prof.stim_ms += ms; ev->prof.stim_launches += sp.launches; break;
    }
  }
  ev->spans.clear();
  ev->ev_used = 0;
  return DP_OK;
}

// --- chunking of the simulated words
// The simulation holds `cols` query columns' word buffers per stream (a
// column group, simulated by the same launches), each Tc words (plus a
// two-word halo when the run is cut into chunks) per net.
struct ChunkPlan {
  int64_t T = 0, Tc = 0, pitch = 0;
  int32_t halo = 0, n_chunks = 0;
  int32_t cols = 1;      // query columns per launch
  int32_t n_groups = 1;  // column groups, ceil(B / cols)
};

int32_t n_sim_streams(const dp_eval *ev) { return ev->sim_streams > 0 ? ev->sim_streams : 1; }

ChunkPlan plan_chunks(const dp_eval *ev) {
  ChunkPlan c;
  c.T = n_words(ev->prm);
  // words per net that fit one stream's share of the budget, over all the
  // columns of its buffer
  const int64_t row_budget = std::max<int64_t>(
      kAutoWordBudget / (8 * (int64_t)ev->d->n_nets * n_sim_streams(ev)), 4);
  int64_t want = ev->words_per_chunk;
  if (want <= 0) want = c.T + (c.T & 1) <= row_budget ? c.T : row_budget - 2;
  want = std::max<int64_t>(2, want + (want & 1));
  if (want >= c.T) {
    c.Tc = c.T + (c.T & 1);
    c.halo = 0;
    c.n_chunks = 1;
  } else {
    c.Tc = want;
    c.halo = 2;
    c.n_chunks = (int32_t)((c.T + c.Tc - 1) / c.Tc);
  }
  c.pitch = c.halo + c.Tc;
  // as many columns per launch as the budget holds at this pitch
  c.cols = (int32_t)std::max<int64_t>(1, std::min<int64_t>(ev->B, row_budget / c.pitch));
  if (ev->sim_cols > 0) c.cols = std::min(c.cols, ev->sim_cols);
  c.n_groups = (ev->B + c.cols - 1) / c.cols;
  return c;
}

// Chunk k of column group `grp` on simulation stream `lane`.
dp::ChunkView chunk_view(const dp_eval *ev, const ChunkPlan &pl, int32_t k, int32_t lane,
                         int32_t grp) {
  dp::ChunkView v;
  const int64_t col_stride = (int64_t)ev->d->n_nets * pl.pitch;
  v.W = ev->words.as<uint64_t>() + (size_t)lane * pl.cols * col_stride;
  v.pitch = pl.pitch;
  v.col_stride = col_stride;
  const int64_t t0 = (int64_t)k * pl.Tc;
  const int64_t nw = std::min<int64_t>(pl.Tc, pl.T - t0);
  v.t_first = t0 - pl.halo;
  v.u_lo = pl.halo;
  v.u_hi = (int32_t)(pl.halo + nw);
  v.u_tog_lo = t0 == 0 ? pl.halo + 1 : pl.halo;
  v.pairs = (v.u_hi + 1) / 2;
  v.n_cols = std::min(pl.cols, ev->B - grp * pl.cols);
  return v;
}

int32_t pick_iters(const dp_eval *ev, const ChunkPlan &pl) {
  if (ev->sim_iters > 0) return ev->sim_iters;
  // about two waves per row: enough waves per level, few carry recomputes
  const int64_t pairs = pl.pitch / 2;
  if (pairs >= 1024) return 8;
  if (pairs >= 512) return 4;
  if (pairs >= 256) return 2;
  return 1;
}

bool hybrid(const dp_eval *ev) { return ev->prm.mode == DP_HYBRID; }

// A cooperative launch cannot be enqueued on the null stream; there it runs
// on a private stream that waits for the caller's stream and that the caller's
// stream then waits for.  Elsewhere it goes to `s` itself.
template <class F>
dp_status on_coop_stream(dp_eval *ev, hipStream_t s, F launch) {
  if (s) {
    DP_HIP_TRY(launch(s));
    return DP_OK;
  }
  if (!ev->coop_stream) {
    DP_HIP_TRY(hipStreamCreateWithFlags(&ev->coop_stream, hipStreamNonBlocking));
    for (hipEvent_t &e : ev->coop_events) DP_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  DP_HIP_TRY(hipEventRecord(ev->coop_events[0], s));
  DP_HIP_TRY(hipStreamWaitEvent(ev->coop_stream, ev->coop_events[0], 0));
  DP_HIP_TRY(launch(ev->coop_stream));
  DP_HIP_TRY(hipEventRecord(ev->coop_events[1], ev->coop_stream));
  DP_HIP_TRY(hipStreamWaitEvent(s, ev->coop_events[1], 0));
  return DP_OK;
}

// The persistent sweeps' barrier words (allocated and zeroed when the
// schedule is chosen; the launcher zeroes all but the report word before
// each launch).
dp_status grid_barrier(dp_eval *ev, dp::GridBarrier *out) {
  if (!ev->barrier.ptr) return fail(DP_E_STATE, "persistent sweep without its barrier words");
  const double ticks = ev->barrier_limit_us * 100.0;  // the real-time counter runs at 100 MHz
  *out = dp::GridBarrier{ev->barrier.as<uint32_t>(), (uint64_t)std::max(ticks, 0.0)};
  ev->barrier_pending = true;
  return DP_OK;
}

// At a host synchronization of the eval (its stream idle): whether a
// persistent sweep since the last check had a barrier wait give up.  Reads
// and clears the report word.
dp_status barrier_status(dp_eval *ev) {
  if (!ev->barrier_pending) return DP_OK;
  uint32_t rep = 0;
  uint32_t *w = ev->barrier.as<uint32_t>() + dp::kBarrierReport;
  DP_HIP_TRY(hipMemcpy(&rep, w, sizeof(uint32_t), hipMemcpyDeviceToHost));
  ev->barrier_pending = false;
  if (rep == 0u) return DP_OK;
  DP_HIP_TRY(dp::launch_fill_u32(w, 1, 0u, ev->stream()));
  DP_HIP_TRY(hipStreamSynchronize(ev->stream()));
  return fail(DP_E_HIP, "a persistent sweep's grid barrier gave up waiting (no progress for " +
                            std::to_string(ev->barrier_limit_us) +
                            " us); that sweep's outputs are NaN and not a result");
}

// Synchronize the eval's stream when a persistent sweep is unchecked, then
// report it (host-output calls end here).
dp_status sync_and_check(dp_eval *ev) {
  if (!ev->barrier_pending) return DP_OK;
  DP_HIP_TRY(hipStreamSynchronize(ev->stream()));
  return barrier_status(ev);
}

// Per-net beta [n_nets][B] of the last forward: the computed one (hybrid),
// the frozen one as given, or null in modeled mode (beta = 1).  (A frozen
// beta shared by every column is [n_nets]: see backward_args.)
float *beta_or_null(dp_eval *ev) {
  if (ev->prm.mode == DP_MODELED) return nullptr;
  return ev->prm.mode == DP_HYBRID ? ev->beta.as<float>() : ev->beta_frozen.as<float>();
}

// Whether the forward draws Markov stimulus words (a target transition rate
// per PI and no explicit stimulus).
bool markov(const dp_eval *ev) { return ev->have_tau && !ev->have_stim; }

// Launches of the modeled sweep's SP levels.
int64_t sp_sweep_launches(const dp_design *d, int32_t B) {
  int64_t n = 0;
  for (int32_t l = 1; l <= d->depth;) {
    if (pairs_levels(d, l, B)) {
      ++n;
      l += 2;
    } else {
      n += d->lvl_fixed[l] > 0 ? 1 : 0;
      n += d->lvl_fixed[l] < d->level_ptr[l + 1] - d->level_ptr[l] ? 1 : 0;
      ++l;
    }
  }
  return n;
}

// Kernel launches of one forward sweep (what a captured graph would hold).
int64_t forward_launches(const dp_eval *ev, const ChunkPlan *pl) {
  const int64_t depth = ev->d->depth + ev->d->split_levels;
  if (!pl) return sp_sweep_launches(ev->d, ev->B) + 2;
  return (int64_t)pl->n_groups * pl->n_chunks * (depth + 1) + 4 + (markov(ev) ? 1 : 0) +
         ev->d->cell_levels;  // the library cells' SP launches
}

// Allocate everything the forward sweep touches (before any capture).
dp_status ensure_forward_buffers(dp_eval *ev, const ChunkPlan *pl) {
  const dp_design *d = ev->d;
  const size_t nb = (size_t)d->n_nets * ev->B;
  if (ev->prm.mode == DP_HYBRID) DP_TRY(ev->beta.alloc(nb * sizeof(float)));
  const int32_t cols = ev->B * s_prime(ev);
  DP_TRY(ev->power_partial.alloc(
      (size_t)dp::power_partial_doubles(d->n_nets, ev->B, ev->S, ev->paired_sizes) *
      sizeof(double)));
  DP_TRY(ev->power.alloc((size_t)cols * sizeof(float)));
  if (pl) {
    DP_TRY(ev->ones.alloc(nb * sizeof(uint32_t)));
    DP_TRY(ev->tog.alloc(nb * sizeof(uint32_t)));
    const int32_t L = n_sim_streams(ev);
    DP_TRY(ev->words.alloc((size_t)L * pl->cols * d->n_nets * pl->pitch * sizeof(uint64_t)));
    if (markov(ev))
      DP_TRY(ev->mstim.alloc(std::max<size_t>((size_t)ev->B * d->n_pi * pl->T * sizeof(uint64_t), 16)));
    while ((int32_t)ev->lane_streams.size() < L - 1) {
      hipStream_t st = nullptr;
      DP_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      ev->lane_streams.push_back(st);
    }
    while ((int32_t)ev->lane_events.size() < L) {
      hipEvent_t e = nullptr;
      DP_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      ev->lane_events.push_back(e);
    }
  }
  return DP_OK;
}

// Algorithmic bytes of one simulation launch of level l over `cols`
// columns of `words` words each (and the level's SP over B columns when
// fused).
double sim_level_bytes(const dp_design *d, int32_t l, int64_t words, int32_t cols, int32_t B,
                       bool fused) {
  const int64_t n = d->level_ptr[l + 1] - d->level_ptr[l];
  const int64_t pins = d->lvl_pins[l], read = d->lvl_read[l];
  // per column: fan-in words, output words of the nets that have readers (a
  // net without readers needs only its counts, so its words are not
  // stored), counters; per launch: indices, cell, fan-out range
  double b = (double)cols * ((double)(8 * pins + 8 * read) * (double)words + 8.0 * n)
             + (double)(4 * pins + n) + 8.0 * n;
  if (fused) b += (double)B * (4 * pins + 4 * n);  // SP gathers and writes
  return b;
}

double sp_level_bytes(const dp_design *d, int32_t l, int32_t B) {
  const int64_t n = d->level_ptr[l + 1] - d->level_ptr[l];
  const int64_t pins = d->lvl_pins[l];
  return (double)B * (4 * pins + 4 * n) + (double)(4 * pins + n);  // stored SP gathers, writes
}

double bwd_level_bytes(const dp_design *d, int32_t l, int32_t C) {
  const int64_t n = d->level_ptr[l + 1] - d->level_ptr[l];
  const int64_t pins = d->lvl_pins[l], fo = d->lvl_fanout[l];
  // per column: own SP (the seed), pulled contributions, fan-in SP gathers,
  // contribution writes
  const double per_col = 4.0 * n + 4.0 * fo + 4.0 * pins + 4.0 * pins;
  // structure: fan-out offsets and edge ids, fan-in indices, cell
  const double structure = 8.0 * n + 4.0 * fo + 4.0 * pins + n;
  return (double)C * per_col + structure;
}

// Enqueue the whole forward sweep (no host sync, no allocation).
dp_status enqueue_forward_tail(dp_eval *ev, const ChunkPlan *pl);


dp_status enqueue_forward(dp_eval *ev, const ChunkPlan *pl) {
  const dp_design *d = ev->d;
  hipStream_t s = ev->stream();
  const dp::GraphView g = view(d);
  const bool prof = ev->profiling;
  float *sp = ev->sp.as<float>();
  if (!pl) {  // modeled (or frozen-beta) sweep: one span over all level launches
    double bytes = 0.0;
    for (int32_t l = 1; l <= d->depth; ++l) bytes += sp_level_bytes(d, l, ev->B);
    SpanGuard sg(ev, SPAN_SP, bytes, prof && d->depth > 0,
                 ev->schedule == DP_SCHED_PERSISTENT ? 1 : sp_sweep_launches(d, ev->B));
    if (ev->schedule == DP_SCHED_PERSISTENT) {
      dp::SpLevel lv{sp, ev->B, 0, 0};
      dp::GridBarrier bar;
      DP_TRY(grid_barrier(ev, &bar));
      DP_TRY(on_coop_stream(ev, s, [&](hipStream_t cs) {
        return dp::launch_sp_persistent(g, lv, d->level_dev.as<int32_t>(), d->depth,
                                        (int64_t)d->max_level_width * ev->B, bar, cs);
      }));
    } else {
      for (int32_t l = 1; l <= d->depth;) {
        if (pairs_levels(d, l, ev->B)) {  // levels l and l + 1 in one launch
          const int32_t a0 = d->level_ptr[l], a1 = d->level_ptr[l + 1], b1 = d->level_ptr[l + 2];
          DP_HIP_TRY(dp::launch_sp_pair(g, dp::SpLevel{sp, ev->B, a0, a1 - a0},
                                        dp::SpLevel{sp, ev->B, a1, b1 - a1}, s));
          l += 2;
          continue;
        }
        DP_TRY(for_level_parts(d, l, [&](int32_t g0, int32_t n, bool cells) -> dp_status {
          DP_HIP_TRY(dp::launch_sp_level(g, dp::SpLevel{sp, ev->B, g0, n}, cells, s));
          return DP_OK;
        }));
        ++l;
      }
    }
  } else {
    const size_t nb = (size_t)d->n_nets * ev->B;
    DP_HIP_TRY(dp::launch_fill_u32(ev->ones.as<uint32_t>(), (int64_t)nb, 0u, s));
    DP_HIP_TRY(dp::launch_fill_u32(ev->tog.as<uint32_t>(), (int64_t)nb, 0u, s));
    dp::SimTune tune{pick_iters(ev, *pl)};
    const int32_t *streams = ev->have_streams ? ev->streams.as<int32_t>() : nullptr;
    const uint64_t *stim_all = nullptr;  // [B][n_pi][T] words, or the generator
    if (ev->have_stim) {
      stim_all = ev->stim.as<uint64_t>();
    } else if (markov(ev)) {
      SpanGuard sg(ev, SPAN_STIM, 0.0, prof, 1);
      DP_HIP_TRY(dp::launch_markov_words(sp, ev->tau.as<float>(), streams, d->n_pi, ev->B, pl->T,
                                         ev->prm.seed, ev->mstim.as<uint64_t>(), s));
      stim_all = ev->mstim.as<uint64_t>();
    }
    // (column group, chunk) pieces are independent: piece j runs on stream
    // j % L with its own word buffers; the SP of each level is fused into
    // piece 0.
    const int32_t n_pieces = pl->n_groups * pl->n_chunks;
    // a capture records one stream only (multi-stream captures are off)
    const int32_t L = ev->capturing ? 1 : std::min<int32_t>(n_sim_streams(ev), n_pieces);
    if (L > 1) {
      DP_HIP_TRY(hipEventRecord(ev->lane_events[0], s));
      for (int32_t i = 1; i < L; ++i)
        DP_HIP_TRY(hipStreamWaitEvent(ev->lane_streams[i - 1], ev->lane_events[0], 0));
    }
    for (int32_t j = 0; j < n_pieces; ++j) {
      const int32_t grp = j / pl->n_chunks, k = j % pl->n_chunks, lane = j % L;
      const int32_t b = grp * pl->cols;  // first column of the group
      hipStream_t ls = lane == 0 ? s : ev->lane_streams[lane - 1];
      dp::CountView cnt{ev->ones.as<uint32_t>(), ev->tog.as<uint32_t>(), ev->B, b};
      const uint64_t *stim = stim_all ? stim_all + (size_t)b * d->n_pi * pl->T : nullptr;
      const dp::ChunkView cv = chunk_view(ev, *pl, k, lane, grp);
      {
        SpanGuard sg(ev, SPAN_STIM, 0.0, prof, 1, ls);
        DP_HIP_TRY(dp::launch_stimulus(g, cv, cnt, sp, stim, pl->T, streams, ev->prm.seed, tune,
                                       ls));
      }
      const bool fuse = (j == 0);
      const int64_t nw = cv.u_hi - cv.u_lo;
      double bytes = 0.0;
      for (int32_t l = 1; l <= d->depth; ++l)
        bytes += sim_level_bytes(d, l, nw, cv.n_cols, ev->B, fuse);
      // one span over the piece's level launches (their back-to-back time)
      SpanGuard sg(ev, SPAN_SIM, bytes, prof && d->depth > 0, d->depth + d->split_levels, ls);
      for (int32_t l = 1; l <= d->depth; ++l)
        DP_TRY(for_level_parts(d, l, [&](int32_t g0, int32_t n, bool cells) -> dp_status {
          const dp::SpLevel lv{sp, ev->B, g0, n};
          if (!cells) {
            DP_HIP_TRY(dp::launch_sim_level(g, cv, cnt, g0, n, fuse ? &lv : nullptr, false, tune,
                                            ls));
            return DP_OK;
          }
          // library cells: the narrow ones (sorted first) and the wider ones in
          // launches of their own; the range's SP rides with the first
          const int32_t ns = d->lvl_small_cells[l];
          if (ns > 0)
            DP_HIP_TRY(dp::launch_sim_level(g, cv, cnt, g0, ns, fuse ? &lv : nullptr, true, tune,
                                            ls, dp::kSmallCellInputs));
          if (ns < n)
            DP_HIP_TRY(dp::launch_sim_level(g, cv, cnt, g0 + ns, n - ns,
                                            fuse && ns == 0 ? &lv : nullptr, true, tune, ls));
          return DP_OK;
        }));
    }
    if (L > 1)
      for (int32_t i = 1; i < L; ++i) {
        DP_HIP_TRY(hipEventRecord(ev->lane_events[i], ev->lane_streams[i - 1]));
        DP_HIP_TRY(hipStreamWaitEvent(s, ev->lane_events[i], 0));
      }
  }
  return enqueue_forward_tail(ev, pl);
}

// The power terms (TR, beta) and their sum over nets, after a forward sweep.
dp_status enqueue_forward_tail(dp_eval *ev, const ChunkPlan *pl) {
  const dp_design *d = ev->d;
  hipStream_t s = ev->stream();
  float *sp = ev->sp.as<float>();
  dp::PowerArgs pa{};
  pa.sp = sp;
  pa.tog = pl ? ev->tog.as<uint32_t>() : nullptr;
  pa.beta_frozen = ev->prm.mode == DP_FROZEN_BETA ? ev->beta_frozen.as<float>() : nullptr;
  pa.beta_shared = ev->beta_shared;
  pa.cap = ev->cap.as<float>();
  pa.size = ev->S > 0 ? ev->size.as<float>() : nullptr;
  pa.T = pl ? pl->T : 0;
  pa.kappa = (float)kappa_of(ev->prm);
  pa.beta_min = (float)ev->prm.beta_min;
  pa.beta_max = (float)ev->prm.beta_max;
  pa.mode = ev->prm.mode;
  pa.beta = hybrid(ev) ? ev->beta.as<float>() : nullptr;  // hybrid: stored on the way
  pa.n_pi = d->n_pi;
  pa.n_nets = d->n_nets;
  pa.G = d->n_gates;
  pa.B = ev->B;
  pa.S = ev->S;
  pa.paired = ev->paired_sizes;
  pa.partial = ev->power_partial.as<double>();
  pa.n_chunks = dp::power_chunks(d->n_nets);
  pa.power = ev->power.as<float>();
  DP_HIP_TRY(dp::launch_power(pa, s));
  return DP_OK;
}

// Output helper: a caller pointer, or a staging buffer copied out later.
struct OutMap {
  dp_eval *ev;
  int on_device;
  int slot = 0;
  struct Copy { void *dst; const void *src; size_t bytes; };
  std::vector<Copy> copies;
  template <class T>
  dp_status map(T *user, size_t count, T **dev) {
    *dev = nullptr;
    if (!user) return DP_OK;
    if (on_device) {
      *dev = user;
      return DP_OK;
    }
    DevBuf &b = ev->stage[slot++ % 8];
    DP_TRY(b.alloc(std::max<size_t>(count * sizeof(T), 16)));
    *dev = b.as<T>();
    copies.push_back({user, b.ptr, count * sizeof(T)});
    return DP_OK;
  }
  dp_status flush(hipStream_t s) {
    for (auto &c : copies)
      DP_HIP_TRY(hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyDeviceToHost, s));
    if (!on_device && !copies.empty()) DP_HIP_TRY(hipStreamSynchronize(s));
    return DP_OK;
  }
};

// Capture what `enqueue` puts on the eval's stream into *exec.  The capture
// runs on a private stream (the caller's stream may be the null stream,
// which cannot be captured); the graph is then launched on the caller's
// stream.  An older graph in *exec is destroyed once the stream drains.
template <class F>
dp_status capture_into(dp_eval *ev, hipGraphExec_t *exec, F &&enqueue) {
  if (!ev->capture_stream_owned)
    DP_HIP_TRY(hipStreamCreateWithFlags(&ev->capture_stream_owned, hipStreamNonBlocking));
  if (*exec) {
    DP_HIP_TRY(hipStreamSynchronize(ev->stream()));  // no launch of the old graph in flight
    (void)hipGraphExecDestroy(*exec);
    *exec = nullptr;
  }
  hipStream_t s = ev->capture_stream_owned;
  DP_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  const bool prof = ev->profiling;
  ev->profiling = false;
  ev->capturing = true;  // stream() is the capture stream meanwhile
  dp_status st = enqueue();
  ev->capturing = false;
  ev->profiling = prof;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(s, &graph);
  if (st != DP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return fail(DP_E_HIP, std::string("graph capture failed: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *exec = nullptr;
    return fail(DP_E_HIP, std::string("graph instantiate failed: ") + hipGetErrorString(e));
  }
  return DP_OK;
}

// Capture the forward sweep into ev->graph_fwd.
dp_status capture_forward(dp_eval *ev, const ChunkPlan *pl, uint64_t key) {
  DP_TRY(capture_into(ev, &ev->graph_fwd, [&]() { return enqueue_forward(ev, pl); }));
  ev->graph_key = key;
  return DP_OK;
}

uint64_t graph_key(const dp_eval *ev, const ChunkPlan *pl) {
  uint64_t k = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { k = (k ^ v) * 1099511628211ull; };
  mix((uint64_t)ev->prm.mode);
  mix((uint64_t)ev->prm.beta_grad);
  mix((uint64_t)ev->prm.n_sim);
  mix(ev->prm.seed);
  uint64_t bits;
  double kap = kappa_of(ev->prm);
  std::memcpy(&bits, &kap, 8); mix(bits);
  std::memcpy(&bits, &ev->prm.beta_min, 8); mix(bits);
  std::memcpy(&bits, &ev->prm.beta_max, 8); mix(bits);
  mix((uint64_t)ev->have_stim);
  mix((uint64_t)(uintptr_t)ev->stim.ptr);
  mix((uint64_t)markov(ev));
  mix((uint64_t)(uintptr_t)ev->mstim.ptr);
  mix((uint64_t)(uintptr_t)ev->tau.ptr);
  mix((uint64_t)ev->have_streams);
  mix((uint64_t)(uintptr_t)ev->streams.ptr);
  mix((uint64_t)(uintptr_t)ev->words.ptr);
  mix((uint64_t)(uintptr_t)ev->beta_frozen.ptr);
  mix((uint64_t)(uintptr_t)ev->size.ptr);
  mix((uint64_t)(uintptr_t)ev->stream());
  mix((uint64_t)ev->B);
  mix((uint64_t)ev->S);
  mix((uint64_t)ev->paired_sizes);
  mix((uint64_t)ev->beta_shared);
  if (pl) {
    mix((uint64_t)pl->Tc);
    mix((uint64_t)pl->cols);
    mix((uint64_t)pick_iters(ev, *pl));
    mix((uint64_t)n_sim_streams(ev));
  }
  return k;
}

// Copy the last forward's results out (caller numbering), on the eval's
// stream; host outputs are complete on return.
dp_status export_forward(dp_eval *ev, const dp_fwd_out *out, const ChunkPlan *pl) {
  const dp_design *d = ev->d;
  hipStream_t s = ev->stream();
  OutMap om{ev, out->on_device};
  const int64_t nb = (int64_t)d->n_nets * ev->B;
  dp::ExportArgs ea{};
  ea.sp = ev->sp.as<float>();
  ea.beta = beta_or_null(ev);
  ea.ones = pl ? ev->ones.as<uint32_t>() : nullptr;
  ea.tog = pl ? ev->tog.as<uint32_t>() : nullptr;
  ea.int2ext = d->int2ext.as<int32_t>();
  ea.T = pl ? pl->T : 0;
  ea.n_nets = d->n_nets;
  ea.B = ev->B;
  DP_TRY(om.map(out->sp, nb, &ea.o_sp));
  DP_TRY(om.map(out->tr, nb, &ea.o_tr));
  DP_TRY(om.map(out->sp_acc, nb, &ea.o_sp_acc));
  DP_TRY(om.map(out->tr_acc, nb, &ea.o_tr_acc));
  DP_TRY(om.map(out->beta, nb, &ea.o_beta));
  DP_TRY(om.map(out->tr_hyb, nb, &ea.o_tr_hyb));
  DP_TRY(om.map(out->ones, nb, &ea.o_ones));
  DP_TRY(om.map(out->toggles, nb, &ea.o_tog));
  if (ea.o_sp || ea.o_tr || ea.o_sp_acc || ea.o_tr_acc || ea.o_beta || ea.o_tr_hyb || ea.o_ones ||
      ea.o_tog)
    DP_HIP_TRY(dp::launch_export(ea, s));
  if (out->power) {
    const size_t bytes = (size_t)ev->B * s_prime(ev) * sizeof(float);
    DP_HIP_TRY(hipMemcpyAsync(out->power, ev->power.ptr, bytes,
                              out->on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
  }
  DP_TRY(om.flush(s));
  if (!out->on_device && out->power) DP_HIP_TRY(hipStreamSynchronize(s));
  return DP_OK;
}

// Arguments of the reverse sweep over C columns with upstream weights w
// (device, or null = 1).
dp::BwdArgs backward_args(dp_eval *ev, const float *w, int per_column, int32_t C) {
  const dp_design *d = ev->d;
  dp::BwdArgs ba{};
  ba.sp = ev->sp.as<float>();
  if (ev->beta_shared && ev->prm.mode == DP_FROZEN_BETA) {  // one beta per net (serving)
    ba.beta = ev->beta_frozen.as<float>();
    ba.beta_shared = 1;
  } else {
    ba.beta = beta_or_null(ev);
  }
  ba.cap = ev->cap.as<float>();
  ba.w = w;
  ba.size = ev->S > 0 ? ev->size.as<float>() : nullptr;
  ba.contrib = ev->contrib.as<float>();
  ba.kappa = (float)kappa_of(ev->prm);
  ba.n_pi = d->n_pi;
  ba.G = d->n_gates;
  ba.B = ev->B;
  ba.S = ev->S;
  ba.C = C;
  ba.cdiv = per_column ? s_prime(ev) : 1;
  ba.ste = ev->prm.beta_grad == DP_BETA_STE;
  ba.per_column = per_column;
  ba.paired = ev->paired_sizes;
  ba.fixed = ev->have_fixed ? ev->fixed.as<uint8_t>() : nullptr;
  return ba;
}

// Enqueue the reverse levels and the PI adjoints into dst [C][n_pi] (device)
// on the eval's stream; no allocation, no host synchronisation.
dp_status enqueue_backward(dp_eval *ev, const dp::BwdArgs &ba, float *dst) {
  const dp_design *d = ev->d;
  hipStream_t s = ev->stream();
  const dp::GraphView g = view(d);
  double bwd_bytes = 0.0;
  for (int32_t l = d->depth; l >= 1; --l) bwd_bytes += bwd_level_bytes(d, l, ba.C);
  if (ev->schedule == DP_SCHED_PERSISTENT) {
    dp::GridBarrier bar;
    DP_TRY(grid_barrier(ev, &bar));
    SpanGuard sg(ev, SPAN_BWD, bwd_bytes, ev->profiling && d->depth > 0, d->depth);
    return on_coop_stream(ev, s, [&](hipStream_t cs) {
      return dp::launch_bwd_persistent(g, ba, d->level_dev.as<int32_t>(), d->depth,
                                       (int64_t)d->max_level_width * ba.C, dst, bar, cs);
    });
  }
  {
    SpanGuard sg(ev, SPAN_BWD, bwd_bytes, ev->profiling && d->depth > 0, d->depth + d->split_levels);
    for (int32_t l = d->depth; l >= 1; --l)
      DP_TRY(for_level_parts(d, l, [&](int32_t g0, int32_t n, bool cells) -> dp_status {
        const dp::HeavySpan hs = dp::heavy_span(d, g0, n);
        DP_HIP_TRY(dp::launch_bwd_level(g, ba, g0, n, cells, s, hs.gates, hs.n));
        return DP_OK;
      }));
  }
  const dp::HeavySpan hp = dp::heavy_pis(d);
  DP_HIP_TRY(dp::launch_bwd_pi(g, ba, dst, s, hp.gates, hp.n));
  return DP_OK;
}

// Every argument the reverse sweep's launches take (a captured sweep is
// replayed only while all of them are unchanged).
uint64_t reverse_key(const dp_eval *ev, const dp::BwdArgs &ba, const float *dst) {
  uint64_t k = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { k = (k ^ v) * 1099511628211ull; };
  for (const void *ptr : {(const void *)ba.sp, (const void *)ba.beta, (const void *)ba.cap,
                          (const void *)ba.w, (const void *)ba.size, (const void *)ba.contrib,
                          (const void *)ba.lam, (const void *)ba.fixed, (const void *)dst,
                          (const void *)ev->stream()})
    mix((uint64_t)(uintptr_t)ptr);
  uint32_t kb;
  std::memcpy(&kb, &ba.kappa, 4);
  mix(kb);
  for (int32_t v : {ba.n_pi, ba.G, ba.B, ba.S, ba.C, ba.cdiv, ba.ste, ba.per_column, ba.paired,
                    ba.beta_shared})
    mix((uint64_t)(uint32_t)v);
  return k;
}

// The reverse sweep of run_backward: under DP_SCHED_GRAPH captured once
// into ev->graph_bwd (re-captured when any launch argument changes) and
// replayed, otherwise enqueued launch by launch.
dp_status reverse_sweep(dp_eval *ev, const dp::BwdArgs &ba, float *dst) {
  const dp_design *d = ev->d;
  const int64_t launches = (int64_t)d->depth + d->split_levels + 1;
  if (ev->schedule != DP_SCHED_GRAPH || ev->profiling || launches > kMaxGraphLaunches)
    return enqueue_backward(ev, ba, dst);
  const uint64_t k = reverse_key(ev, ba, dst);
  if (!ev->graph_bwd || ev->graph_bwd_key != k) {
    DP_TRY(capture_into(ev, &ev->graph_bwd, [&]() { return enqueue_backward(ev, ba, dst); }));
    ev->graph_bwd_key = k;
  }
  DP_HIP_TRY(hipGraphLaunch(ev->graph_bwd, ev->stream()));
  return DP_OK;
}

}  // namespace

namespace dp {
dp_status params_ok(const dp_params *p) { return check_params(p); }
double kappa(const dp_params &p) { return kappa_of(p); }
}  // namespace dp

dp_eval::~dp_eval() {
  if (graph_fwd) (void)hipGraphExecDestroy(graph_fwd);
  if (graph_bwd) (void)hipGraphExecDestroy(graph_bwd);
  if (graph_fb) (void)hipGraphExecDestroy(graph_fb);
  if (capture_stream_owned) (void)hipStreamDestroy(capture_stream_owned);
  if (coop_stream) {
    (void)hipStreamSynchronize(coop_stream);
    (void)hipStreamDestroy(coop_stream);
  }
  for (auto e : coop_events)
    if (e) (void)hipEventDestroy(e);
  for (auto e : ev_pool) (void)hipEventDestroy(e);
  for (auto st : lane_streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto e : lane_events) (void)hipEventDestroy(e);
}

// =========================================================================
extern "C" {

void dp_params_default(dp_params *p) {
  if (!p) return;
  p->vdd = 1.0;
  p->fclk = 1.0;
  p->energy_factor = 0.5;
  p->beta_min = 0.1;
  p->beta_max = 10.0;
  p->mode = DP_MODELED;
  p->beta_grad = DP_BETA_LOCAL;
  p->n_sim = 4096;
  p->seed = 1;
}

const char *dp_last_error(void) { return dp::g_err.c_str(); }
const char *dp_version(void) { return kVersion; }

dp_status dp_ctx_create(int32_t device, void *hip_stream, dp_ctx **out) {
  if (!out) return fail(DP_E_INVALID, "dp_ctx_create: NULL out");
  int n = 0;
  DP_HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n)
    return fail(DP_E_INVALID, "dp_ctx_create: no device " + std::to_string(device));
  DP_HIP_TRY(hipSetDevice(device));
  DP_TRY(dp::static_scratch_init(device));  // once per device: dp_forward_static's scratch
  auto *c = new dp_ctx();
  c->device = device;
  if (hip_stream == (void *)hipStreamLegacy) {
    c->stream = nullptr;  // the null stream
  } else if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->owned, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(DP_E_HIP, std::string("hipStreamCreate failed: ") + hipGetErrorString(e));
    }
    c->stream = c->owned;
  }
  *out = c;
  return DP_OK;
}

dp_status dp_ctx_set_stream(dp_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(DP_E_INVALID, "dp_ctx_set_stream: NULL ctx");
  if (hip_stream == (void *)hipStreamLegacy) {
    ctx->stream = nullptr;  // the null stream
    return DP_OK;
  }
  if (!hip_stream && !ctx->owned) {
    DP_HIP_TRY(hipSetDevice(ctx->device));
    DP_HIP_TRY(hipStreamCreateWithFlags(&ctx->owned, hipStreamNonBlocking));
  }
  ctx->stream = hip_stream ? (hipStream_t)hip_stream : ctx->owned;
  return DP_OK;
}

dp_status dp_ctx_synchronize(dp_ctx *ctx) {
  if (!ctx) return fail(DP_E_INVALID, "dp_ctx_synchronize: NULL ctx");
  DP_HIP_TRY(hipStreamSynchronize(ctx->stream));
  return DP_OK;
}

void dp_ctx_destroy(dp_ctx *ctx) {
  if (ctx) dp::ctx_release(ctx);
}

dp_status dp_compile(dp_ctx *ctx, const dp_netlist *netlist, dp_design **out) {
  if (ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(DP_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  return dp::compile_design(ctx, netlist, 0, nullptr, nullptr, out);
}

dp_status dp_compile_cells(dp_ctx *ctx, const dp_netlist *netlist, int32_t n_cells,
                           const char *const *cells, dp_design **out) {
  if (ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(DP_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  return dp::compile_design(ctx, netlist, n_cells, cells, nullptr, out);
}

dp_status dp_compile_library(dp_ctx *ctx, const dp_netlist *netlist, int32_t n_cells,
                             const char *const *cells, const char *const *pins,
                             dp_design **out) {
  if (ctx) {
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return fail(DP_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  }
  return dp::compile_design(ctx, netlist, n_cells, cells, pins, out);
}

dp_status dp_design_cell_logic(const dp_design *d, int32_t *logic, int32_t *n_logic) {
  if (!d) return fail(DP_E_INVALID, "dp_design_cell_logic: NULL design");
  if (logic && !d->h_cell_logic.empty())
    std::memcpy(logic, d->h_cell_logic.data(), sizeof(int32_t) * d->h_cell_logic.size());
  if (n_logic) *n_logic = d->n_cells;
  return DP_OK;
}

dp_status dp_design_info(const dp_design *d, dp_design_info_t *out) {
  if (!d || !out) return fail(DP_E_INVALID, "dp_design_info: NULL argument");
  out->n_pi = d->n_pi;
  out->n_gates = d->n_gates;
  out->n_nets = d->n_nets;
  out->depth = d->depth;
  out->n_edges = d->n_edges;
  out->max_level_width = d->max_level_width;
  out->reserved = 0;
  out->device_bytes = d->device_bytes;
  return DP_OK;
}

dp_status dp_design_levels(const dp_design *d, int32_t *level) {
  if (!d || !level) return fail(DP_E_INVALID, "dp_design_levels: NULL argument");
  std::memcpy(level, d->h_level.data(), sizeof(int32_t) * d->n_nets);
  return DP_OK;
}

void dp_design_destroy(dp_design *d) {
  if (d) dp::design_release(d);
}

dp_status dp_eval_create(dp_design *d, int32_t n_cols, int32_t n_size, const dp_params *params,
                         dp_eval **out) {
  if (!d || !out) return fail(DP_E_INVALID, "dp_eval_create: NULL argument");
  if (n_cols < 1 || n_size < 0) return fail(DP_E_INVALID, "dp_eval_create: need B >= 1, S >= 0");
  DP_TRY(check_params(params));
  DP_HIP_TRY(hipSetDevice(d->ctx->device));
  auto *ev = new dp_eval();
  ev->d = d;
  ev->B = n_cols;
  ev->S = n_size;
  ev->prm = *params;
  dp_status st = ev->sp.alloc((size_t)d->n_nets * n_cols * sizeof(float));
  if (st == DP_OK) st = ev->cap.alloc((size_t)d->n_nets * sizeof(float));
  if (st == DP_OK && n_size > 0) st = ev->size.alloc((size_t)n_size * d->n_gates * sizeof(float));
  if (st != DP_OK) {
    delete ev;
    return st;
  }
  dp::design_retain(d);
  *out = ev;
  return DP_OK;
}

dp_status dp_eval_set_params(dp_eval *ev, const dp_params *params) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_set_params: NULL eval");
  DP_TRY(check_params(params));
  ev->prm = *params;
  ev->inputs_version++;
  return DP_OK;
}

void dp_eval_destroy(dp_eval *ev) {
  if (!ev) return;
  (void)hipStreamSynchronize(ev->stream());
  dp_design *d = ev->d;
  delete ev;
  dp::design_release(d);
}

dp_status dp_set_pi_prob(dp_eval *ev, const float *p, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_pi_prob: NULL eval");
  const dp_design *d = ev->d;
  const int64_t n = (int64_t)ev->B * d->n_pi;
  if (n == 0) {
    ev->have_pi = true;
    ev->inputs_version++;
    return DP_OK;
  }
  DP_TRY(check_values(ev, p, n, 0.0f, 1.0f, on_device, "dp_set_pi_prob"));
  hipStream_t s = ev->stream();
  DP_TRY(stage_in(ev->p_stage, p, n * sizeof(float), on_device, s));
  DP_HIP_TRY(dp::launch_load_pi(ev->p_stage.as<float>(), ev->sp.as<float>(), d->n_pi, ev->B, s));
  if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  ev->have_pi = true;
  ev->inputs_version++;
  return DP_OK;
}

dp_status dp_set_caps(dp_eval *ev, const float *cap, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_caps: NULL eval");
  const dp_design *d = ev->d;
  DP_TRY(check_values(ev, cap, d->n_nets, 0.0f, 3.0e38f, on_device, "dp_set_caps"));
  hipStream_t s = ev->stream();
  DP_TRY(stage_in(ev->cap_stage, cap, (size_t)d->n_nets * sizeof(float), on_device, s));
  DP_HIP_TRY(dp::launch_gather_nets_f32(ev->cap_stage.as<float>(), d->int2ext.as<int32_t>(),
                                        ev->cap.as<float>(), d->n_nets, s));
  if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  ev->have_cap = true;
  ev->inputs_version++;
  return DP_OK;
}

dp_status dp_set_cell_sizes(dp_eval *ev, const float *size, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_cell_sizes: NULL eval");
  if (ev->S == 0) return fail(DP_E_INVALID, "dp_set_cell_sizes: eval was created with S = 0");
  const dp_design *d = ev->d;
  const int64_t n = (int64_t)ev->S * d->n_gates;
  DP_TRY(check_values(ev, size, n, 0.0f, 3.0e38f, on_device, "dp_set_cell_sizes"));
  hipStream_t s = ev->stream();
  DP_TRY(stage_in(ev->size_stage, size, n * sizeof(float), on_device, s));
  DP_HIP_TRY(dp::launch_import_sizes(ev->size_stage.as<float>(), d->int2ext.as<int32_t>(),
                                     ev->size.as<float>(), d->n_pi, d->n_gates, ev->S, s));
  if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  ev->have_size = true;
  ev->inputs_version++;
  return DP_OK;
}

dp_status dp_set_beta(dp_eval *ev, const float *beta, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_beta: NULL eval");
  const dp_design *d = ev->d;
  const int64_t n = (int64_t)ev->B * d->n_nets;
  DP_TRY(check_values(ev, beta, n, 0.0f, 3.0e38f, on_device, "dp_set_beta"));
  hipStream_t s = ev->stream();
  DP_TRY(ev->beta_frozen.alloc(n * sizeof(float)));
  DP_TRY(stage_in(ev->beta_stage, beta, n * sizeof(float), on_device, s));
  DP_HIP_TRY(dp::launch_import_cols_f32(ev->beta_stage.as<float>(), d->int2ext.as<int32_t>(),
                                        ev->beta_frozen.as<float>(), d->n_nets, ev->B, s));
  if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  ev->have_beta = true;
  ev->inputs_version++;
  return DP_OK;
}

dp_status dp_set_stimulus(dp_eval *ev, const uint64_t *words, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_stimulus: NULL eval");
  ev->inputs_version++;
  if (!words) {
    ev->have_stim = false;
    return DP_OK;
  }
  const dp_design *d = ev->d;
  const int64_t T = n_words(ev->prm);
  if (T <= 0) return fail(DP_E_INVALID, "dp_set_stimulus: params.n_sim is 0");
  const size_t bytes = (size_t)ev->B * d->n_pi * T * sizeof(uint64_t);
  hipStream_t s = ev->stream();
  DP_TRY(stage_in(ev->stim, words, bytes, on_device, s));
  if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  ev->have_stim = true;
  return DP_OK;
}

dp_status dp_set_pi_rates(dp_eval *ev, const float *tau, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_pi_rates: NULL eval");
  ev->inputs_version++;
  if (!tau) {
    ev->have_tau = false;
    return DP_OK;
  }
  const int64_t n = (int64_t)ev->B * ev->d->n_pi;
  if (n > 0) {
    DP_TRY(check_values(ev, tau, n, 0.0f, 1.0f, on_device, "dp_set_pi_rates"));
    hipStream_t s = ev->stream();
    DP_TRY(stage_in(ev->tau, tau, (size_t)n * sizeof(float), on_device, s));
    if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  }
  ev->have_tau = true;
  return DP_OK;
}

dp_status dp_set_pi_streams(dp_eval *ev, const int32_t *stream) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_pi_streams: NULL eval");
  ev->inputs_version++;
  if (!stream) {
    ev->have_streams = false;
    return DP_OK;
  }
  const int32_t n_pi = ev->d->n_pi;
  for (int32_t i = 0; i < n_pi; ++i)
    if (stream[i] < 0 || stream[i] >= n_pi)
      return fail(DP_E_INVALID, "dp_set_pi_streams: stream " + std::to_string(stream[i]) +
                                    " of PI " + std::to_string(i) + " is not a PI");
  if (n_pi > 0) {
    hipStream_t s = ev->stream();
    DP_TRY(stage_in(ev->streams, stream, (size_t)n_pi * sizeof(int32_t), 0, s));
    DP_HIP_TRY(hipStreamSynchronize(s));
  }
  ev->have_streams = true;
  return DP_OK;
}

dp_status dp_set_pi_fixed(dp_eval *ev, const uint8_t *fixed) {
  if (!ev) return fail(DP_E_INVALID, "dp_set_pi_fixed: NULL eval");
  ev->have_fixed = false;  // read by the reverse sweep only: the forward stays valid
  const int32_t n_pi = ev->d->n_pi;
  if (!fixed || n_pi == 0) return DP_OK;
  hipStream_t s = ev->stream();
  DP_TRY(stage_in(ev->fixed, fixed, (size_t)n_pi, 0, s));
  DP_HIP_TRY(hipStreamSynchronize(s));
  ev->have_fixed = true;
  return DP_OK;
}

dp_status dp_eval_set_schedule(dp_eval *ev, int32_t schedule, int64_t words_per_chunk,
                               int32_t sim_pairs_per_lane) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_set_schedule: NULL eval");
  if (schedule < DP_SCHED_AUTO || schedule > DP_SCHED_PERSISTENT)
    return fail(DP_E_INVALID, "dp_eval_set_schedule: unknown schedule");
  if (words_per_chunk < 0 || (words_per_chunk > 0 && words_per_chunk < 2))
    return fail(DP_E_INVALID, "dp_eval_set_schedule: words_per_chunk must be 0 or >= 2");
  if (!(sim_pairs_per_lane == 0 || sim_pairs_per_lane == 1 || sim_pairs_per_lane == 2 ||
        sim_pairs_per_lane == 4 || sim_pairs_per_lane == 8))
    return fail(DP_E_INVALID, "dp_eval_set_schedule: sim_pairs_per_lane must be 0, 1, 2, 4 or 8");
  if (schedule == DP_SCHED_PERSISTENT && ev->d->has_cell_gates)
    return fail(DP_E_UNSUPPORTED,
                "dp_eval_set_schedule: the persistent schedule runs the fixed cells only");
  if (schedule == DP_SCHED_PERSISTENT && !ev->barrier.ptr) {
    DP_TRY(ev->barrier.alloc(dp::kBarrierAlloc * sizeof(uint32_t)));
    DP_HIP_TRY(dp::launch_fill_u32(ev->barrier.as<uint32_t>(), dp::kBarrierAlloc, 0u, ev->stream()));
  }
  ev->schedule = schedule;
  ev->words_per_chunk = words_per_chunk;
  ev->sim_iters = sim_pairs_per_lane;
  return DP_OK;
}

static dp_status run_backward(dp_eval *ev, const float *grad_power, int per_column,
                              float *dpi, float *dcap, float *dsize, int32_t on_device);

dp_status dp_eval_autotune(dp_eval *ev, int32_t reps, int32_t with_backward, double *best_ms) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_autotune: NULL eval");
  if (reps < 1) reps = 1;
  const int32_t s0 = ev->schedule, i0 = ev->sim_iters, l0 = ev->sim_streams;
  const int64_t c0 = ev->words_per_chunk;
  const bool prof = ev->profiling;
  ev->profiling = false;
  struct Cand { int32_t sched; int32_t iters; int64_t chunk; int32_t lanes; };
  std::vector<Cand> cands;
  const int64_t T = n_words(ev->prm);
  if (hybrid(ev)) {
    const int64_t chunks[3] = {0, (T / 2 + 1) & ~1ll, (T / 4 + 1) & ~1ll};
    for (int k = 0; k < 3; ++k) {
      if (k > 0 && chunks[k] < 128) continue;
      for (int32_t lanes : {1, 2, 4}) {
        const int64_t keep_chunk = ev->words_per_chunk;
        const int32_t keep_lanes = ev->sim_streams;
        ev->words_per_chunk = chunks[k];
        ev->sim_streams = lanes;
        const ChunkPlan cp = plan_chunks(ev);
        ev->words_per_chunk = keep_chunk;
        ev->sim_streams = keep_lanes;
        const int64_t pieces = (int64_t)cp.n_groups * cp.n_chunks;  // independent pieces
        if (lanes > 1 && lanes > pieces) continue;
        if ((int64_t)lanes * ev->d->n_nets * 8 * (k == 0 ? T : chunks[k] + 2) > kAutoWordBudget)
          continue;
        for (int32_t it : {1, 2, 4, 8})
          for (int32_t sc : {DP_SCHED_LEVEL, DP_SCHED_GRAPH}) cands.push_back({sc, it, chunks[k], lanes});
      }
    }
  } else {
    for (int32_t sc : {DP_SCHED_LEVEL, DP_SCHED_GRAPH}) cands.push_back({sc, 0, 0, 1});
  }
  DevBuf bwd_out;  // scratch for the timed reverse sweeps
  if (with_backward) DP_TRY(bwd_out.alloc((size_t)ev->B * std::max(ev->d->n_pi, 1) * 4));
  hipStream_t s = ev->stream();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  DP_HIP_TRY(hipEventCreate(&e0));
  DP_HIP_TRY(hipEventCreate(&e1));
  double best = 1e300;
  Cand win{s0, i0, c0, l0};
  dp_status st = DP_OK;
  for (const Cand &c : cands) {
    ev->schedule = c.sched;
    ev->sim_iters = c.iters;
    ev->words_per_chunk = c.chunk;
    ev->sim_streams = c.lanes;
    if (c.sched == DP_SCHED_GRAPH) {
      if (c.lanes > 1) continue;  // a graph is captured on one stream: same as lanes = 1
      ChunkPlan cp;
      if (hybrid(ev)) cp = plan_chunks(ev);
      if (forward_launches(ev, hybrid(ev) ? &cp : nullptr) > kMaxGraphLaunches) continue;
    }
    auto once = [&]() -> dp_status {
      dp_status r = dp_forward(ev, nullptr);
      if (r == DP_OK && with_backward)
        r = run_backward(ev, nullptr, 0, bwd_out.as<float>(), nullptr, nullptr, 1);
      return r;
    };
    if ((st = once()) != DP_OK) break;  // warm-up, graph capture
    if (hipEventRecord(e0, s) != hipSuccess) { st = fail(DP_E_HIP, "autotune: event"); break; }
    for (int32_t r = 0; r < reps && st == DP_OK; ++r) st = once();
    if (st != DP_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(DP_E_HIP, "autotune: event timing failed");
      break;
    }
    if (ms / reps < best) {
      best = ms / reps;
      win = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ev->profiling = prof;
  ev->schedule = win.sched;
  ev->sim_iters = win.iters;
  ev->words_per_chunk = win.chunk;
  ev->sim_streams = win.lanes;
  if (st != DP_OK) return st;
  if (best_ms) *best_ms = best;
  return DP_OK;
}

dp_status dp_eval_set_sim_streams(dp_eval *ev, int32_t sim_streams) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_set_sim_streams: NULL eval");
  if (sim_streams < 0 || sim_streams > 16)
    return fail(DP_E_INVALID, "dp_eval_set_sim_streams: need 0 <= sim_streams <= 16");
  ev->sim_streams = sim_streams;
  return DP_OK;
}

dp_status dp_eval_set_sim_columns(dp_eval *ev, int32_t columns) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_set_sim_columns: NULL eval");
  if (columns < 0) return fail(DP_E_INVALID, "dp_eval_set_sim_columns: need columns >= 0");
  ev->sim_cols = columns;
  return DP_OK;
}

dp_status dp_eval_get_schedule(const dp_eval *ev, int32_t *schedule, int64_t *words_per_chunk,
                               int32_t *sim_pairs_per_lane, int32_t *sim_streams) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_get_schedule: NULL eval");
  if (schedule) *schedule = ev->schedule;
  if (words_per_chunk) *words_per_chunk = ev->words_per_chunk;
  if (sim_pairs_per_lane) *sim_pairs_per_lane = ev->sim_iters;
  if (sim_streams) *sim_streams = n_sim_streams(ev);
  return DP_OK;
}

dp_status dp_eval_synchronize(dp_eval *ev) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_synchronize: NULL eval");
  DP_HIP_TRY(hipSetDevice(ev->d->ctx->device));
  DP_HIP_TRY(hipStreamSynchronize(ev->stream()));
  return barrier_status(ev);
}

dp_status dp_eval_set_barrier_timeout(dp_eval *ev, double microseconds) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_set_barrier_timeout: NULL eval");
  if (!(microseconds >= 0.0) || !std::isfinite(microseconds))
    return fail(DP_E_INVALID, "dp_eval_set_barrier_timeout: need a finite time >= 0");
  ev->barrier_limit_us = microseconds;
  return DP_OK;
}

dp_status dp_eval_profile(dp_eval *ev, int32_t enable) {
  if (!ev) return fail(DP_E_INVALID, "dp_eval_profile: NULL eval");
  ev->profiling = enable != 0;
  ev->prof = dp_profile{};
  return DP_OK;
}

dp_status dp_eval_get_profile(dp_eval *ev, dp_profile *out) {
  if (!ev || !out) return fail(DP_E_INVALID, "dp_eval_get_profile: NULL argument");
  DP_TRY(resolve_profile(ev));
  *out = ev->prof;
  return DP_OK;
}

dp_status dp_forward(dp_eval *ev, const dp_fwd_out *out) {
  if (!ev) return fail(DP_E_INVALID, "dp_forward: NULL eval");
  const dp_design *d = ev->d;
  if (!ev->have_pi) return fail(DP_E_STATE, "dp_forward: PI probabilities not set");
  if (!ev->have_cap) return fail(DP_E_STATE, "dp_forward: capacitances not set");
  if (ev->S > 0 && !ev->have_size) return fail(DP_E_STATE, "dp_forward: cell sizes not set");
  if (ev->prm.mode == DP_FROZEN_BETA && !ev->have_beta)
    return fail(DP_E_STATE, "dp_forward: DP_FROZEN_BETA needs dp_set_beta");
  const bool hyb = hybrid(ev);
  if (out && !hyb && (out->sp_acc || out->tr_acc || out->ones || out->toggles))
    return fail(DP_E_INVALID, "dp_forward: simulation outputs need DP_HYBRID");
  if (hyb && ev->have_stim &&
      ev->stim.bytes < (size_t)ev->B * d->n_pi * n_words(ev->prm) * sizeof(uint64_t))
    return fail(DP_E_STATE, "dp_forward: the explicit stimulus is shorter than n_sim/64 words");
  DP_HIP_TRY(hipSetDevice(d->ctx->device));
  hipStream_t s = ev->stream();
  ChunkPlan plan;
  if (hyb) plan = plan_chunks(ev);
  const ChunkPlan *pl = hyb ? &plan : nullptr;
  DP_TRY(ensure_forward_buffers(ev, pl));
  if (ev->schedule == DP_SCHED_GRAPH && forward_launches(ev, pl) > kMaxGraphLaunches)
    return fail(DP_E_UNSUPPORTED, "dp_forward: the sweep has " +
                std::to_string(forward_launches(ev, pl)) + " launches, more than the " +
                std::to_string(kMaxGraphLaunches) + " a graph may hold; use DP_SCHED_LEVEL");
  const bool use_graph = ev->schedule == DP_SCHED_GRAPH && !ev->profiling;
  if (use_graph) {
    const uint64_t key = graph_key(ev, pl);
    if (!ev->graph_fwd || ev->graph_key != key) DP_TRY(capture_forward(ev, pl, key));
    DP_HIP_TRY(hipGraphLaunch(ev->graph_fwd, s));
  } else {
    DP_TRY(enqueue_forward(ev, pl));
  }
  ev->fwd_version = ev->inputs_version;
  if (out) DP_TRY(export_forward(ev, out, pl));
  if (out && !out->on_device) DP_TRY(sync_and_check(ev));
  return DP_OK;
}

static dp_status run_backward(dp_eval *ev, const float *grad_power, int per_column,
                              float *dpi, float *dcap, float *dsize, int32_t on_device) {
  const dp_design *d = ev->d;
  if (ev->fwd_version != ev->inputs_version || ev->fwd_version == 0)
    return fail(DP_E_STATE, "dp_backward: no completed forward for the current inputs");
  DP_HIP_TRY(hipSetDevice(d->ctx->device));
  hipStream_t s = ev->stream();
  const int32_t Sp = s_prime(ev);
  const int32_t cols = ev->B * Sp;
  const int32_t C = per_column ? cols : ev->B;
  const float *w = nullptr;
  if (grad_power) {
    DP_TRY(check_values(ev, grad_power, cols, -3.0e38f, 3.0e38f, on_device, "dp_backward grad"));
    DP_TRY(stage_in(ev->w, grad_power, (size_t)cols * sizeof(float), on_device, s));
    w = ev->w.as<float>();
  }
  if (dpi) {
    DP_TRY(ev->contrib.alloc(std::max<size_t>((size_t)d->n_edges * C * sizeof(float), 16)));
    const dp::BwdArgs ba = backward_args(ev, w, per_column, C);
    float *dst = dpi;
    const size_t bytes = (size_t)C * d->n_pi * sizeof(float);
    if (!on_device) {
      DP_TRY(ev->pi_out.alloc(std::max<size_t>(bytes, 16)));
      dst = ev->pi_out.as<float>();
    }
    DP_TRY(reverse_sweep(ev, ba, dst));
    if (!on_device && bytes)
      DP_HIP_TRY(hipMemcpyAsync(dpi, dst, bytes, hipMemcpyDeviceToHost, s));
  }
  if (dcap || (dsize && ev->S > 0)) {
    OutMap om{ev, on_device};
    dp::GradExportArgs ga{};
    ga.sp = ev->sp.as<float>();
    ga.beta = beta_or_null(ev);
    ga.beta_shared = ev->beta_shared && ev->prm.mode == DP_FROZEN_BETA;
    if (ga.beta_shared) ga.beta = ev->beta_frozen.as<float>();
    ga.kappa = (float)kappa_of(ev->prm);
    ga.cap = ev->cap.as<float>();
    ga.w = w;
    ga.size = ev->S > 0 ? ev->size.as<float>() : nullptr;
    ga.int2ext = d->int2ext.as<int32_t>();
    ga.n_pi = d->n_pi;
    ga.n_nets = d->n_nets;
    ga.G = d->n_gates;
    ga.B = ev->B;
    ga.S = ev->S;
    ga.paired = ev->paired_sizes;
    DP_TRY(om.map(dcap, (size_t)d->n_nets, &ga.dcap));
    if (ev->S > 0) DP_TRY(om.map(dsize, (size_t)ev->S * d->n_gates, &ga.dsize));
    DP_HIP_TRY(dp::launch_grad_export(ga, s));
    DP_TRY(om.flush(s));
  }
  if (!on_device) DP_TRY(sync_and_check(ev));
  if (!on_device) DP_HIP_TRY(hipStreamSynchronize(s));
  return DP_OK;
}

dp_status dp_backward(dp_eval *ev, const float *grad_power, float *dpower_dpi, float *dpower_dcap,
                      float *dpower_dsize, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_backward: NULL eval");
  if (dpower_dsize && ev->S == 0)
    return fail(DP_E_INVALID, "dp_backward: dpower_dsize needs cell sizes (S > 0)");
  return run_backward(ev, grad_power, 0, dpower_dpi, dpower_dcap, dpower_dsize, on_device);
}

dp_status dp_power_gradients(dp_eval *ev, float *dpower_dsp, float *score, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_power_gradients: NULL eval");
  const dp_design *d = ev->d;
  if (ev->fwd_version != ev->inputs_version || ev->fwd_version == 0)
    return fail(DP_E_STATE, "dp_power_gradients: no completed forward for the current inputs");
  if (!dpower_dsp && !score) return DP_OK;
  DP_HIP_TRY(hipSetDevice(d->ctx->device));
  hipStream_t s = ev->stream();
  const int32_t B = ev->B;
  DP_TRY(ev->contrib.alloc(std::max<size_t>((size_t)d->n_edges * B * sizeof(float), 16)));
  DP_TRY(ev->pi_out.alloc(std::max<size_t>((size_t)B * d->n_pi * sizeof(float), 16)));
  DevBuf lam;
  DP_TRY(lam.alloc((size_t)B * d->n_nets * sizeof(float)));
  dp::BwdArgs ba = backward_args(ev, nullptr, 0, B);
  ba.lam = lam.as<float>();
  DP_TRY(enqueue_backward(ev, ba, ev->pi_out.as<float>()));
  OutMap om{ev, on_device};
  float *o_lam = nullptr, *o_score = nullptr;
  DP_TRY(om.map(dpower_dsp, (size_t)B * d->n_nets, &o_lam));
  DP_TRY(om.map(score, (size_t)B * d->n_gates, &o_score));
  DP_HIP_TRY(dp::launch_grad_lambda_export(lam.as<float>(), ev->sp.as<float>(),
                                           d->int2ext.as<int32_t>(), d->n_pi, d->n_nets, B, B, 1,
                                           0x1p-20f, o_lam, o_score, s));
  DP_TRY(om.flush(s));
  DP_HIP_TRY(hipStreamSynchronize(s));  // the adjoint buffer is freed on return
  return barrier_status(ev);
}

dp_status dp_power_virus(dp_eval *ev, int32_t steps, double eta, uint8_t *v0, float *p_final,
                         double *p_virus, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_power_virus: NULL eval");
  if (steps < 0 || !std::isfinite(eta))
    return fail(DP_E_INVALID, "dp_power_virus: need steps >= 0 and a finite eta");
  if (ev->prm.mode == DP_HYBRID)
    return fail(DP_E_UNSUPPORTED, "dp_power_virus: the ascent runs DP_MODELED or DP_FROZEN_BETA");
  if (ev->S > 0) return fail(DP_E_UNSUPPORTED, "dp_power_virus: size vectors are not supported");
  if (!ev->have_pi) return fail(DP_E_STATE, "dp_power_virus: start probabilities not set");
  if (!ev->have_cap) return fail(DP_E_STATE, "dp_power_virus: capacitances not set");
  if (ev->prm.mode == DP_FROZEN_BETA && !ev->have_beta)
    return fail(DP_E_STATE, "dp_power_virus: DP_FROZEN_BETA needs dp_set_beta");
  const dp_design *d = ev->d;
  DP_HIP_TRY(hipSetDevice(d->ctx->device));
  hipStream_t s = ev->stream();
  const int32_t B = ev->B;
  const size_t nb = (size_t)d->n_nets * B, pb = (size_t)d->n_pi * B;
  DP_TRY(ensure_forward_buffers(ev, nullptr));
  DP_TRY(ev->contrib.alloc(std::max<size_t>((size_t)d->n_edges * B * sizeof(float), 16)));
  DP_TRY(ev->pi_out.alloc(std::max<size_t>(pb * sizeof(float), 16)));
  // the proxy is the power without kappa: upstream weight 1 / kappa per column
  DP_TRY(ev->w.alloc(std::max<size_t>((size_t)B * sizeof(float), 16)));
  DP_HIP_TRY(dp::launch_fill_f32(ev->w.as<float>(), B, (float)(1.0 / kappa_of(ev->prm)), s));
  const dp::BwdArgs ba = backward_args(ev, ev->w.as<float>(), 0, B);
  for (int32_t t = 0; t < steps; ++t) {
    DP_TRY(enqueue_forward(ev, nullptr));
    DP_TRY(enqueue_backward(ev, ba, ev->pi_out.as<float>()));
    DP_HIP_TRY(dp::launch_virus_step(ev->sp.as<float>(), ev->pi_out.as<float>(), (float)eta,
                                     d->n_pi, B, s));
  }
  // v0, v1 = 1 - v0 and a two-cycle bit-parallel simulation of the pair
  DevBuf stim, words, v0_dev, p_dev, pv;
  DP_TRY(stim.alloc(std::max<size_t>(pb * 2 * sizeof(uint64_t), 16)));
  DP_TRY(words.alloc((size_t)B * d->n_nets * 2 * sizeof(uint64_t)));
  DP_TRY(v0_dev.alloc(std::max<size_t>(pb, 16)));
  DP_TRY(p_dev.alloc(std::max<size_t>(pb * sizeof(float), 16)));
  DP_TRY(pv.alloc(std::max<size_t>((size_t)B * sizeof(double), 16)));
  DP_TRY(ev->ones.alloc(nb * sizeof(uint32_t)));
  DP_TRY(ev->tog.alloc(nb * sizeof(uint32_t)));
  DP_HIP_TRY(dp::launch_virus_vectors(ev->sp.as<float>(), stim.as<uint64_t>(), v0_dev.as<uint8_t>(),
                                      p_dev.as<float>(), d->n_pi, B, s));
  DP_HIP_TRY(dp::launch_fill_u32(ev->ones.as<uint32_t>(), (int64_t)nb, 0u, s));
  DP_HIP_TRY(dp::launch_fill_u32(ev->tog.as<uint32_t>(), (int64_t)nb, 0u, s));
  const dp::GraphView g = view(d);
  const dp::SimTune tune{1};
  dp::ChunkView cv{};  // every column's pair in one launch per level
  cv.W = words.as<uint64_t>();
  cv.pitch = 2;
  cv.col_stride = (int64_t)d->n_nets * 2;
  cv.t_first = 0;
  cv.pairs = 1;
  cv.u_lo = 0;
  cv.u_hi = 2;
  cv.u_tog_lo = 1;
  cv.n_cols = B;
  const dp::CountView cnt{ev->ones.as<uint32_t>(), ev->tog.as<uint32_t>(), B, 0};
  DP_HIP_TRY(dp::launch_stimulus(g, cv, cnt, ev->sp.as<float>(), stim.as<uint64_t>(), 2, nullptr,
                                 0, tune, s));
  for (int32_t l = 1; l <= d->depth; ++l)
    DP_TRY(for_level_parts(d, l, [&](int32_t g0, int32_t n, bool cells) -> dp_status {
      DP_HIP_TRY(dp::launch_sim_level(g, cv, cnt, g0, n, nullptr, cells, tune, s));
      return DP_OK;
    }));
  DP_HIP_TRY(dp::launch_virus_power(ev->tog.as<uint32_t>(), ev->cap.as<float>(), d->n_nets, B,
                                    pv.as<double>(), s));
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (v0 && pb) DP_HIP_TRY(hipMemcpyAsync(v0, v0_dev.ptr, pb, k, s));
  if (p_final && pb) DP_HIP_TRY(hipMemcpyAsync(p_final, p_dev.ptr, pb * sizeof(float), k, s));
  if (p_virus) DP_HIP_TRY(hipMemcpyAsync(p_virus, pv.ptr, (size_t)B * sizeof(double), k, s));
  DP_HIP_TRY(hipStreamSynchronize(s));  // the scratch buffers are freed on return
  ev->inputs_version++;  // the PI probabilities are now the ascended ones
  return barrier_status(ev);
}

dp_status dp_backward_columns(dp_eval *ev, float *dpower_dpi, int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_backward_columns: NULL eval");
  if (!dpower_dpi) return fail(DP_E_INVALID, "dp_backward_columns: NULL output");
  return run_backward(ev, nullptr, 1, dpower_dpi, nullptr, nullptr, on_device);
}

dp_status dp_forward_backward_columns(dp_eval *ev, float *power, float *dpower_dpi,
                                      int32_t on_device) {
  if (!ev) return fail(DP_E_INVALID, "dp_forward_backward_columns: NULL eval");
  const dp_design *d = ev->d;
  // the schedules that capture: the whole pair of sweeps as one graph;
  // otherwise the two calls as they are
  const bool hyb = hybrid(ev);
  ChunkPlan plan;
  if (hyb) plan = plan_chunks(ev);
  const ChunkPlan *pl = hyb ? &plan : nullptr;
  const int64_t launches = forward_launches(ev, pl) + d->depth + d->split_levels + 1;
  if (ev->schedule != DP_SCHED_GRAPH || ev->profiling || launches > kMaxGraphLaunches) {
    DP_TRY(dp_forward(ev, nullptr));
    if (power) {
      const size_t bytes = (size_t)ev->B * s_prime(ev) * sizeof(float);
      DP_HIP_TRY(hipMemcpyAsync(power, ev->power.ptr, bytes,
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                ev->stream()));
    }
    if (dpower_dpi) return run_backward(ev, nullptr, 1, dpower_dpi, nullptr, nullptr, on_device);
    if (!on_device) {
      DP_TRY(sync_and_check(ev));
      DP_HIP_TRY(hipStreamSynchronize(ev->stream()));
    }
    return DP_OK;
  }
  // the checks of dp_forward and dp_backward, then every buffer before the
  // capture
  if (!ev->have_pi) return fail(DP_E_STATE, "dp_forward_backward_columns: PI probabilities not set");
  if (!ev->have_cap) return fail(DP_E_STATE, "dp_forward_backward_columns: capacitances not set");
  if (ev->S > 0 && !ev->have_size)
    return fail(DP_E_STATE, "dp_forward_backward_columns: cell sizes not set");
  if (ev->prm.mode == DP_FROZEN_BETA && !ev->have_beta)
    return fail(DP_E_STATE, "dp_forward_backward_columns: DP_FROZEN_BETA needs dp_set_beta");
  if (hyb && ev->have_stim &&
      ev->stim.bytes < (size_t)ev->B * d->n_pi * n_words(ev->prm) * sizeof(uint64_t))
    return fail(DP_E_STATE, "dp_forward_backward_columns: the explicit stimulus is shorter than "
                            "n_sim/64 words");
  DP_HIP_TRY(hipSetDevice(d->ctx->device));
  hipStream_t s = ev->stream();
  DP_TRY(ensure_forward_buffers(ev, pl));
  const int32_t C = ev->B * s_prime(ev);
  DP_TRY(ev->contrib.alloc(std::max<size_t>((size_t)d->n_edges * C * sizeof(float), 16)));
  const size_t dpi_bytes = (size_t)C * d->n_pi * sizeof(float);
  float *dst = on_device ? dpower_dpi : nullptr;
  if (!dst) {  // host output, or none: the sweep writes the staging buffer
    DP_TRY(ev->pi_out.alloc(std::max<size_t>(dpi_bytes, 16)));
    dst = ev->pi_out.as<float>();
  }
  const dp::BwdArgs ba = backward_args(ev, nullptr, 1, C);
  // the forward's key and the reverse sweep's, combined
  const uint64_t key = graph_key(ev, pl) * 1099511628211ull ^ reverse_key(ev, ba, dst);
  if (!ev->graph_fb || ev->graph_fb_key != key) {
    DP_TRY(capture_into(ev, &ev->graph_fb, [&]() -> dp_status {
      DP_TRY(enqueue_forward(ev, pl));
      return enqueue_backward(ev, ba, dst);
    }));
    ev->graph_fb_key = key;
  }
  DP_HIP_TRY(hipGraphLaunch(ev->graph_fb, s));
  ev->fwd_version = ev->inputs_version;
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (power)
    DP_HIP_TRY(hipMemcpyAsync(power, ev->power.ptr, (size_t)C * sizeof(float), k, s));
  if (dpower_dpi && !on_device && dpi_bytes)
    DP_HIP_TRY(hipMemcpyAsync(dpower_dpi, dst, dpi_bytes, hipMemcpyDeviceToHost, s));
  if (!on_device) {
    DP_TRY(sync_and_check(ev));
    DP_HIP_TRY(hipStreamSynchronize(s));
  }
  return DP_OK;
}

}  // extern "C"

// =========================================================================
// Design groups: the sweeps of several evals as one graph launch.
constexpr int32_t kGroupBranches = 4;  // streams beyond the hardware queues only queue

// Host threads that enqueue a group's branches side by side: a launch-bound
// sweep is limited by how fast one thread submits kernels, so each branch
// gets a thread of its own.  Workers live as long as the group.
namespace dp {

namespace {
// Range of level l of one kind: fixed cells first, then library cells.
void level_part(const dp_design *d, int32_t l, int k, int32_t *g0, int32_t *n) {
  const int32_t a = d->level_ptr[l], nl = d->level_ptr[l + 1] - a, nf = d->lvl_fixed[l];
  *g0 = k == 0 ? a : a + nf;
  *n = k == 0 ? nf : nl - nf;
}
}  // namespace

void MergedTables::build(const Lane *lanes, int32_t n) {
  D = 0;
  for (int32_t j = 0; j < n; ++j) D = std::max(D, lanes[j].ev->d->depth);
  fs.clear();
  bs.clear();
  f_launch.clear();
  const size_t m = 2 * (size_t)(D + 1);
  b_off.assign(m, 0);
  b_cnt.assign(m, 0);
  b_blk.assign(m, 0);
  // forward: level indices l and l + 1 share a launch when every design that
  // has level l holds fixed cells only there and pairs it with l + 1 (or
  // ends at l)
  for (int32_t l = 1; l <= D;) {
    bool pair = l + 1 <= D;
    for (int32_t j = 0; j < n && pair; ++j) {
      const dp_eval *ev = lanes[j].ev;
      const dp_design *d = ev->d;
      if (l > d->depth) continue;
      if (d->lvl_fixed[l] != d->level_ptr[l + 1] - d->level_ptr[l]) pair = false;
      else if (l + 1 <= d->depth && !pairs_levels(d, l, ev->B)) pair = false;
    }
    for (int k = 0; k < (pair ? 1 : 2); ++k) {
      FwdLaunch fl{(int32_t)fs.size(), 0, 0, k == 1};
      for (int32_t j = 0; j < n; ++j) {
        dp_eval *ev = lanes[j].ev;
        const dp_design *d = ev->d;
        if (l > d->depth) continue;
        int32_t g0, cnt;
        level_part(d, l, k, &g0, &cnt);
        if (cnt == 0) continue;
        SpLevel second{ev->sp.as<float>(), ev->B, 0, 0};
        if (pair && l + 1 <= d->depth) {
          second.g0 = d->level_ptr[l + 1];
          second.n = d->level_ptr[l + 2] - second.g0;
        }
        const uint32_t blocks =
            (uint32_t)(((int64_t)(cnt + second.n) * ev->B + kMergedBlock - 1) / kMergedBlock);
        fs.push_back({view(d), SpLevel{ev->sp.as<float>(), ev->B, g0, cnt}, second, fl.blocks});
        fl.blocks += blocks;
      }
      fl.cnt = (int32_t)fs.size() - fl.off;
      if (fl.cnt > 0) f_launch.push_back(fl);
    }
    l += pair ? 2 : 1;
  }
  for (int32_t l = 1; l <= D; ++l)
    for (int k = 0; k < 2; ++k) {
      const size_t i = 2 * (size_t)l + k;
      b_off[i] = (int32_t)bs.size();
      for (int32_t j = 0; j < n; ++j) {
        dp_eval *ev = lanes[j].ev;
        const dp_design *d = ev->d;
        if (l > d->depth || !lanes[j].backward) continue;
        int32_t g0, cnt;
        level_part(d, l, k, &g0, &cnt);
        if (cnt == 0) continue;
        const uint32_t blocks =
            (uint32_t)(((int64_t)cnt * ev->B + kMergedBlock - 1) / kMergedBlock);
        bs.push_back({view(d), backward_args(ev, nullptr, 0, ev->B), g0, cnt, b_blk[i]});
        b_blk[i] += blocks;
      }
      b_cnt[i] = (int32_t)bs.size() - b_off[i];
    }
}

int64_t MergedTables::level_launches(const Lane *lanes, int32_t n) {
  int32_t depth = 0;
  for (int32_t j = 0; j < n; ++j) depth = std::max(depth, lanes[j].ev->d->depth);
  int64_t c = 0;
  for (int32_t l = 1; l <= depth; ++l)
    for (int k = 0; k < 2; ++k) {
      bool any = false;
      for (int32_t j = 0; j < n && !any; ++j) {
        const dp_design *d = lanes[j].ev->d;
        int32_t g0, cnt = 0;
        if (l <= d->depth) level_part(d, l, k, &g0, &cnt);
        any = cnt > 0;
      }
      c += any;
    }
  return c;
}

size_t MergedTables::bwd_offset() const { return (fs.size() * sizeof(SpSeg) + 255) & ~(size_t)255; }

size_t MergedTables::bytes() const {
  return std::max<size_t>(bwd_offset() + bs.size() * sizeof(BwdSeg), 256);
}

void MergedTables::pack(void *host) const {
  if (!fs.empty()) std::memcpy(host, fs.data(), fs.size() * sizeof(SpSeg));
  if (!bs.empty())
    std::memcpy((char *)host + bwd_offset(), bs.data(), bs.size() * sizeof(BwdSeg));
}

dp_status MergedTables::launch_forward(const SpSeg *dev, hipStream_t s) const {
  for (const FwdLaunch &fl : f_launch)
    DP_HIP_TRY(launch_sp_multi(dev + fl.off, fl.cnt, fl.blocks, fl.cells, s));
  return DP_OK;
}

dp_status MergedTables::launch_reverse(const BwdSeg *dev, hipStream_t s) const {
  for (int32_t l = D; l >= 1; --l)
    for (int k = 0; k < 2; ++k) {
      const size_t i = 2 * (size_t)l + k;
      DP_HIP_TRY(launch_bwd_multi(dev + b_off[i], b_cnt[i], b_blk[i], k == 1, s));
    }
  return DP_OK;
}

}  // namespace dp

struct GroupPool {
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv, done;
  std::function<void(int)> task;
  uint64_t gen = 0;
  int n_tasks = 0, pending = 0;
  bool stop = false;

  void start(int n, int device) {
    for (int k = 0; k < n; ++k)
      workers.emplace_back([this, k, device]() {
        (void)hipSetDevice(device);
        uint64_t seen = 0;
        for (;;) {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return stop || gen != seen; });
          if (stop) return;
          seen = gen;
          const bool mine = k < n_tasks;
          lk.unlock();
          if (mine) task(k);
          lk.lock();
          if (mine && --pending == 0) done.notify_all();
        }
      });
  }
  // Run f(0) .. f(n - 1) on the workers and wait for all of them.
  void run(int n, std::function<void(int)> f) {
    std::unique_lock<std::mutex> lk(mu);
    task = std::move(f);
    n_tasks = n;
    pending = n;
    ++gen;
    cv.notify_all();
    done.wait(lk, [&] { return pending == 0; });
  }
  ~GroupPool() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
    for (auto &t : workers) t.join();
  }
};

struct dp_group {
  GroupPool pool;
  // Merged level launches of the group's modeled evals (one launch per level
  // index and kind covers that level of every such eval): host tables and
  // their device copy (forward segments, then reverse at tab_dev_bwd).
  std::vector<int32_t> merged;      // eval indices
  dp::MergedTables tab;
  dp::DevBuf tab_dev;
  size_t tab_dev_bwd = 0;
  bool have_tables = false;
  uint64_t tables_key = 0;
  dp_ctx *ctx = nullptr;
  std::vector<dp_eval *> evs;
  std::vector<hipStream_t> branch;  // up to kGroupBranches
  std::vector<hipEvent_t> join;     // one per branch
  std::vector<int32_t> branch_of;   // eval -> branch
  int32_t max_branches = 0;         // 0 = automatic
  bool use_graph = true;
  hipEvent_t fork = nullptr;
  hipStream_t capture = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t key = 0;
  ~dp_group() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (auto st : branch) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    for (auto e : join) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (capture) (void)hipStreamDestroy(capture);
  }
};

namespace {

// Assign evals to branches: longest first, each to the least loaded branch
// (load = kernel launches, the cost of a launch-bound sweep).
void assign_branches(dp_group *g, const std::vector<int64_t> &cost) {
  const int32_t nb = (int32_t)g->branch.size();
  std::vector<int32_t> order(g->evs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
  std::vector<int64_t> load(nb, 0);
  g->branch_of.assign(g->evs.size(), 0);
  for (int32_t i : order) {
    const int32_t k = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
    g->branch_of[i] = k;
    load[k] += cost[i];
  }
}

// Fork from `origin` into the branches, enqueue each eval's forward (and
// reverse) sweep on its branch with per-level launches, join back.
// Segment tables of the merged level launches (host work, one upload).
dp_status build_merged_tables(dp_group *g) {
  std::vector<dp::MergedTables::Lane> lanes;
  for (int32_t i : g->merged) lanes.push_back({g->evs[i], true});
  g->tab.build(lanes.data(), (int32_t)lanes.size());
  g->tab_dev_bwd = g->tab.bwd_offset();
  DP_TRY(g->tab_dev.alloc(g->tab.bytes()));
  std::vector<char> host(g->tab.bytes());
  g->tab.pack(host.data());
  DP_HIP_TRY(hipMemcpy(g->tab_dev.ptr, host.data(), host.size(), hipMemcpyHostToDevice));
  g->have_tables = true;
  return DP_OK;
}

// The modeled evals as merged level launches on `origin`: SP levels, each
// eval's finalize and power, and with backward the reverse levels and each
// eval's PI adjoints.
dp_status enqueue_merged(dp_group *g, hipStream_t origin, bool backward) {
  if (g->merged.empty()) return DP_OK;
  const dp::SpSeg *fs = g->tab_dev.as<dp::SpSeg>();
  const auto *bs = reinterpret_cast<const dp::BwdSeg *>((char *)g->tab_dev.ptr + g->tab_dev_bwd);
  DP_TRY(g->tab.launch_forward(fs, origin));
  for (int32_t i : g->merged) {
    dp_eval *ev = g->evs[i];
    ev->branch = origin;
    const dp_status st = enqueue_forward_tail(ev, nullptr);
    ev->branch = nullptr;
    DP_TRY(st);
  }
  if (!backward) return DP_OK;
  DP_TRY(g->tab.launch_reverse(bs, origin));
  for (int32_t i : g->merged) {
    dp_eval *ev = g->evs[i];
    const dp::HeavySpan hp = dp::heavy_pis(ev->d);
    DP_HIP_TRY(dp::launch_bwd_pi(view(ev->d), backward_args(ev, nullptr, 0, ev->B),
                                 ev->pi_out.as<float>(), origin, hp.gates, hp.n));
  }
  return DP_OK;
}

// `threads`: enqueue the branches from the group's worker threads, one
// each.  `single`: everything on `origin` itself, no branches (captures
// record one stream only).
dp_status enqueue_group(dp_group *g, hipStream_t origin, bool backward,
                        const std::vector<ChunkPlan> &plans, bool threads, bool single) {
  if (single) {
    for (size_t i = 0; i < g->evs.size(); ++i) {
      if (std::find(g->merged.begin(), g->merged.end(), (int32_t)i) != g->merged.end()) continue;
      dp_eval *ev = g->evs[i];
      const int32_t sched = ev->schedule;
      const bool prof = ev->profiling;
      ev->branch = origin;
      ev->schedule = DP_SCHED_LEVEL;
      ev->profiling = false;
      dp_status st = enqueue_forward(ev, &plans[i]);
      if (st == DP_OK && backward)
        st = enqueue_backward(ev, backward_args(ev, nullptr, 0, ev->B), ev->pi_out.as<float>());
      ev->branch = nullptr;
      ev->schedule = sched;
      ev->profiling = prof;
      DP_TRY(st);
    }
    return enqueue_merged(g, origin, backward);
  }
  DP_HIP_TRY(hipEventRecord(g->fork, origin));
  for (hipStream_t b : g->branch) DP_HIP_TRY(hipStreamWaitEvent(b, g->fork, 0));
  std::vector<bool> is_merged(g->evs.size(), false);
  for (int32_t i : g->merged) is_merged[i] = true;
  auto branch_task = [&](int32_t k) -> dp_status {
    for (size_t i = 0; i < g->evs.size(); ++i) {
      if (g->branch_of[i] != k || is_merged[i]) continue;
      dp_eval *ev = g->evs[i];
      const int32_t sched = ev->schedule;
      const bool prof = ev->profiling;
      ev->branch = g->branch[k];
      ev->schedule = DP_SCHED_LEVEL;
      ev->profiling = false;
      dp_status st = enqueue_forward(ev, hybrid(ev) ? &plans[i] : nullptr);
      if (st == DP_OK && backward)
        st = enqueue_backward(ev, backward_args(ev, nullptr, 0, ev->B), ev->pi_out.as<float>());
      ev->branch = nullptr;
      ev->schedule = sched;
      ev->profiling = prof;
      if (st != DP_OK) return st;
    }
    return DP_OK;
  };
  const int32_t nb = (int32_t)g->branch.size();
  if (threads && nb > 1) {
    std::vector<dp_status> st(nb, DP_OK);
    std::vector<std::string> msg(nb);
    g->pool.run(nb, [&](int k) {
      st[k] = branch_task(k);
      if (st[k] != DP_OK) msg[k] = dp_last_error();
    });
    for (int32_t k = 0; k < nb; ++k)
      if (st[k] != DP_OK) return fail(st[k], msg[k]);
  } else {
    for (int32_t k = 0; k < nb; ++k) DP_TRY(branch_task(k));
  }
  DP_TRY(enqueue_merged(g, origin, backward));
  for (size_t k = 0; k < g->branch.size(); ++k) {
    DP_HIP_TRY(hipEventRecord(g->join[k], g->branch[k]));
    DP_HIP_TRY(hipStreamWaitEvent(origin, g->join[k], 0));
  }
  return DP_OK;
}

}  // namespace

extern "C" {

dp_status dp_group_create(dp_ctx *ctx, dp_eval *const *evals, int32_t n_evals, dp_group **out) {
  if (!ctx || !evals || !out) return fail(DP_E_INVALID, "dp_group_create: NULL argument");
  if (n_evals < 1) return fail(DP_E_INVALID, "dp_group_create: need at least one eval");
  for (int32_t i = 0; i < n_evals; ++i) {
    if (!evals[i]) return fail(DP_E_INVALID, "dp_group_create: NULL eval");
    if (evals[i]->d->ctx != ctx)
      return fail(DP_E_INVALID, "dp_group_create: every eval's design must belong to this context");
    if (evals[i]->own_stream) return fail(DP_E_INVALID, "dp_group_create: serving lanes cannot join");
    for (int32_t j = 0; j < i; ++j)
      if (evals[j] == evals[i]) return fail(DP_E_INVALID, "dp_group_create: an eval appears twice");
  }
  DP_HIP_TRY(hipSetDevice(ctx->device));
  auto *g = new dp_group();
  g->ctx = ctx;
  g->evs.assign(evals, evals + n_evals);
  hipError_t e = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&g->capture, hipStreamNonBlocking);
  for (int32_t i = 0; i < std::min(n_evals, kGroupBranches) && e == hipSuccess; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) g->branch.push_back(st);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) g->join.push_back(ev);
  }
  if (e != hipSuccess) {
    delete g;
    return fail(DP_E_HIP, std::string("dp_group_create: ") + hipGetErrorString(e));
  }
  if (g->branch.size() > 1) g->pool.start((int)g->branch.size(), ctx->device);
  dp::ctx_retain(ctx);
  *out = g;
  return DP_OK;
}

dp_status dp_group_run(dp_group *g, int32_t backward, const dp_fwd_out *outs,
                       float *const *dpower_dpi, int32_t on_device) {
  if (!g) return fail(DP_E_INVALID, "dp_group_run: NULL group");
  DP_HIP_TRY(hipSetDevice(g->ctx->device));
  const size_t n = g->evs.size();
  std::vector<ChunkPlan> plans(n);
  std::vector<int64_t> cost(n, 0);
  int64_t launches = 0;
  uint64_t key = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { key = (key ^ v) * 1099511628211ull; };
  mix((uint64_t)(backward != 0));
  for (size_t i = 0; i < n; ++i) {
    dp_eval *ev = g->evs[i];
    const dp_design *d = ev->d;
    if (!ev->have_pi || !ev->have_cap || (ev->S > 0 && !ev->have_size) ||
        (ev->prm.mode == DP_FROZEN_BETA && !ev->have_beta))
      return fail(DP_E_STATE, "dp_group_run: eval " + std::to_string(i) + " has inputs missing");
    if (outs && !hybrid(ev) &&
        (outs[i].sp_acc || outs[i].tr_acc || outs[i].ones || outs[i].toggles))
      return fail(DP_E_INVALID, "dp_group_run: simulation outputs need DP_HYBRID");
    if (hybrid(ev) && ev->have_stim &&
        ev->stim.bytes < (size_t)ev->B * d->n_pi * n_words(ev->prm) * sizeof(uint64_t))
      return fail(DP_E_STATE, "dp_group_run: an explicit stimulus is too short");
    if (hybrid(ev)) plans[i] = plan_chunks(ev);
    DP_TRY(ensure_forward_buffers(ev, hybrid(ev) ? &plans[i] : nullptr));
    cost[i] = forward_launches(ev, hybrid(ev) ? &plans[i] : nullptr);
    if (backward) {
      DP_TRY(ev->contrib.alloc(std::max<size_t>((size_t)d->n_edges * ev->B * sizeof(float), 16)));
      DP_TRY(ev->pi_out.alloc(std::max<size_t>((size_t)ev->B * d->n_pi * sizeof(float), 16)));
      cost[i] += d->depth + d->split_levels + 1;
    }
    launches += cost[i];
    const int32_t sched = ev->schedule;
    ev->schedule = DP_SCHED_LEVEL;
    mix(graph_key(ev, hybrid(ev) ? &plans[i] : nullptr));
    ev->schedule = sched;
    mix((uint64_t)(uintptr_t)ev->contrib.ptr);
    mix((uint64_t)(uintptr_t)ev->pi_out.ptr);
    mix((uint64_t)(uintptr_t)(ev->have_fixed ? ev->fixed.ptr : nullptr));
    mix((uint64_t)ev->B);
    mix((uint64_t)(uintptr_t)ev->sp.ptr);
    mix((uint64_t)(uintptr_t)ev->beta.ptr);
    mix((uint64_t)(uintptr_t)ev->cap.ptr);
  }
  // modeled evals go into the merged level launches; the others (hybrid)
  // run on the branches
  g->merged.clear();
  for (size_t i = 0; i < n; ++i)
    if (!hybrid(g->evs[i])) {
      g->merged.push_back((int32_t)i);
      launches -= cost[i];
      cost[i] = 0;
    }
  if (!g->merged.empty()) {
    std::vector<dp::MergedTables::Lane> lanes;
    for (int32_t i : g->merged) lanes.push_back({g->evs[i], true});
    const int64_t per_sweep = dp::MergedTables::level_launches(lanes.data(), (int32_t)lanes.size());
    launches += per_sweep * (backward ? 2 : 1) + (int64_t)g->merged.size() * (backward ? 4 : 3);
  }
  const int32_t want = g->max_branches > 0 ? g->max_branches : kGroupBranches;
  const int32_t nb = std::max<int32_t>(1, std::min<int32_t>({want, (int32_t)g->branch.size(), (int32_t)n}));
  std::vector<hipStream_t> all = g->branch;
  g->branch.resize(nb);
  assign_branches(g, cost);
  for (size_t i = 0; i < n; ++i) mix((uint64_t)g->branch_of[i]);
  hipStream_t s = g->ctx->stream;
  struct Restore {
    dp_group *g;
    std::vector<hipStream_t> all;
    ~Restore() { g->branch = all; }
  } restore{g, all};
  if (g->tables_key != key || !g->have_tables) {
    DP_HIP_TRY(hipStreamSynchronize(s));  // no run reads the old tables
    DP_TRY(build_merged_tables(g));
    g->tables_key = key;
  }
  if (g->use_graph && launches <= kMaxGraphLaunches) {
    if (!g->exec || g->key != key) {
      if (g->exec) {
        DP_HIP_TRY(hipStreamSynchronize(s));
        (void)hipGraphExecDestroy(g->exec);
        g->exec = nullptr;
      }
      DP_HIP_TRY(hipStreamBeginCapture(g->capture, hipStreamCaptureModeThreadLocal));
      const dp_status st = enqueue_group(g, g->capture, backward != 0, plans, false, true);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(g->capture, &graph);
      if (st != DP_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
      }
      if (e != hipSuccess) return fail(DP_E_HIP, std::string("group capture failed: ") + hipGetErrorString(e));
      const hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ei != hipSuccess) {
        g->exec = nullptr;
        return fail(DP_E_HIP, std::string("group instantiate failed: ") + hipGetErrorString(ei));
      }
      g->key = key;
    }
    DP_HIP_TRY(hipGraphLaunch(g->exec, s));
  } else {
    DP_TRY(enqueue_group(g, s, backward != 0, plans, true, false));
  }
  bool host_out = false;
  for (size_t i = 0; i < n; ++i) {
    dp_eval *ev = g->evs[i];
    ev->fwd_version = ev->inputs_version;
    if (outs) {
      DP_TRY(export_forward(ev, &outs[i], hybrid(ev) ? &plans[i] : nullptr));
      host_out = host_out || !outs[i].on_device;
    }
    if (backward && dpower_dpi && dpower_dpi[i] && ev->d->n_pi > 0) {
      DP_HIP_TRY(hipMemcpyAsync(dpower_dpi[i], ev->pi_out.ptr,
                                (size_t)ev->B * ev->d->n_pi * sizeof(float),
                                on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                ev->stream()));
      host_out = host_out || !on_device;
    }
  }
  if (host_out) DP_HIP_TRY(hipStreamSynchronize(s));
  return DP_OK;
}

dp_status dp_group_configure(dp_group *g, int32_t use_graph, int32_t max_branches) {
  if (!g) return fail(DP_E_INVALID, "dp_group_configure: NULL group");
  if (max_branches < 0) return fail(DP_E_INVALID, "dp_group_configure: max_branches < 0");
  g->use_graph = use_graph != 0;
  g->max_branches = max_branches;
  return DP_OK;
}

void dp_group_destroy(dp_group *g) {
  if (!g) return;
  dp_ctx *c = g->ctx;
  (void)hipStreamSynchronize(c->stream);
  delete g;
  dp::ctx_release(c);
}

}  // extern "C"

// =========================================================================
// Serving lanes (internal).
namespace dp {

size_t lane_bytes(const dp_design *d, int32_t capacity) {
  const size_t nn = d->n_nets, G = d->n_gates, np = d->n_pi;
  // SP per net (the frozen beta is one per net, shared by the columns);
  // contributions per edge; sizes (and their staging) per gate;
  // probabilities (and staging, dP/dp)
  const size_t per_col = 4 * (nn + (size_t)d->n_edges + 2 * G + 2 * np) +
                         8 * (size_t)power_chunks(d->n_nets) + 16;
  return (size_t)capacity * per_col + 8 * nn;
}

dp_status lane_create(dp_design *d, int32_t capacity, const dp_params *prm, hipStream_t stream,
                      const float *cap_int, const float *beta_int, dp_eval **out) {
  DP_TRY(check_params(prm));
  if (prm->mode == DP_HYBRID) return fail(DP_E_UNSUPPORTED, "serving lanes run DP_MODELED or DP_FROZEN_BETA");
  auto *ev = new dp_eval();
  ev->d = d;
  ev->B = capacity;
  ev->S = capacity;
  ev->paired_sizes = true;
  ev->prm = *prm;
  ev->own_stream = stream;
  ev->schedule = DP_SCHED_LEVEL;
  const size_t nn = d->n_nets;
  dp_status st = DP_OK;
  auto A = [&](DevBuf &b, size_t bytes) {
    if (st == DP_OK) st = b.alloc(std::max<size_t>(bytes, 16));
  };
  A(ev->sp, nn * capacity * 4);
  A(ev->cap, nn * 4);
  A(ev->size, (size_t)capacity * d->n_gates * 4);
  A(ev->size_stage, (size_t)capacity * d->n_gates * 4);
  A(ev->p_stage, (size_t)capacity * d->n_pi * 4);
  if (prm->mode == DP_HYBRID) A(ev->beta, nn * capacity * 4);
  A(ev->power_partial, (size_t)power_chunks(d->n_nets) * capacity * 8);
  A(ev->power, (size_t)capacity * 4);
  A(ev->contrib, (size_t)d->n_edges * capacity * 4);
  A(ev->pi_out, (size_t)capacity * d->n_pi * 4);
  if (beta_int) A(ev->beta_frozen, nn * 4);
  if (st != DP_OK) {
    delete ev;
    return st;
  }
  hipError_t e = hipMemcpyAsync(ev->cap.ptr, cap_int, nn * 4, hipMemcpyDeviceToDevice, stream);
  if (e == hipSuccess && beta_int)
    e = hipMemcpyAsync(ev->beta_frozen.ptr, beta_int, nn * 4, hipMemcpyDeviceToDevice, stream);
  // steps run on streams of their own: the lane's inputs must be in place
  // before any of them reads the lane
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    delete ev;
    return fail(DP_E_HIP, std::string("lane_create: ") + hipGetErrorString(e));
  }
  ev->beta_shared = beta_int != nullptr;
  ev->have_cap = ev->have_pi = true;
  ev->have_beta = beta_int != nullptr;
  design_retain(d);
  *out = ev;
  return DP_OK;
}

dp_status lane_run(dp_eval *ev, int32_t n, const float *p, const float *size, bool backward,
                   float *power, float *dpi) {
  const dp_design *d = ev->d;
  hipStream_t s = ev->stream();
  ev->B = n;
  ev->S = size ? n : 0;
  ev->paired_sizes = size != nullptr;
  if (d->n_pi > 0) {
    DP_HIP_TRY(hipMemcpyAsync(ev->p_stage.ptr, p, (size_t)n * d->n_pi * 4, hipMemcpyHostToDevice, s));
    DP_HIP_TRY(launch_load_pi(ev->p_stage.as<float>(), ev->sp.as<float>(), d->n_pi, n, s));
  }
  if (size && d->n_gates > 0) {
    DP_HIP_TRY(hipMemcpyAsync(ev->size_stage.ptr, size, (size_t)n * d->n_gates * 4,
                              hipMemcpyHostToDevice, s));
    DP_HIP_TRY(launch_import_sizes(ev->size_stage.as<float>(), d->int2ext.as<int32_t>(),
                                   ev->size.as<float>(), d->n_pi, d->n_gates, n, s));
  }
  DP_TRY(enqueue_forward(ev, nullptr));
  DP_HIP_TRY(hipMemcpyAsync(power, ev->power.ptr, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  if (backward) {
    const GraphView g = view(d);
    const BwdArgs ba = backward_args(ev, nullptr, 0, n);
    for (int32_t l = d->depth; l >= 1; --l)
      DP_TRY(for_level_parts(d, l, [&](int32_t g0, int32_t n, bool cells) -> dp_status {
        const HeavySpan hs = heavy_span(d, g0, n);
        DP_HIP_TRY(launch_bwd_level(g, ba, g0, n, cells, s, hs.gates, hs.n));
        return DP_OK;
      }));
    const HeavySpan hp = heavy_pis(d);
    DP_HIP_TRY(launch_bwd_pi(g, ba, ev->pi_out.as<float>(), s, hp.gates, hp.n));
    if (dpi && d->n_pi > 0)
      DP_HIP_TRY(hipMemcpyAsync(dpi, ev->pi_out.ptr, (size_t)n * d->n_pi * 4,
                                hipMemcpyDeviceToHost, s));
  }
  return DP_OK;
}

StepScratch::~StepScratch() {
  if (host) (void)hipHostFree(host);
}

namespace {

// Stage one lane's inputs on `s` (the first half of lane_run).
dp_status lane_stage(dp_eval *ev, int32_t n, const float *p, const float *size, hipStream_t s) {
  const dp_design *d = ev->d;
  ev->B = n;
  ev->S = size ? n : 0;
  ev->paired_sizes = size != nullptr;
  if (d->n_pi > 0) {
    DP_HIP_TRY(hipMemcpyAsync(ev->p_stage.ptr, p, (size_t)n * d->n_pi * 4, hipMemcpyHostToDevice, s));
    DP_HIP_TRY(launch_load_pi(ev->p_stage.as<float>(), ev->sp.as<float>(), d->n_pi, n, s));
  }
  if (size && d->n_gates > 0) {
    DP_HIP_TRY(hipMemcpyAsync(ev->size_stage.ptr, size, (size_t)n * d->n_gates * 4,
                              hipMemcpyHostToDevice, s));
    DP_HIP_TRY(launch_import_sizes(ev->size_stage.as<float>(), d->int2ext.as<int32_t>(),
                                   ev->size.as<float>(), d->n_pi, d->n_gates, n, s));
  }
  return DP_OK;
}

}  // namespace

dp_status lanes_run_merged(const LaneJob *jobs, int32_t n_jobs, hipStream_t s,
                           StepScratch *sc) {
  for (int32_t j = 0; j < n_jobs; ++j)
    DP_TRY(lane_stage(jobs[j].ev, jobs[j].n, jobs[j].p, jobs[j].size, s));
  // segment tables: forward over every lane, reverse over the lanes that
  // want gradients
  std::vector<MergedTables::Lane> lanes(n_jobs);
  bool any_backward = false;
  for (int32_t j = 0; j < n_jobs; ++j) {
    lanes[j] = {jobs[j].ev, jobs[j].backward};
    any_backward = any_backward || jobs[j].backward;
  }
  MergedTables tab;
  tab.build(lanes.data(), n_jobs);
  const size_t bytes = tab.bytes();
  if (bytes > sc->cap) {
    if (sc->host) (void)hipHostFree(sc->host);
    sc->host = nullptr;
    sc->cap = 0;
    DP_HIP_TRY(hipHostMalloc(&sc->host, bytes));
    DP_TRY(sc->dev.alloc(bytes));
    sc->cap = bytes;
  }
  tab.pack(sc->host);
  DP_HIP_TRY(hipMemcpyAsync(sc->dev.ptr, sc->host, bytes, hipMemcpyHostToDevice, s));
  const SpSeg *fd = sc->dev.as<SpSeg>();
  const BwdSeg *bd = reinterpret_cast<const BwdSeg *>((char *)sc->dev.ptr + tab.bwd_offset());
  DP_TRY(tab.launch_forward(fd, s));
  for (int32_t j = 0; j < n_jobs; ++j) {
    dp_eval *ev = jobs[j].ev;
    ev->branch = s;
    const dp_status st = enqueue_forward_tail(ev, nullptr);
    ev->branch = nullptr;
    DP_TRY(st);
    DP_HIP_TRY(hipMemcpyAsync(jobs[j].power, ev->power.ptr, (size_t)jobs[j].n * 4,
                              hipMemcpyDeviceToHost, s));
  }
  if (!any_backward) return DP_OK;
  DP_TRY(tab.launch_reverse(bd, s));
  for (int32_t j = 0; j < n_jobs; ++j) {
    if (!jobs[j].backward) continue;
    dp_eval *ev = jobs[j].ev;
    const dp_design *d = ev->d;
    const HeavySpan hp = heavy_pis(d);
    DP_HIP_TRY(launch_bwd_pi(view(d), backward_args(ev, nullptr, 0, ev->B),
                             ev->pi_out.as<float>(), s, hp.gates, hp.n));
    if (jobs[j].dpi && d->n_pi > 0)
      DP_HIP_TRY(hipMemcpyAsync(jobs[j].dpi, ev->pi_out.ptr, (size_t)jobs[j].n * d->n_pi * 4,
                                hipMemcpyDeviceToHost, s));
  }
  return DP_OK;
}

dp_status calibrate_beta(dp_design *d, const float *cap_ext, const dp_params *prm, float p_all,
                         float *beta_int) {
  dp_params hp = *prm;
  hp.mode = DP_HYBRID;
  dp_eval *ev = nullptr;
  DP_TRY(dp_eval_create(d, 1, 0, &hp, &ev));
  std::vector<float> p(d->n_pi, p_all);
  dp_status st = dp_set_pi_prob(ev, p.data(), 0);
  if (st == DP_OK) st = dp_set_caps(ev, cap_ext, 0);
  if (st == DP_OK) st = dp_forward(ev, nullptr);
  if (st == DP_OK) {
    hipError_t e = hipMemcpyAsync(beta_int, ev->beta.ptr, (size_t)d->n_nets * 4,
                                  hipMemcpyDeviceToDevice, ev->stream());
    if (e == hipSuccess) e = hipStreamSynchronize(ev->stream());
    if (e != hipSuccess) st = fail(DP_E_HIP, std::string("calibrate_beta: ") + hipGetErrorString(e));
  }
  dp_eval_destroy(ev);
  return st;
}

}  // namespace dp

