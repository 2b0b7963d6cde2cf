// Evaluation state (host side).  Not part of the ABI.
#pragma once

#include <vector>

#include "dp_internal.h"
#include "dp_kernels.h"

struct dp_eval {
  dp_design *d = nullptr;
  int32_t B = 1, S = 0;      // query columns, size vectors (0 = none)
  dp_params prm{};
  // schedule
  int32_t schedule = DP_SCHED_AUTO;
  int64_t words_per_chunk = 0;
  int32_t sim_iters = 0;
  int32_t sim_streams = 0;                 // 0 = automatic (1)
  int32_t sim_cols = 0;                    // columns per simulation launch, 0 = what the budget holds
  std::vector<hipStream_t> lane_streams;   // extra simulation streams (owned)
  std::vector<hipEvent_t> lane_events;     // fork + one join per extra stream
  // inputs
  dp::DevBuf p_stage;        // [B][n_pi] caller layout
  dp::DevBuf sp;             // [n_nets][B]
  dp::DevBuf cap;            // [n_nets] internal
  dp::DevBuf cap_stage;      // [n_nets] caller numbering
  dp::DevBuf size;           // [S][G] internal gate order
  dp::DevBuf size_stage;     // [S][G] caller gate order
  dp::DevBuf beta_frozen;    // [n_nets][B]
  dp::DevBuf beta_stage;     // [B][n_nets]
  dp::DevBuf stim;           // [B][n_pi][T]
  dp::DevBuf tau;            // [B][n_pi] target transition rates (caller layout)
  dp::DevBuf streams;        // int32 [n_pi] Philox stream of each PI
  dp::DevBuf fixed;          // uint8 [n_pi] PIs excluded from the gradients
  dp::DevBuf mstim;          // [B][n_pi][T] Markov stimulus words of the forward
  bool have_pi = false, have_cap = false, have_size = false, have_beta = false,
       have_stim = false, have_tau = false, have_streams = false, have_fixed = false;
  uint64_t inputs_version = 1, fwd_version = 0;
  // forward state
  dp::DevBuf words;          // simulation chunk [n_nets][pitch]
  dp::DevBuf ones, tog;      // [n_nets][B]
  dp::DevBuf beta;           // [n_nets][B] computed beta (hybrid mode only)
  dp::DevBuf power_partial;  // [chunks][B*S'] double
  dp::DevBuf power;          // [B*S']
  dp::DevBuf flag;           // int32 validation flag
  dp::DevBuf barrier;        // persistent sweeps: grid-barrier words (dp::kBarrierAlloc)
  bool barrier_pending = false;      // a persistent sweep ran since the report word was read
  double barrier_limit_us = 1000.0;  // a barrier wait gives up after this long without progress
  // reverse state
  dp::DevBuf w;              // [B*S'] upstream weights
  dp::DevBuf contrib;        // [n_edges][C]
  dp::DevBuf pi_out;         // [C][n_pi] staging for host outputs
  dp::DevBuf stage[8];       // host-output staging
  // A stream of its own (serving lanes); null = the context's stream.
  hipStream_t own_stream = nullptr;
  // Private stream graphs are captured on, and whether a capture is running.
  hipStream_t capture_stream_owned = nullptr;
  // Private stream and fork/join events for cooperative launches when the
  // caller's stream is the null stream.
  hipStream_t coop_stream = nullptr;
  hipEvent_t coop_events[2] = {nullptr, nullptr};
  bool capturing = false;
  // Stream of the eval's branch while a design group enqueues it.
  hipStream_t branch = nullptr;
  hipStream_t stream() const {
    if (capturing) return capture_stream_owned;
    if (branch) return branch;
    return own_stream ? own_stream : d->ctx->stream;
  }
  // Column b uses size vector b (S == B) and power is [B] (serving).
  bool paired_sizes = false;
  // DP_FROZEN_BETA with one beta [n_nets] shared by every column (serving).
  bool beta_shared = false;
  // profiling
  bool profiling = false;
  dp_profile prof{};
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Span { size_t a, b; int kind; double bytes; int64_t launches; };
  std::vector<Span> spans;
  // captured sweeps
  hipGraphExec_t graph_fwd = nullptr;
  uint64_t graph_key = 0;
  hipGraphExec_t graph_bwd = nullptr;  // the reverse sweep of dp_backward
  uint64_t graph_bwd_key = 0;
  hipGraphExec_t graph_fb = nullptr;   // both sweeps of dp_forward_backward_columns
  uint64_t graph_fb_key = 0;
  ~dp_eval();
};

namespace dp {

// Serving lanes: an eval with its own stream that runs whole batches without
// validation or host synchronisation.  Implemented in dp_api.cpp.
//   cap_int:   [n_nets] internal-order capacitances (device)
//   beta_int:  [n_nets] internal-order frozen beta (device) or null
dp_status lane_create(dp_design *d, int32_t capacity, const dp_params *prm, hipStream_t stream,
                      const float *cap_int, const float *beta_int, dp_eval **out);
// Enqueue one batch of n columns: p [n][n_pi] and sizes [n][n_gates] (caller
// gate order, or null) in pinned host memory; outputs power [n] and, when
// backward, dP/dp [n][n_pi] into pinned host memory.
dp_status lane_run(dp_eval *ev, int32_t n, const float *p, const float *size, bool backward,
                   float *power, float *dpi);
// Device bytes a lane of `capacity` columns holds.
size_t lane_bytes(const dp_design *d, int32_t capacity);

// Scratch of one serving step: the merged launches' segment tables, staged
// in pinned host memory and copied to the device on the step's stream.  Only
// touched while the step is idle.
struct StepScratch {
  void *host = nullptr;
  dp::DevBuf dev;
  size_t cap = 0;
  ~StepScratch();
};
// One lane's share of a step: n columns, inputs p [n][n_pi] and sizes
// [n][n_gates] (or null) in pinned memory, outputs power [n] and, when
// backward, dP/dp [n][n_pi] in pinned memory.
struct LaneJob {
  dp_eval *ev;
  int32_t n;
  const float *p, *size;
  bool backward;
  float *power, *dpi;
};
// Enqueue one step over several lanes (of any designs) on `stream`: their
// SP levels as merged launches (one per level index), each lane's finalize
// and power, then the merged reverse levels of the lanes that want
// gradients.  Each lane's results equal lane_run's bit for bit.
dp_status lanes_run_merged(const LaneJob *jobs, int32_t n_jobs, hipStream_t stream,
                           StepScratch *scratch);
// Segment tables of merged level launches over several evals (design groups
// and serving steps): for each level index l and kind k (0: fixed cells,
// 1: library cells) the segments of every eval's level-l range of that kind,
// one launch each.  Segments start on block boundaries, so a block belongs to
// one eval.
struct MergedTables {
  struct Lane {
    dp_eval *ev;
    bool backward;  // reverse segments too
  };
  int32_t D = 0;
  std::vector<SpSeg> fs;
  std::vector<BwdSeg> bs;
  // the forward's launches in order: first segment, segment count, blocks,
  // kind (a launch covers one level index, or two when every design in it
  // pairs them)
  struct FwdLaunch {
    int32_t off, cnt;
    uint32_t blocks;
    bool cells;
  };
  std::vector<FwdLaunch> f_launch;
  // reverse, [2 (D + 1)], index 2 l + k: first segment, segment count, blocks
  std::vector<int32_t> b_off, b_cnt;
  std::vector<uint32_t> b_blk;
  void build(const Lane *lanes, int32_t n);
  // Launches of one merged sweep over these lanes (the reverse; the
  // forward's are at most as many).
  static int64_t level_launches(const Lane *lanes, int32_t n);
  // Packed layout: forward segments, then the reverse ones at bwd_offset().
  size_t bwd_offset() const;
  size_t bytes() const;
  void pack(void *host) const;
  dp_status launch_forward(const SpSeg *dev, hipStream_t s) const;
  dp_status launch_reverse(const BwdSeg *dev, hipStream_t s) const;
};

// Hybrid calibration at probability p_all for every PI: beta [n_nets] in
// internal order into beta_int (device), on the context's stream.
dp_status calibrate_beta(dp_design *d, const float *cap_ext, const dp_params *prm, float p_all,
                         float *beta_int);

}  // namespace dp

