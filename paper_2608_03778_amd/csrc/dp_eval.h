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
  bool have_pi = false, have_cap = false, have_size = false, have_beta = false,
       have_stim = false;
  uint64_t inputs_version = 1, fwd_version = 0;
  // forward state
  dp::DevBuf words;          // simulation chunk [n_nets][pitch]
  dp::DevBuf ones, tog;      // [n_nets][B]
  dp::DevBuf beta, xterm, seed_base;  // [n_nets][B]
  dp::DevBuf power_partial;  // [chunks][B*S'] double
  dp::DevBuf power;          // [B*S']
  dp::DevBuf flag;           // int32 validation flag
  // reverse state
  dp::DevBuf w;              // [B*S'] upstream weights
  dp::DevBuf seed;           // [n_nets][C]
  dp::DevBuf contrib;        // [3][G][C]
  dp::DevBuf pi_out;         // [C][n_pi] staging for host outputs
  dp::DevBuf stage[8];       // host-output staging
  // profiling
  bool profiling = false;
  dp_profile prof{};
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Span { size_t a, b; int kind; double bytes; };
  std::vector<Span> spans;
  // captured sweeps
  hipGraphExec_t graph_fwd = nullptr;
  uint64_t graph_key = 0;
  ~dp_eval();
};
