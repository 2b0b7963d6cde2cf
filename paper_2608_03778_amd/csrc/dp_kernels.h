// Launch interface of the gfx950 kernels (dp_kernels.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dp {

// Net-level graph arrays in internal numbering (see dp_design).
// Library cells: the host compiles each expression to post-order code for
// a stack machine that the kernels interpret.  An instruction is
// op | arg << 8; arg is the input index of kCellIn.
constexpr int kCellBase = 16;  // gate opcode of library cell c is kCellBase + c
constexpr int kCellMaxIn = 6;
constexpr int kCellMaxCode = 32;
constexpr int kCellMaxStack = 8;
enum : int { kCellIn = 0, kCellNot = 1, kCellAnd = 2, kCellOr = 3, kCellXor = 4,
             kCellZero = 5, kCellOne = 6 };

struct GraphView {
  const uint8_t *op;        // [G]
  const int32_t *in;        // [pins][G] (unused pins alias pin 0)
  const int32_t *rev_ptr;   // [n_nets + 1]
  const int32_t *rev_edge;  // [n_edges]
  const int32_t *slot;      // [pins][G] fan-out position of each pin
  const uint16_t *code;     // [n_cells][kCellMaxCode] library cells' stack code (op | arg << 8), padded
  const int32_t *cell;      // [n_cells][3]: code offset, length, inputs
  const uint64_t *tt;       // [n_cells] truth tables: bit m = output for input pattern m
  const uint8_t *arity;     // [G] input count of each gate
  int32_t pins;             // rows of in and slot (3, or the widest cell)
  int32_t n_pi, G, n_nets;
};

// Simulation word buffers of the query columns a launch covers: column
// cnt.col + c has its own buffer at W + c * col_stride, whose row r (an
// internal net) holds words [t0 - halo, t0 - halo + pitch) of the current
// chunk at r * pitch.  Local word u counts ones when u in [u_lo, u_hi) and
// toggles (against word u - 1) when u in [u_tog_lo, u_hi).
struct ChunkView {
  uint64_t *W;
  int64_t pitch;       // words per row (even)
  int64_t col_stride;  // words between the buffers of consecutive columns
  int64_t t_first;     // global cycle of local word 0 (t0 - halo)
  int32_t pairs;       // word pairs per row to compute, ceil(u_hi / 2)
  int32_t u_lo, u_hi, u_tog_lo;
  int32_t n_cols;      // columns of the launch, cnt.col .. cnt.col + n_cols - 1
};

// Counter arrays [n_nets][B]; a launch adds into columns cnt.col onwards.
struct CountView {
  uint32_t *ones, *tog;
  int32_t B, col;
};

// Signal probabilities are stored as one float per net and column,
// [n_nets][B]: the smaller of p and q = 1 - p, negated when it is q.  The
// kernels work on the pair (p, q): every cell rule has a form without
// cancellation for both, so TR = 2 p q keeps its relative accuracy when p is
// near 0 or 1, and the larger of the two is always 1 minus the smaller, so
// the one float holds the pair exactly.

// SP of one level of B columns, optionally fused into a simulation launch.
struct SpLevel {
  float *sp;          // [n_nets][B]
  int32_t B;
  int32_t g0, n;      // level gate range (internal ids)
};

// Tunables of the simulation launch.
struct SimTune {
  int32_t iters;      // word pairs per lane per wave: 1, 2, 4 or 8
};

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);

// PI probabilities [B][n_pi] (caller layout) -> stored SP [n_pi][B].
hipError_t launch_load_pi(const float *p, float *sp, int32_t n_pi, int32_t B, hipStream_t s);
// Check values are finite and inside [lo, hi]; sets *bad = 1 otherwise.
hipError_t launch_check_range(const float *v, int64_t n, float lo, float hi, int32_t *bad,
                              hipStream_t s);
// Caller-numbered per-net array [n_nets] -> internal numbering.
hipError_t launch_gather_nets_f32(const float *src_ext, const int32_t *int2ext, float *dst_int,
                                  int32_t n_nets, hipStream_t s);
// [B][n_nets] caller numbering -> [n_nets][B] internal.
hipError_t launch_import_cols_f32(const float *src, const int32_t *int2ext, float *dst,
                                  int32_t n_nets, int32_t B, hipStream_t s);
// Sizes [S][G] caller gate numbering -> [S][G] internal gate order.
hipError_t launch_import_sizes(const float *src, const int32_t *int2ext, float *dst, int32_t n_pi,
                               int32_t G, int32_t S, hipStream_t s);

// One SP level (modeled sweep).
// cells: the range holds library cells only (every launch below that takes
// the flag runs a range of one kind; a level's library cells follow its
// fixed cells).
hipError_t launch_sp_level(const GraphView &g, const SpLevel &lv, bool cells, hipStream_t s);
// Two consecutive levels of fixed cells in one launch (b starts where a
// ends; the same columns and SP array): level b's lanes recompute the pins
// level a drives instead of waiting for them, bit for bit as level a's
// lanes compute them.
hipError_t launch_sp_pair(const GraphView &g, const SpLevel &a, const SpLevel &b, hipStream_t s);

// PI rows of one chunk for the launch's columns: Philox stimulus (stim ==
// nullptr) or explicit words stim[c][i][T] (c counted from column cnt.col);
// counts ones/toggles of the PI nets.
// stream [n_pi]: the Philox stream of each PI (null = its own index).
hipError_t launch_stimulus(const GraphView &g, const ChunkView &c, const CountView &cnt,
                           const float *p_col /* stored SP [n_pi][B] */,
                           const uint64_t *stim, int64_t T, const int32_t *stream, uint64_t seed,
                           const SimTune &tune, hipStream_t s);
// Markov stimulus words out [B][n_pi][T] from the PI probabilities (stored
// SP [n_pi][B]), the target transition rates tau [B][n_pi] and the streams
// (null = own).
hipError_t launch_markov_words(const float *sp, const float *tau, const int32_t *stream,
                               int32_t n_pi, int32_t B, int64_t T, uint64_t seed, uint64_t *out,
                               hipStream_t s);

// Library cells with at most this many inputs run in simulation launches
// of their own, with more word pairs per lane than the wider cells.
constexpr int kSmallCellInputs = 3;

// One simulation level of one chunk for the launch's columns, with SP of
// the gates of sp (every column; gates of the launch's kind) fused in when
// sp != nullptr.  cell_inputs: the most inputs a library cell of the range
// has (kSmallCellInputs or fewer selects the narrow instance).
hipError_t launch_sim_level(const GraphView &g, const ChunkView &c, const CountView &cnt,
                            int32_t g0, int32_t n, const SpLevel *sp, bool cells,
                            const SimTune &tune, hipStream_t s, int cell_inputs = 6);

// Caller-numbered exports of forward quantities, [B][n_nets].
struct ExportArgs {
  const float *sp;            // [n_nets][B]
  const float *beta;
  const uint32_t *ones, *tog;
  const int32_t *int2ext;
  int64_t T;
  float *o_sp, *o_tr, *o_sp_acc, *o_tr_acc, *o_beta, *o_tr_hyb;
  uint32_t *o_ones, *o_tog;
  int32_t n_nets, B;
};
hipError_t launch_export(const ExportArgs &a, hipStream_t s);

// The per-net power terms and their sum (Eq. 1, 2, 5).  For net n and
// column b: TR_model = 2 P (1 - P); beta = 1 (modeled), the frozen beta,
// or in hybrid mode clip(TR_acc / TR_model) with TR_acc = toggles /
// (64 (T - 1)) (0/0 -> 1, x/0 -> beta_max), stored in `beta`; the term
// x = kappa beta TR_model, and P[b][s] = sum_n x[n][b] C_n s_s(drv n),
// accumulated in double in an order fixed by the net index alone.  No
// per-net term array is stored: whatever needs x again (the gradient with
// respect to C and s) recomputes it from SP and beta.
struct PowerArgs {
  const float *sp;                  // [n_nets][B]
  const uint32_t *tog;              // [n_nets][B] toggle counts (hybrid), or null
  const float *beta_frozen;         // [n_nets][B], [n_nets] when beta_shared, or null
  int32_t beta_shared;              // one frozen beta for every column
  const float *cap, *size;          // cap [n_nets] internal; size [S][G] internal or null
  int64_t T;                        // simulated words (hybrid)
  float kappa, beta_min, beta_max;
  int32_t mode;                     // DP_MODELED, DP_HYBRID, DP_FROZEN_BETA
  float *beta;                      // out [n_nets][B] (hybrid), or null
  int32_t n_pi, n_nets, G, B, S;    // S = 0: no sizes
  int32_t paired;                   // column b uses size row b; power is [B]
  double *partial;                  // scratch
  int32_t n_chunks;
  float *power;                     // [B][S'] (device)
};
int32_t power_chunks(int32_t n_nets);
// Doubles of partial-sum scratch launch_power needs.
int32_t power_partial_doubles(int32_t n_nets, int32_t B, int32_t S, int32_t paired);
hipError_t launch_power(const PowerArgs &a, hipStream_t s);

// Reverse sweep.  Columns c in [0, C); the SP column of c is c / cdiv.  The
// local seed of net n in column c is computed where it is used:
//   kappa C_n 2 (q - p) * (beta unless STE) * weight(n, c),
// with weight the upstream weight times the driver's size factor:
//   per_column: w[c] s_{c mod S'}(n);  paired: w[b] s_b(n);
//   otherwise (contracted): sum_s w[b][s] s_s(n).
struct BwdArgs {
  const float *sp;            // [n_nets][B]
  const float *beta;          // [n_nets][B], [n_nets] when beta_shared, or null (beta = 1)
  const float *cap;           // [n_nets] internal
  const float *w;             // [B][S'] (null = 1)
  const float *size;          // [S][G] internal, or null (all 1)
  float *contrib;             // [n_edges][C], in fan-out (reader) order
  float *lam;                 // [C][n_nets] internal: every net's adjoint, or null
  const uint8_t *fixed;       // [n_pi]: nonzero = excluded from the gradients (0), or null
  float kappa;
  int32_t n_pi, G, B, S, C, cdiv, ste, per_column, paired;
  int32_t beta_shared;        // one beta per net for every column
};
// Gates whose fan-out range has more than kHeavyPull entries are "heavy":
// with kSerialColumns columns or more, heavy[0, n_heavy) lists the launch
// range's heavy gates (internal ids, ascending; all of them, no others),
// which cooperative workgroups pull; fewer columns ignore the list.
constexpr int32_t kHeavyPull = 32;
hipError_t launch_bwd_level(const GraphView &g, const BwdArgs &a, int32_t g0, int32_t n,
                            bool cells, hipStream_t s, const int32_t *heavy = nullptr,
                            int32_t n_heavy = 0);
// PI adjoints -> out[c][n_pi].
// heavy[0, n_heavy): every PI with more than kHeavyPull fan-out entries
// (ascending), pulled by cooperative workgroups at kSerialColumns columns or
// more; fewer columns ignore the list.
hipError_t launch_bwd_pi(const GraphView &g, const BwdArgs &a, float *out, hipStream_t s,
                         const int32_t *heavy = nullptr, int32_t n_heavy = 0);

// Several designs in one launch: one level index of every design of a group.
// Segment k owns the blocks [block0_k, block0_{k+1}) (block0 ascending, the
// first 0); its items are the (gate, column) pairs of its level range, column
// innermost, as in the single-design launches.
struct SpSeg {
  GraphView g;
  SpLevel lv;
  // the design's next level in the same launch (fixed cells, launch_sp_pair's
  // recomputation), or n = 0; the segment's items are then (lv.n + lv2.n) B
  SpLevel lv2;
  uint32_t block0;
};
struct BwdSeg {
  GraphView g;
  BwdArgs a;
  int32_t g0, n;
  uint32_t block0;
};
// Threads per workgroup of the merged launches; a segment's block0 and the
// launch's block count are in these units.  One wave: the launches are
// latency-bound gathers, and one-wave groups spread them over more CUs.
constexpr int kMergedBlock = 64;
// segs: device array of n_segs; blocks: total blocks of the launch.
hipError_t launch_sp_multi(const SpSeg *segs, int32_t n_segs, uint32_t blocks, bool cells,
                           hipStream_t s);
hipError_t launch_bwd_multi(const BwdSeg *segs, int32_t n_segs, uint32_t blocks, bool cells,
                            hipStream_t s);

// Every net's adjoint in caller numbering, lam_out [C][n_nets], and the
// Eq. 8 score of every gate from its output net, score [C][G] caller gate
// order: |lambda| P (1 - P) / max(|1 - 2P|, eps).  Either may be null.
hipError_t launch_grad_lambda_export(const float *lam, const float *sp, const int32_t *int2ext,
                                     int32_t n_pi, int32_t n_nets, int32_t B, int32_t C,
                                     int32_t cdiv, float eps, float *lam_out, float *score,
                                     hipStream_t s);

// Power-virus ascent (Alg. 4): P <- clip(P + eta * grad) on the PI rows of
// the stored SP [n_pi][B]; grad is [B][n_pi].
hipError_t launch_virus_step(float *sp, const float *grad, float eta, int32_t n_pi, int32_t B,
                             hipStream_t s);
// v0 = [P >= 1/2] ([B][n_pi] bytes), P ([B][n_pi] floats, or null) and the
// two-cycle stimulus [B][n_pi][2]: word 0 is v0 on every lane, word 1 its
// complement.
hipError_t launch_virus_vectors(const float *sp, uint64_t *stim, uint8_t *v0, float *p_out,
                                int32_t n_pi, int32_t B, hipStream_t s);
// P_virus[b] = sum_n cap[n] [net n toggled in column b] (toggles [n_nets][B]),
// accumulated in double in a fixed order.
hipError_t launch_virus_power(const uint32_t *tog, const float *cap, int32_t n_nets, int32_t B,
                              double *out, hipStream_t s);

// Persistent (cooperative) sweeps: all levels in one launch with a grid
// barrier between levels; fixed cells only.  level_ptr is the device copy of
// the design's level table; max_items the largest level's item count.
//
// The barrier's device words (kBarrierWords uint32, zeroed by the launcher
// on the stream before each launch): one arrival flag per block (block b
// stores the number of the barrier it reached to word b; a launch has at
// most kBarrierFlags blocks) and the timeout flag.  A wait that sees no new
// arrival for limit_ticks ticks of the 100 MHz real-time counter sets the
// timeout flag and stops, and every later wait of the launch stops at once;
// the sweep's outputs are then NaN and the report word (kBarrierReport) is
// set for the host to read.
constexpr int kBarrierFlags = 1024;
constexpr int kBarrierStride = 32;  // 128 bytes
constexpr int kBarrierTimeout = kBarrierFlags;
constexpr int kBarrierWords = kBarrierTimeout + kBarrierStride;
// One more word after them, not zeroed per launch: a wait that gives up also
// sets it, so it records that some sweep since the host last cleared it
// failed.
constexpr int kBarrierReport = kBarrierWords;
constexpr int kBarrierAlloc = kBarrierWords + kBarrierStride;
struct GridBarrier {
  uint32_t *words;       // [kBarrierAlloc]
  uint64_t limit_ticks;  // 100 MHz ticks without progress before a wait gives up
};
hipError_t launch_sp_persistent(const GraphView &g, const SpLevel &lv, const int32_t *level_ptr,
                                int32_t depth, int64_t max_items, GridBarrier bar,
                                hipStream_t s);
// Reverse levels depth..1 and then the PI adjoints into pi_out[c][n_pi].
hipError_t launch_bwd_persistent(const GraphView &g, const BwdArgs &a, const int32_t *level_ptr,
                                 int32_t depth, int64_t max_items, float *pi_out,
                                 GridBarrier bar, hipStream_t s);
// dcap[ext n] = sum_{b,s} w[b][s] x[n][b] size_s(n) and dsize[s][ext g] =
// sum_b w[b][s] x[out g][b] C_out g, with x = kappa beta TR_model
// recomputed from SP and beta.
struct GradExportArgs {
  const float *sp;            // [n_nets][B]
  const float *beta;          // [n_nets][B], [n_nets] when beta_shared, or null (beta = 1)
  int32_t beta_shared;
  float kappa;
  const float *cap;           // [n_nets]
  const float *w;             // [B][S'] or null
  const float *size;          // [S][G] internal or null
  const int32_t *int2ext;
  int32_t n_pi, n_nets, G, B, S;
  int32_t paired;             // column b uses size row b
  float *dcap;                // [n_nets] caller numbering (sum over b, s) or null
  float *dsize;               // [S][G] caller gate numbering (sum over b) or null
};
hipError_t launch_grad_export(const GradExportArgs &a, hipStream_t s);

}  // namespace dp
