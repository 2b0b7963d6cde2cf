/*
 * diffpower.h -- C ABI of the MI355X (gfx950) DiffPower hot path.
 *
 * DiffPower (arXiv 2608.03778) estimates switching power of a gate netlist by
 * propagating static probabilities (SP) level by level (Sec. III-A/B,
 * Alg. 2), turns them into toggle rates under temporal independence (Eq. 2),
 * calibrates them with a bit-packed logic simulation (Sec. III-C, Eq. 4) via
 * a clipped per-net ratio beta (Sec. III-D, Eq. 5), sums C-weighted activity
 * into power (Eq. 1) and differentiates that power in one reverse sweep
 * (Sec. III-E, Eq. 6-7).  This library runs all of it on one AMD GPU.
 *
 * Conventions shared by every call:
 *  - Every call returns a dp_status; nothing throws or aborts across the
 *    ABI.  dp_last_error() returns a thread-local message for the last
 *    failing call of the calling thread.
 *  - The caller owns every buffer it passes.  dp_compile and dp_set_* copy
 *    what they need before returning (host inputs) or before the stream
 *    work they enqueue runs (device inputs).  The library owns designs,
 *    evals and servers and their device memory until *_destroy.
 *  - `on_device` = 1 means a pointer is GPU memory on the context's device
 *    (e.g. a torch tensor's data_ptr()); 0 means host memory.  Host outputs
 *    are complete when the call returns; device outputs are complete when
 *    the context's stream reaches the point where the call enqueued them.
 *  - Per-net arrays use the caller's net numbering: nets [0, n_pi) are the
 *    primary inputs (PIs), net n_pi + g is the output of gate g.  The
 *    library's internal renumbering never shows.
 *  - Floating point on the GPU is float32; counts are uint32.
 *  - Designs are immutable after dp_compile and may be shared by many evals.
 *    An eval, a server and a context are used by one host thread at a time.
 */
#ifndef DIFFPOWER_H
#define DIFFPOWER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DP_OK = 0,
  DP_E_INVALID = -1,     /* malformed argument or netlist, value out of range */
  DP_E_CYCLE = -2,       /* the netlist has a combinational cycle */
  DP_E_OOM = -3,         /* device or host allocation failed */
  DP_E_HIP = -4,         /* a HIP runtime call failed */
  DP_E_UNSUPPORTED = -5, /* a valid request the library does not implement */
  DP_E_STATE = -6,       /* call out of order (e.g. backward before forward) */
  DP_E_BUDGET = -7,      /* request can never fit the server's memory budget */
  DP_E_NOTFOUND = -8     /* unknown ticket or design id */
} dp_status;

/* The nine fixed cells (Sec. III-A routes common gates to hand-written
 * rules; AOI21 and MUX2 get their exact single-cell rules as well).
 * Pin order in brackets; the SP rule assumes independent inputs (Sec. II-B). */
enum {
  DP_INV = 0,   /* [A]        !A               SP 1-a               */
  DP_BUF = 1,   /* [A]        A                SP a                 */
  DP_AND2 = 2,  /* [A,B]      A&B              SP ab                */
  DP_OR2 = 3,   /* [A,B]      A|B              SP a+b-ab            */
  DP_NAND2 = 4, /* [A,B]      !(A&B)           SP 1-ab              */
  DP_NOR2 = 5,  /* [A,B]      !(A|B)           SP (1-a)(1-b)        */
  DP_XOR2 = 6,  /* [A,B]      A^B              SP a+b-2ab           */
  DP_AOI21 = 7, /* [A1,A2,B]  !((A1&A2)|B)     SP (1-a1 a2)(1-b)    */
  DP_MUX2 = 8,  /* [I0,I1,S]  S?I1:I0          SP (1-s)i0 + s i1    */
  DP_N_OPS = 9
};

/* Propagation modes (Sec. V-B names all three). */
enum {
  DP_MODELED = 0,     /* algebraic SP only, beta = 1 */
  DP_HYBRID = 1,      /* SP + bit-packed simulation + beta calibration */
  DP_FROZEN_BETA = 2  /* algebraic SP scaled by a beta set with dp_set_beta */
};

/* How beta enters the gradient (Eq. 6). */
enum {
  DP_BETA_LOCAL = 0, /* beta scales each net's local power term: the exact
                        gradient of sum beta*C*TR_model with beta frozen */
  DP_BETA_STE = 1    /* Eq. 6 literally: a net's accumulated gradient is
                        multiplied by its beta before it flows upstream */
};

/* Sweep schedules (see dp_eval_set_schedule). */
enum {
  DP_SCHED_AUTO = 0,      /* the autotuned choice (default) */
  DP_SCHED_LEVEL = 1,     /* one launch per level (an SP-only forward with
                             few columns: one per two levels of fixed cells,
                             the second level recomputing the pins the first
                             drives; bit for bit the same results) */
  DP_SCHED_GRAPH = 2,     /* the same launches captured once into HIP graphs,
                             one per forward sweep and one per reverse sweep
                             of dp_backward / dp_backward_columns (forward
                             sweeps of at most 1024 launches; a larger one
                             returns DP_E_UNSUPPORTED; a larger reverse sweep
                             runs launch by launch) */
  DP_SCHED_PERSISTENT = 3 /* SP-only sweeps (modeled forward, reverse sweep) as
                             one cooperative launch (at most one workgroup per
                             compute unit) with a grid barrier per level; the
                             simulation keeps one launch per level.  Opt-in:
                             the autotuner does not pick it.  Fixed cells
                             only: dp_eval_set_schedule returns
                             DP_E_UNSUPPORTED for a design with library-cell
                             gates.  A barrier wait that sees no progress for
                             dp_eval_set_barrier_timeout's limit (1 ms by
                             default; it cannot run out while the launch's
                             blocks stay resident) gives up, every later wait
                             of that launch stops at once and its outputs are
                             NaN; the eval's next host synchronization (a
                             call with host outputs, dp_power_gradients,
                             dp_power_virus or dp_eval_synchronize) then
                             returns DP_E_HIP saying so.  Each launch starts
                             with its barrier reset, so later sweeps are not
                             affected */
};

typedef struct dp_ctx dp_ctx;
typedef struct dp_design dp_design;
typedef struct dp_eval dp_eval;
typedef struct dp_server dp_server;

/* A combinational gate netlist (Sec. III-A: sequential outputs become PIs
 * with fixed probability).  fanin[fanin_ptr[g] .. fanin_ptr[g+1]) are the
 * input nets of gate g in pin order; their count must equal the cell's
 * arity.  Gates may be given in any order. */
typedef struct {
  int32_t n_pi;
  int32_t n_gates;
  const uint8_t *op;        /* [n_gates] DP_INV .. DP_MUX2, or DP_CELL_BASE + c */
  const int32_t *fanin_ptr; /* [n_gates + 1], fanin_ptr[0] = 0 */
  const int32_t *fanin;     /* [fanin_ptr[n_gates]] net ids */
} dp_netlist;

/* Electrical and calibration parameters.
 * Power = energy_factor * vdd^2 * fclk * sum_n beta_n C_eff,n TR_model,n
 * (Eq. 1 with energy_factor = 1/2).  With vdd in V, fclk in GHz and C in fF
 * the unit is uW.  beta is clipped to [beta_min, beta_max] (Eq. 5; the paper
 * uses 0.1 and 10).  n_sim is the number of simulated vectors (a multiple of
 * 64, at least 128 in DP_HYBRID); seed keys the stimulus generator. */
typedef struct {
  double vdd;
  double fclk;
  double energy_factor;
  double beta_min;
  double beta_max;
  int32_t mode;      /* DP_MODELED | DP_HYBRID | DP_FROZEN_BETA */
  int32_t beta_grad; /* DP_BETA_LOCAL | DP_BETA_STE */
  int64_t n_sim;
  uint64_t seed;
} dp_params;

/* Sizes of a compiled design. */
typedef struct {
  int32_t n_pi, n_gates, n_nets;
  int32_t depth;           /* number of gate levels */
  int64_t n_edges;         /* total fan-in pins */
  int32_t max_level_width; /* gates in the widest level */
  int32_t reserved;
  int64_t device_bytes;    /* device memory held by the design */
} dp_design_info_t;

/* Forward outputs.  Any pointer may be NULL to skip that output.  Per-net
 * arrays are [B][n_nets] (caller numbering, column-major over queries);
 * power is [B][S'] with S' = max(S, 1).  In DP_MODELED mode sp_acc, tr_acc,
 * ones and toggles are not produced (must be NULL) and beta is 1. */
typedef struct {
  float *sp;         /* static probability (Alg. 2) */
  float *tr;         /* TR_model = 2 SP (1 - SP) (Eq. 2) */
  float *sp_acc;     /* simulated SP = ones / (64 T) */
  float *tr_acc;     /* simulated TR = toggles / (64 (T - 1)) (Eq. 4) */
  float *beta;       /* clip(TR_acc / TR_model, beta_min, beta_max) (Eq. 5) */
  float *tr_hyb;     /* beta * TR_model */
  uint32_t *ones;    /* lanes at 1 over all simulated words */
  uint32_t *toggles; /* lane transitions between consecutive words */
  float *power;      /* [B][S'] switching power (Eq. 1) */
  int32_t on_device; /* all pointers above are device (1) or host (0) */
} dp_fwd_out;

/* Defaults: vdd 1, fclk 1, energy_factor 0.5, beta in [0.1, 10],
 * DP_MODELED, DP_BETA_LOCAL, n_sim 4096, seed 1. */
void dp_params_default(dp_params *p);

/* Thread-local message of the calling thread's last failure ("" if none). */
const char *dp_last_error(void);

/* Library version string. */
const char *dp_version(void);

/* --- context ----------------------------------------------------------- */
/* Bind to GPU `device`; work is enqueued on `hip_stream` (a hipStream_t;
 * NULL = the library creates and owns a non-blocking stream;
 * hipStreamLegacy = the device's null stream, e.g. the one torch uses by
 * default).  Graphs are captured on a private stream and launched on this
 * one, so any of these may be used with DP_SCHED_GRAPH.  Errors:
 * DP_E_INVALID (no such device), DP_E_HIP. */
dp_status dp_ctx_create(int32_t device, void *hip_stream, dp_ctx **out);
/* Switch the stream later calls enqueue on (same meanings as above). */
dp_status dp_ctx_set_stream(dp_ctx *ctx, void *hip_stream);
/* Block until the context's stream is idle. */
dp_status dp_ctx_synchronize(dp_ctx *ctx);
void dp_ctx_destroy(dp_ctx *ctx);

/* --- design (Sec. III-A, Alg. 1's role: build the levelized graph) ------- */
/* Validate the netlist (arity, net ids, no cycles), levelize it as soon as
 * possible (PIs at level 0, a gate one above its deepest input), sort gates
 * by (level, cell), renumber nets so a level's outputs are contiguous, build
 * the per-pin fan-in arrays and the fan-out lists, and upload everything.
 * Host inputs only; they are copied.  Errors: DP_E_INVALID, DP_E_CYCLE,
 * DP_E_OOM, DP_E_HIP. */
dp_status dp_compile(dp_ctx *ctx, const dp_netlist *netlist, dp_design **out);

/* The same with a cell library (Sec. III-A, Alg. 1-3): cells[c] is the
 * Boolean function of library cell c, and a gate whose opcode is
 * DP_CELL_BASE + c is an instance of it.  Grammar: identifiers, 0, 1,
 * parentheses, NOT '!' or '~' (binds tightest), then AND '&' or '*', XOR '^',
 * OR '|' or '+', binary operators left associative.  A cell's inputs are its
 * distinct identifiers in order of first appearance, and a gate's fan-in
 * list follows that order; at most 6 inputs, 32 operations, 8 stack entries.
 * Each expression is compiled to post-order stack code that the SP and
 * reverse kernels interpret operation by operation (the probability of an
 * operation assumes independent operands, so an expression that reads an
 * input twice, such as a multiplexer written out, gets the paper's op-by-op
 * value), with reverse-mode partials over the same code; the simulation
 * evaluates the expression's exact truth table.  Library-cell gates run in
 * kernels of their own after a level's fixed cells.  A cell needs at least
 * one input.  An expression whose
 * code is one of the fixed cells' (for example "A&B" or "!((A&B)|C)") runs
 * as that cell.  n_cells <= 240; copies the expressions.  Errors as dp_compile,
 * plus DP_E_INVALID for an expression that does not compile. */
#define DP_CELL_BASE 16
dp_status dp_compile_cells(dp_ctx *ctx, const dp_netlist *netlist, int32_t n_cells,
                           const char *const *cells, dp_design **out);
/* The same with pin lists (Alg. 1's perm): pins[c] names the pins of
 * library cell c in the order a gate of that cell lists its fan-in, names
 * separated by commas or blanks, for example "I0,I1,S" for the multiplexer
 * "(I0&!S)|(I1&S)", whose inputs in order of first appearance are
 * [I0, S, I1].  Each list names every identifier of the expression once
 * and nothing else; pins NULL or pins[c] NULL keeps the order of first
 * appearance.  Cells whose compiled code is the same share one logic id
 * (Alg. 1's dedup: one code-table entry, and their gates sort together
 * within a level).  Errors as dp_compile_cells, plus DP_E_INVALID for a pin
 * list that does not match its expression. */
dp_status dp_compile_library(dp_ctx *ctx, const dp_netlist *netlist, int32_t n_cells,
                             const char *const *cells, const char *const *pins,
                             dp_design **out);
/* Logic ids of a design's library cells: logic[c] ([n_cells] of the
 * compile call, host; may be NULL) is the id of cell c's compiled code
 * (cells with the same code share it), or -1 - op for a cell that runs as
 * fixed cell op; *n_logic (may be NULL) receives the number of distinct
 * ids.  Errors: DP_E_INVALID. */
dp_status dp_design_cell_logic(const dp_design *design, int32_t *logic, int32_t *n_logic);
dp_status dp_design_info(const dp_design *design, dp_design_info_t *out);
/* Level of every net in caller numbering ([n_nets], host). */
dp_status dp_design_levels(const dp_design *design, int32_t *level);
void dp_design_destroy(dp_design *design);

/* --- evaluation state -------------------------------------------------- */
/* Workspaces for B query columns (independent PI-probability vectors) and S
 * cell-size vectors (S = 0: no sizes, every s = 1).  Every (b, s) pair is
 * one power value.  Errors: DP_E_INVALID (B < 1, S < 0, bad params),
 * DP_E_OOM. */
dp_status dp_eval_create(dp_design *design, int32_t n_cols, int32_t n_size,
                         const dp_params *params, dp_eval **out);
dp_status dp_eval_set_params(dp_eval *ev, const dp_params *params);
void dp_eval_destroy(dp_eval *ev);

/* PI probabilities p[b][i], [B][n_pi], each in [0, 1] (Alg. 2 inputs,
 * "startpoint SPs").  DP_E_INVALID on NaN or out of range. */
dp_status dp_set_pi_prob(dp_eval *ev, const float *p, int32_t on_device);
/* Net load capacitances C[n], [n_nets] (Eq. 1), finite and >= 0. */
dp_status dp_set_caps(dp_eval *ev, const float *cap, int32_t on_device);
/* Cell size factors s[s][g], [S][n_gates], finite and >= 0.  A gate's size
 * scales the load of the net it drives: C_eff = C * s_driver. */
dp_status dp_set_cell_sizes(dp_eval *ev, const float *size, int32_t on_device);
/* Frozen calibration beta[b][n], [B][n_nets], used by DP_FROZEN_BETA. */
dp_status dp_set_beta(dp_eval *ev, const float *beta, int32_t on_device);
/* Replace the generated stimulus with explicit PI words w[b][i][t],
 * [B][n_pi][n_sim/64] (bit j of word t = lane j at cycle t); NULL restores
 * the generator.  A test and replay hook. */
dp_status dp_set_stimulus(dp_eval *ev, const uint64_t *words, int32_t on_device);
/* Startpoint stimulus model of DP_HYBRID (Sec. III-C: 64-lane words from
 * Markov chains calibrated to a target SP and TR).  tau[b][i], [B][n_pi],
 * finite in [0, 1]: the target transition rate of PI i in column b.  Each
 * lane of the PI is a two-state chain whose stationary law is its
 * probability p (dp_set_pi_prob): cycle 0 is a Bernoulli(p) draw, then a
 * lane at 1 stays with probability 1 - tau / (2p) and a lane at 0 rises with
 * probability tau / (2 (1 - p)) (computed in double, clamped to [0, 1], so a
 * tau beyond 2 min(p, 1 - p) gives the fastest chain there is).  Cycle t
 * lane j compares lane j mod 4 of Philox4x32-10(counter (t, stream, j / 4,
 * 0), key seed) with floor(probability * 2^32), as the independent
 * stimulus does.  NULL restores independent cycles (tau = 2p(1-p)).  The
 * modeled side is unchanged (Eq. 2); beta carries the difference.  An
 * explicit stimulus (dp_set_stimulus) takes precedence.  Errors:
 * DP_E_INVALID (a value out of range). */
dp_status dp_set_pi_rates(dp_eval *ev, const float *tau, int32_t on_device);
/* Shared streams (Sec. III-C: startpoints behind one sequential driver get
 * one bitstream): stream[i], [n_pi] host memory, in [0, n_pi), is the
 * Philox stream PI i draws from (its counter's second word); PIs with one
 * stream and one (p, tau) get identical words.  NULL: every PI its own
 * stream.  Applies to the generated stimulus, independent or Markov.
 * Errors: DP_E_INVALID (a stream id out of range). */
dp_status dp_set_pi_streams(dp_eval *ev, const int32_t *stream);
/* Startpoints excluded from the gradients, such as fixed infrastructure nets
 * (clocks, resets, scan enables) whose probabilities are not design
 * variables: fixed[i] nonzero, [n_pi] host memory.  Their dP/dp (and their
 * adjoint in dp_power_gradients) is 0, and dp_power_virus leaves their
 * probabilities where they are; the forward is unchanged.  NULL: none. */
dp_status dp_set_pi_fixed(dp_eval *ev, const uint8_t *fixed);

/* Forward pass over all B columns (and S size vectors): SP sweep; in
 * DP_HYBRID also stimulus, bit-packed simulation and beta; finalize; power
 * reduction.  Errors: DP_E_STATE (PI probabilities or caps never set),
 * DP_E_INVALID (output not available in this mode), DP_E_HIP. */
dp_status dp_forward(dp_eval *ev, const dp_fwd_out *out);

/* Reverse sweep (Eq. 7) of the last forward, weighted by the upstream
 * gradient w[b][s] ([B][S'], NULL = all ones; the adjoint is linear in it):
 *  dpower_dpi  [B][n_pi]     sum_s w[b][s] dP[b][s]/dp[b][i]
 *  dpower_dcap [n_nets]      sum_{b,s} w[b][s] dP[b][s]/dC[n]
 *  dpower_dsize[S][n_gates]  sum_b w[b][s] dP[b][s]/ds[s][g]   (S > 0 only)
 * Any output may be NULL.  beta, C, s and the stimulus are held fixed.
 * Errors: DP_E_STATE (no completed forward since the inputs changed). */
dp_status dp_backward(dp_eval *ev, const float *grad_power, float *dpower_dpi,
                      float *dpower_dcap, float *dpower_dsize,
                      int32_t on_device);

/* Per-(b, s) gradients with respect to the PI probabilities, [B][S'][n_pi]:
 * one multi-right-hand-side reverse sweep that applies each column b's
 * partial derivatives to its S' seeds.  Errors as dp_backward. */
dp_status dp_backward_columns(dp_eval *ev, float *dpower_dpi, int32_t on_device);

/* The forward pass and the per-(b, s) reverse sweep of dp_backward_columns
 * in one call (a sizing sweep over B PI vectors and S size vectors, Sec.
 * III-E applied to every column): power [B][S'] and dpower_dpi
 * [B][S'][n_pi], both on the device (on_device = 1) or host.  Under
 * DP_SCHED_GRAPH both sweeps are captured into one graph, so the whole
 * sweep is one graph launch (re-captured when any launch argument
 * changes; a sweep of more than 1024 launches runs launch by launch).
 * Results are bit for bit those of dp_forward followed by
 * dp_backward_columns.  Either output may be NULL.  Errors as dp_forward
 * and dp_backward. */
dp_status dp_forward_backward_columns(dp_eval *ev, float *power, float *dpower_dpi,
                                      int32_t on_device);

/* Power gradients of every net (Sec. IV): one reverse sweep after a
 * completed forward (grad_power = 1, per query column) that keeps every
 * net's adjoint.  dpower_dsp [B][n_nets] (caller numbering) receives
 * lambda_n = dPower/dP_n, the derivative with respect to the net's static
 * probability (Eq. 7; the PI entries equal dp_backward's dPower/dp).  score
 * [B][n_gates] (caller gate order) receives the sizing score of Eq. 8 for the
 * gate driving each net, through the chain rule of Eq. 2:
 *   S = |dP/dP_sw| * P_sw = |lambda_n| P_n (1 - P_n) / |1 - 2 P_n|,
 * with 2^-20 standing in for |1 - 2 P_n| where the activity is flat in P.
 * Either output may be NULL; host or device memory as on_device.  Returns
 * after the outputs are written.  Errors: DP_E_STATE (no forward for the
 * current inputs), DP_E_HIP, DP_E_OOM. */
dp_status dp_power_gradients(dp_eval *ev, float *dpower_dsp, float *score,
                             int32_t on_device);

/* Power-virus search by gradient ascent (Sec. IV-B, Alg. 4).  Each of the
 * eval's B columns is one ascent that starts from its PI probabilities (set
 * with dp_set_pi_prob; Alg. 4 starts every startpoint at 0.5).  `steps`
 * times, a forward and a reverse sweep give the gradient of the proxy of
 * Eq. 9 at net level, P_proxy = sum_n beta_n C_n 2 P_n (1 - P_n) (beta = 1 in
 * DP_MODELED; the frozen beta in DP_FROZEN_BETA, Alg. 4's optional scaling),
 * and P <- clip(P + eta * grad, 0, 1).  Then v0 = [P >= 1/2], v1 = 1 - v0,
 * and P_virus = sum_n C_n [net n differs between v0 and v1] (Eq. 3 at net
 * level) comes from a two-cycle bit-parallel simulation of the pair.
 * Outputs (host or device memory as on_device; each may be NULL): v0
 * [B][n_pi] bytes (0/1), p_final [B][n_pi], p_virus [B] (double).  The
 * eval's PI probabilities are left at p_final.  Returns after the results
 * are written.  Needs DP_MODELED or DP_FROZEN_BETA and S = 0.
 * Errors: DP_E_STATE, DP_E_UNSUPPORTED, DP_E_INVALID, DP_E_HIP, DP_E_OOM. */
dp_status dp_power_virus(dp_eval *ev, int32_t steps, double eta, uint8_t *v0,
                         float *p_final, double *p_virus, int32_t on_device);

/* Schedule of the level sweeps (DP_SCHED_*), the number of simulated words
 * held on the device at once (0 = automatic; otherwise a multiple of 2 that
 * splits the n_sim/64 words into chunks carrying a two-word halo), and the
 * word pairs each simulation lane handles per wave (1, 2, 4 or 8; 0 =
 * automatic).  Results are bitwise independent of all three.  Choosing
 * DP_SCHED_PERSISTENT the first time allocates the eval's two barrier words
 * (8 bytes of device memory, zeroed on the eval's stream).
 * Errors: DP_E_INVALID (unknown schedule or tiling), DP_E_UNSUPPORTED
 * (persistent with library cells), DP_E_OOM, DP_E_HIP. */
dp_status dp_eval_set_schedule(dp_eval *ev, int32_t schedule,
                               int64_t words_per_chunk,
                               int32_t sim_pairs_per_lane);

/* Autotuner: time the forward sweep, followed by the reverse sweep when
 * with_backward is nonzero (one warm-up and `reps` timed runs with HIP
 * events on the context's stream), for every schedule candidate --
 * per-level launches or a captured HIP graph (the persistent schedule is
 * opt-in only, through dp_eval_set_schedule); 1/2/4/8 word pairs per lane;
 * the whole run or 2 or 4 word chunks; 1/2/4
 * simulation streams -- and keep the fastest.  Needs the inputs set;
 * overwrites the eval's results.  best_ms (may be NULL) receives the
 * winner's time. */
dp_status dp_eval_autotune(dp_eval *ev, int32_t reps, int32_t with_backward,
                           double *best_ms);
/* Number of streams that simulate independent (query column, word chunk)
 * pieces concurrently, each with its own word buffer (0 = automatic = 1).
 * Counts are integer sums, so results do not depend on it.  A captured
 * graph (DP_SCHED_GRAPH) records its pieces on one stream. */
dp_status dp_eval_set_sim_streams(dp_eval *ev, int32_t sim_streams);
/* Query columns one simulation launch covers (each column with a word
 * buffer of its own; 0 = automatic: as many as the word budget of 32 GiB
 * per simulation stream holds, at least one).  Fewer columns per launch
 * mean more launches per level; counts do not depend on it.
 * Errors: DP_E_INVALID (columns < 0). */
dp_status dp_eval_set_sim_columns(dp_eval *ev, int32_t columns);
/* The schedule in force (as set or as chosen by the autotuner). */
dp_status dp_eval_get_schedule(const dp_eval *ev, int32_t *schedule,
                               int64_t *words_per_chunk,
                               int32_t *sim_pairs_per_lane,
                               int32_t *sim_streams);

/* Block until the eval's stream is idle.  Returns DP_E_HIP if a persistent
 * sweep since the eval's last host synchronization had a grid-barrier wait
 * give up (its outputs are NaN). */
dp_status dp_eval_synchronize(dp_eval *ev);
/* Time a grid-barrier wait of the persistent schedule may see no progress
 * before it gives up (microseconds, finite, >= 0; default 1000).  A guard
 * against a sweep whose blocks are not all resident, and a way for tests
 * to make the give-up path run: at 0 every wait that has to wait at all
 * gives up.  Errors: DP_E_INVALID. */
dp_status dp_eval_set_barrier_timeout(dp_eval *ev, double microseconds);

/* Kernel timing of the last forward/backward, accumulated with HIP events
 * on the context's stream while profiling is enabled. */
typedef struct {
  double sim_ms;          /* simulation level kernels, summed per launch */
  int64_t sim_launches;
  double sim_bytes;       /* algorithmic bytes moved by those launches */
  double sp_ms;           /* SP level kernels (modeled sweeps) */
  int64_t sp_launches;
  double sp_bytes;
  double bwd_ms;          /* reverse level kernels */
  int64_t bwd_launches;
  double bwd_bytes;
  double stim_ms;         /* stimulus generation */
  int64_t stim_launches;
} dp_profile;
dp_status dp_eval_profile(dp_eval *ev, int32_t enable);
dp_status dp_eval_get_profile(dp_eval *ev, dp_profile *out);

/* --- forward without allocation ----------------------------------------- */
/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * forward as dp_forward on a one-column eval in DP_MODELED or DP_FROZEN_BETA
 * (the same launches: one per level, or one per two levels of fixed cells;
 * bit for bit the same results), without an eval: the
 * SP, the internal capacitances and beta and the power partial sums
 * live in a static device array of the library
 * (24 MiB on each GPU it runs on, held until the process ends; its
 * device address is resolved once per GPU by dp_ctx_create).  The call
 * allocates nothing, enqueues on the design's context stream and does not
 * synchronize; the caller still provides every input and output.
 *  pi_prob [n_pi], cap [n_nets] (caller numbering), beta [n_nets] (caller
 *  numbering; DP_FROZEN_BETA only, else NULL), power [1], sp and tr
 *  [n_nets] (caller numbering, each may be NULL): all device memory on the
 *  context's GPU.  Input values are not checked (a NaN or an out-of-range
 *  probability gives NaN or unclipped results).
 * Limit: at most 2^21 nets (2,097,152).  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents: calls that overlap on
 * one GPU (two streams, or two host threads) race and must be serialized
 * by the caller.  Errors: DP_E_INVALID (NULL argument, bad params, beta
 * given in the wrong mode, more nets than the limit), DP_E_UNSUPPORTED
 * (DP_HYBRID), DP_E_STATE (no context was created on the design's GPU),
 * DP_E_HIP. */
dp_status dp_forward_static(const dp_design *design, const dp_params *params,
                            const float *pi_prob, const float *cap, const float *beta,
                            float *power, float *sp, float *tr);

/* --- design groups: several designs in one launch ----------------------- */
/* A group runs several evals -- of any designs of one context, of uneven
 * sizes -- as one unit (the batched form over designs): their forward sweeps,
 * and with `backward` their reverse sweeps, are enqueued on up to four branch
 * streams (the hardware queues a process gets by default; longest sweeps
 * first, each to the least loaded branch), forked from and joined back into
 * the context's stream.  Up to 1024 launches in total the whole unit is
 * captured once into a HIP graph, recorded on one stream (no branches), and
 * each run is one graph launch; larger units, and use_graph = 0, are
 * enqueued directly on the branches.  Results are bitwise
 * those of dp_forward and dp_backward on each eval alone (per-level
 * launches, grad_power = 1).
 *
 * The group does not own the evals: they must outlive it, and must not be
 * used elsewhere while a run is in flight.  Every eval's design must belong
 * to `ctx`; an eval may appear once; serving lanes cannot join.
 * Errors: DP_E_INVALID, DP_E_HIP, DP_E_OOM. */
typedef struct dp_group dp_group;
dp_status dp_group_create(dp_ctx *ctx, dp_eval *const *evals, int32_t n_evals,
                          dp_group **out);
/* One run: the forward of every eval and, if backward != 0, its reverse
 * sweep.  outs: NULL, or n_evals output descriptors (as dp_forward; each
 * with its own on_device).  dpower_dpi: NULL, or n_evals pointers (each
 * NULL or [B_i][n_pi_i], host or device as on_device) for dPower/dp.
 * Errors: DP_E_STATE (an eval's inputs are missing), DP_E_INVALID, DP_E_HIP,
 * DP_E_OOM. */
dp_status dp_group_run(dp_group *g, int32_t backward, const dp_fwd_out *outs,
                       float *const *dpower_dpi, int32_t on_device);
/* use_graph = 0 never captures (direct enqueue on the branches);
 * max_branches = 0 is automatic (4), otherwise at most that many branches
 * (1 = one after another, in one stream).  Errors: DP_E_INVALID. */
dp_status dp_group_configure(dp_group *g, int32_t use_graph, int32_t max_branches);
void dp_group_destroy(dp_group *g);

/* --- serving: continuous batching of queries (see dp_server_*) ---------- */
enum { DP_Q_FWD = 0, DP_Q_FWD_BWD = 1 };

/* One query against a device-resident design.  Host buffers; they must stay
 * valid until dp_wait/dp_poll reports the ticket done. */
typedef struct {
  int32_t design_id;
  int32_t kind;             /* DP_Q_FWD | DP_Q_FWD_BWD */
  const float *pi_prob;     /* [n_pi] */
  const float *cap_scale;   /* [n_gates] per-gate size factor, NULL = 1 */
  float *power;             /* [1] out */
  float *dpower_dpi;        /* [n_pi] out (DP_Q_FWD_BWD), may be NULL */
} dp_query;

/* A server owns a scheduler thread and the device memory of its query
 * slots; `hbm_budget_bytes` bounds the slot memory it may hold at once.
 * The scheduler admits waiting queries into slots of their design and
 * launches what it admitted in one pass as one device step: the slots of
 * all designs in the step share one kernel launch per level index (and per
 * reverse level), so queries that arrive while the device is busy are
 * batched across designs.  A query's results do not depend on the step it
 * rides in. */
dp_status dp_server_create(dp_ctx *ctx, size_t hbm_budget_bytes,
                           dp_server **out);
/* Batching limits: at most max_batch queries per device step (over all
 * its designs) and max_inflight steps on the device at once (defaults 64
 * and 8; 1 and 1 serve one query at a time, first come first served). */
dp_status dp_server_configure(dp_server *srv, int32_t max_batch,
                              int32_t max_inflight);
/* Register a compiled design.  Queries use params->mode (DP_MODELED, or
 * DP_FROZEN_BETA with beta calibrated once here at p = 0.5 from
 * params->n_sim vectors). */
dp_status dp_server_add_design(dp_server *srv, dp_design *design,
                               const float *cap, const dp_params *params,
                               int32_t *design_id);
/* Enqueue a query; returns at once.  DP_E_BUDGET if the query alone can
 * never fit the budget, DP_E_INVALID for a probability outside [0, 1].
 * cap_scale is checked when the query is staged for the device; a bad entry
 * makes dp_wait return DP_E_INVALID for that query. */
dp_status dp_submit(dp_server *srv, const dp_query *q, uint64_t *ticket);
dp_status dp_poll(dp_server *srv, uint64_t ticket, int32_t *done);
/* Block until the ticket is done; latency_s = completion - submission. */
dp_status dp_wait(dp_server *srv, uint64_t ticket, double *latency_s);
typedef struct {
  int64_t submitted, completed, device_steps;
  double busy_s;            /* time with device work in flight */
  int64_t peak_slot_bytes;  /* slot memory high-water mark */
  int32_t max_inflight;     /* most queries on the device at once */
  int32_t reserved;
  int64_t lanes_created;    /* slot groups allocated */
  int64_t lanes_freed;      /* idle slot groups freed to make room under the budget */
  int64_t memory_waits;     /* times a waiting query found no memory for a slot */
} dp_server_stats;
dp_status dp_server_get_stats(dp_server *srv, dp_server_stats *out);
void dp_server_destroy(dp_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* DIFFPOWER_H */
