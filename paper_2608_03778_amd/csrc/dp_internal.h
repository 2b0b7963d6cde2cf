// Internal structures of libdiffpower (host side).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/diffpower.h"
#include "dp_kernels.h"

namespace dp {

// Thread-local error message plus status helper.
dp_status fail(dp_status st, const std::string &msg);
void clear_error();

#define DP_HIP_TRY(expr)                                                     \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess)                                                    \
      return ::dp::fail(DP_E_HIP, std::string(#expr " failed: ") +           \
                                      hipGetErrorString(_e));                \
  } while (0)

#define DP_TRY(expr)                 \
  do {                               \
    dp_status _s = (expr);           \
    if (_s != DP_OK) return _s;      \
  } while (0)

// A device allocation that frees itself.
struct DevBuf {
  void *ptr = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  dp_status alloc(size_t n);  // keeps the buffer if already large enough
  template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// A library cell compiled to stack code (encoding in dp_kernels.h).
struct CellCode {
  std::vector<uint16_t> code;
  int32_t n_in = 0;
  std::vector<std::string> inputs;  // identifiers in order of first appearance (IN index)
};
// Compile one expression; returns an error message, or "" on success.
std::string compile_cell(const char *text, CellCode *out);
// Fan-in position of each input of a compiled cell from its pin list
// (Alg. 1's perm); returns an error message, or "".
std::string pin_permutation(const CellCode &cc, const char *pins, std::vector<int32_t> *perm);
// The fixed cell (DP_INV ..) a compiled expression equals, or -1.
int fixed_op_of(const CellCode &cc);
// Truth table of a compiled cell: bit m is the cell's output when input k
// is bit k of m (m < 2^n_in; higher bits repeat the pattern).
uint64_t truth_table(const CellCode &cc);

}  // namespace dp

// Contexts and designs are reference counted: a design holds its context,
// an eval (and a server lane) holds its design, a server holds its context
// and its designs.  *_destroy drops the caller's reference, so handles may be
// destroyed in any order.
struct dp_ctx {
  int device = 0;
  hipStream_t stream = nullptr;   // stream calls enqueue on
  hipStream_t owned = nullptr;    // stream created by the library, if any
  std::atomic<int> refs{1};
};

// Immutable compiled design.  Internal numbering: PIs keep ids [0, n_pi);
// gates are sorted by (level, cell, caller id) and gate g' drives internal
// net n_pi + g'.  Level l (1..depth) holds gates [level_ptr[l], level_ptr[l+1]).
struct dp_design {
  dp_ctx *ctx = nullptr;
  std::atomic<int> refs{1};
  int32_t n_pi = 0, n_gates = 0, n_nets = 0, depth = 0;
  int64_t n_edges = 0;
  std::vector<int32_t> level_ptr;     // [depth + 2], level_ptr[1] = 0
  std::vector<int32_t> h_level;       // caller numbering, [n_nets]
  std::vector<uint8_t> h_op;          // internal order
  std::vector<int32_t> h_arity_prefix;  // [n_gates+1] internal order (for byte counts)
  std::vector<int32_t> h_int2ext;     // [n_nets]
  std::vector<int32_t> h_ext2int;     // [n_nets]
  int32_t max_level_width = 0;
  std::vector<int64_t> lvl_pins;      // [depth + 1] fan-in pins of the level's gates
  std::vector<int64_t> lvl_fanout;    // [depth + 1] fan-out edges of the level's nets (0 = PIs)
  std::vector<int64_t> lvl_read;      // [depth + 1] the level's gates whose output has readers
  // [depth + 1] fixed-cell gates of each level; its library-cell gates follow
  // them and run in kernels of their own
  std::vector<int32_t> lvl_fixed;
  // [depth + 1] library cells of each level with at most kSmallCellInputs
  // inputs; they precede the level's wider cells
  std::vector<int32_t> lvl_small_cells;
  int32_t split_levels = 0;           // levels holding both kinds (one launch more each)
  int32_t cell_levels = 0;            // levels holding library cells
  bool has_cell_gates = false;
  // device arrays
  int32_t pins = 3;      // rows of `in` and `slot`: 3, or the widest library cell
  int32_t n_cells = 0;   // distinct library-cell logics of the design (after dedup)
  // per library cell of the caller: its logic id (>= 0), or -1 - op for a
  // cell that runs as fixed cell op
  std::vector<int32_t> h_cell_logic;
  dp::DevBuf op;        // uint8 [n_gates]
  dp::DevBuf in;        // int32 [pins][n_gates] input net of pin j (SoA)
  dp::DevBuf rev_ptr;   // int32 [n_nets + 1] fan-out list offsets
  dp::DevBuf rev_edge;  // int32 [n_edges] fan-out edges, id = j * n_gates + g'
  dp::DevBuf slot;      // int32 [pins][n_gates] position of pin (g', j) in its source's fan-out list
  dp::DevBuf code;      // uint16: the library cells' stack code, concatenated
  dp::DevBuf cell;      // int32 [n_cells][3]: code offset, length, inputs
  dp::DevBuf tt;        // uint64 [n_cells] truth tables (the simulation's cell function)
  dp::DevBuf arity;     // uint8 [n_gates] input count of each gate
  dp::DevBuf level_dev; // int32 [depth + 2] device copy of level_ptr
  dp::DevBuf int2ext;   // int32 [n_nets]
  dp::DevBuf ext2int;   // int32 [n_nets]
  // gates (internal ids, ascending) and PIs with more than kHeavyPull
  // fan-out entries, and their device copies
  std::vector<int32_t> h_heavy, h_heavy_pi;
  dp::DevBuf heavy, heavy_pi;
  int64_t device_bytes = 0;
};

namespace dp {

// Device arrays of a design as the kernels see them.
inline GraphView design_view(const dp_design *d) {
  GraphView g;
  g.op = d->op.as<uint8_t>();
  g.in = d->in.as<int32_t>();
  g.rev_ptr = d->rev_ptr.as<int32_t>();
  g.rev_edge = d->rev_edge.as<int32_t>();
  g.slot = d->slot.as<int32_t>();
  g.code = d->code.as<uint16_t>();
  g.cell = d->cell.as<int32_t>();
  g.tt = d->tt.as<uint64_t>();
  g.arity = d->arity.as<uint8_t>();
  g.pins = d->pins;
  g.n_pi = d->n_pi;
  g.G = d->n_gates;
  g.n_nets = d->n_nets;
  return g;
}

// Level l as launch ranges: its fixed cells, then its library cells (ops
// sort ascending inside a level), each range of one kind; f(g0, n, cells).
template <class F>
dp_status for_level_parts(const dp_design *d, int32_t l, F &&f) {
  const int32_t g0 = d->level_ptr[l], n = d->level_ptr[l + 1] - g0, nf = d->lvl_fixed[l];
  if (nf > 0) DP_TRY(f(g0, nf, false));
  if (nf < n) DP_TRY(f(g0 + nf, n - nf, true));
  return DP_OK;
}

// Whether a probability-only sweep runs levels l and l + 1 in one launch
// (launch_sp_pair): both levels hold fixed cells only, and the pair's lanes
// are few enough that a level launch is bound by its latency rather than its
// bytes (the pair recomputes up to three gates per lane of its second level).
constexpr int64_t kPairMaxLanes = 3 << 18;
inline bool pairs_levels(const dp_design *d, int32_t l, int32_t B) {
  if (l + 1 > d->depth) return false;
  const int32_t a = d->level_ptr[l], m = d->level_ptr[l + 1], e = d->level_ptr[l + 2];
  return d->lvl_fixed[l] == m - a && d->lvl_fixed[l + 1] == e - m &&
         (int64_t)(e - a) * B <= kPairMaxLanes;
}

// The heavy gates of the launch range [g0, g0 + n): a slice of the design's
// ascending list.
struct HeavySpan {
  const int32_t *gates;
  int32_t n;
};
inline HeavySpan heavy_span(const dp_design *d, int32_t g0, int32_t n) {
  const auto lo = std::lower_bound(d->h_heavy.begin(), d->h_heavy.end(), g0);
  const auto hi = std::lower_bound(lo, d->h_heavy.end(), g0 + n);
  const int32_t k = (int32_t)(hi - lo);
  return HeavySpan{k ? d->heavy.as<int32_t>() + (lo - d->h_heavy.begin()) : nullptr, k};
}

inline HeavySpan heavy_pis(const dp_design *d) {
  const int32_t k = (int32_t)d->h_heavy_pi.size();
  return HeavySpan{k ? d->heavy_pi.as<int32_t>() : nullptr, k};
}

// Parameter validation and kappa = energy_factor Vdd^2 f (Eq. 1), shared by
// every entry point that takes a dp_params.
dp_status params_ok(const dp_params *p);
double kappa(const dp_params &p);

// The static scratch of dp_forward_static: resolve its device address on
// `device` (the device must be current; once per device).
dp_status static_scratch_init(int device);

// Host-side compile: validation, levelization, sort, renumbering and the
// device upload.  Implemented in dp_compile.cpp.
// pins: per cell, the pin names in a gate's fan-in order (null = the
// expression's inputs in order of first appearance).
dp_status compile_design(dp_ctx *ctx, const dp_netlist *nl, int32_t n_cells,
                         const char *const *cells, const char *const *pins, dp_design **out);

void ctx_retain(dp_ctx *c);
void ctx_release(dp_ctx *c);
void design_retain(dp_design *d);
void design_release(dp_design *d);

}  // namespace dp
