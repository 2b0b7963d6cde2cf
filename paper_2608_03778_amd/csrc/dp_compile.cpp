// Design compilation (host): the levelized graph of Sec. III-A.
//
// The paper levelizes a pin-level DAG so that every node of level L depends
// only on levels < L and all nodes of a level run in one launch.  Here the
// graph is net-level: a sink pin always carries its driver's value, so the
// per-level wire copy of Alg. 2 folds into the gate's gather, and power,
// which sums over nets (Eq. 1), is unchanged.
//
// Steps: validate -> ASAP levels with Kahn's algorithm (cycle detection) ->
// counting sort of gates by (level, kind, heavy fan-out first, cell), then
// by first fan-in net -> renumber nets so
// level l's outputs are one contiguous range and a gate's output id is
// implicit -> per-pin fan-in arrays (structure of arrays) -> fan-out lists
// (reverse CSR, edges in ascending order, which fixes the summation order
// of the reverse sweep) -> upload.
#include <algorithm>
#include <cstring>
#include <numeric>

#include "dp_internal.h"

namespace dp {

static const int kArity[DP_N_OPS] = {1, 1, 2, 2, 2, 2, 2, 3, 3};

dp_status DevBuf::alloc(size_t n) {
  if (n <= bytes && ptr) return DP_OK;
  release();
  if (n == 0) n = 16;
  hipError_t e = hipMalloc(&ptr, n);
  if (e != hipSuccess) {
    ptr = nullptr;
    (void)hipGetLastError();
    return fail(DP_E_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed: " +
                              hipGetErrorString(e));
  }
  bytes = n;
  return DP_OK;
}

template <class T>
static dp_status upload(DevBuf &buf, const std::vector<T> &v, hipStream_t s) {
  DP_TRY(buf.alloc(std::max<size_t>(v.size() * sizeof(T), 16)));
  if (!v.empty())
    DP_HIP_TRY(hipMemcpyAsync(buf.ptr, v.data(), v.size() * sizeof(T),
                              hipMemcpyHostToDevice, s));
  return DP_OK;
}

dp_status compile_design(dp_ctx *ctx, const dp_netlist *nl, int32_t n_cells,
                         const char *const *cells, const char *const *pins, dp_design **out) {
  if (!ctx || !nl || !out) return fail(DP_E_INVALID, "dp_compile: NULL argument");
  if (n_cells < 0 || n_cells > 256 - kCellBase || (n_cells > 0 && !cells))
    return fail(DP_E_INVALID, "dp_compile: need 0 <= n_cells <= 240 and a cell array");
  // library cells (Alg. 1): compile each expression; map each pin list onto
  // the expression's inputs (perm: the fan-in position of input k); an
  // expression that is one of the fixed cells runs as that cell; the others
  // share one logic id per distinct code (dedup), and the kernels see logic
  // ids only
  std::vector<CellCode> lib(n_cells);
  std::vector<std::vector<int32_t>> perm(n_cells);
  std::vector<int> as_fixed(n_cells, -1), logic(n_cells, -1);
  std::vector<int32_t> logic_cell;  // a cell of each logic id
  for (int32_t c = 0; c < n_cells; ++c) {
    std::string err = compile_cell(cells[c], &lib[c]);
    if (err.empty() && pins && pins[c]) err = pin_permutation(lib[c], pins[c], &perm[c]);
    if (!err.empty())
      return fail(DP_E_INVALID, "dp_compile: cell " + std::to_string(c) + ": " + err);
    if (perm[c].empty()) {
      perm[c].resize(lib[c].n_in);
      std::iota(perm[c].begin(), perm[c].end(), 0);
    }
    as_fixed[c] = fixed_op_of(lib[c]);
    if (as_fixed[c] >= 0) continue;
    int32_t id = 0;
    while (id < (int32_t)logic_cell.size() && lib[logic_cell[id]].code != lib[c].code) ++id;
    if (id == (int32_t)logic_cell.size()) logic_cell.push_back(c);
    logic[c] = id;
  }
  const int32_t n_logic = (int32_t)logic_cell.size();
  auto arity_of_op = [&](int op) -> int {
    if (op < DP_N_OPS) return kArity[op];
    if (op >= kCellBase && op - kCellBase < n_cells) return lib[op - kCellBase].n_in;
    return -1;
  };
  auto internal_op = [&](int op) -> int {
    if (op < kCellBase) return op;
    const int c = op - kCellBase;
    return as_fixed[c] >= 0 ? as_fixed[c] : kCellBase + logic[c];
  };
  const int32_t n_pi = nl->n_pi, G = nl->n_gates;
  if (n_pi < 0 || G < 0) return fail(DP_E_INVALID, "dp_compile: negative size");
  if ((int64_t)n_pi + G > INT32_MAX / 2)
    return fail(DP_E_INVALID, "dp_compile: too many nets");
  if (G > 0 && (!nl->op || !nl->fanin_ptr || !nl->fanin))
    return fail(DP_E_INVALID, "dp_compile: NULL netlist array");
  const int32_t n_nets = n_pi + G;
  if (G > 0 && nl->fanin_ptr[0] != 0)
    return fail(DP_E_INVALID, "dp_compile: fanin_ptr[0] must be 0");
  for (int32_t g = 0; g < G; ++g) {
    if (arity_of_op(nl->op[g]) < 0)
      return fail(DP_E_INVALID, "dp_compile: gate " + std::to_string(g) + " has unknown cell " +
                                    std::to_string(nl->op[g]));
    if (nl->fanin_ptr[g + 1] - nl->fanin_ptr[g] != arity_of_op(nl->op[g]))
      return fail(DP_E_INVALID, "dp_compile: gate " + std::to_string(g) +
                                    " has the wrong number of inputs");
    for (int32_t e = nl->fanin_ptr[g]; e < nl->fanin_ptr[g + 1]; ++e)
      if (nl->fanin[e] < 0 || nl->fanin[e] >= n_nets)
        return fail(DP_E_INVALID, "dp_compile: gate " + std::to_string(g) +
                                      " reads net id out of range");
  }
  const int64_t n_edges = G > 0 ? nl->fanin_ptr[G] : 0;

  // --- ASAP levels by Kahn's algorithm over gate->gate edges
  std::vector<int32_t> indeg(G, 0), cons_ptr(G + 1, 0), cons;
  for (int32_t g = 0; g < G; ++g)
    for (int32_t e = nl->fanin_ptr[g]; e < nl->fanin_ptr[g + 1]; ++e)
      if (nl->fanin[e] >= n_pi) {
        ++indeg[g];
        ++cons_ptr[nl->fanin[e] - n_pi + 1];
      }
  for (int32_t d = 0; d < G; ++d) cons_ptr[d + 1] += cons_ptr[d];
  cons.resize(cons_ptr[G]);
  {
    std::vector<int32_t> fill(cons_ptr.begin(), cons_ptr.end() - 1);
    for (int32_t g = 0; g < G; ++g)
      for (int32_t e = nl->fanin_ptr[g]; e < nl->fanin_ptr[g + 1]; ++e)
        if (nl->fanin[e] >= n_pi) cons[fill[nl->fanin[e] - n_pi]++] = g;
  }
  std::vector<int32_t> level(n_nets, 0), queue;
  queue.reserve(G);
  for (int32_t g = 0; g < G; ++g)
    if (indeg[g] == 0) queue.push_back(g);
  for (size_t h = 0; h < queue.size(); ++h) {
    int32_t g = queue[h];
    int32_t l = 0;
    for (int32_t e = nl->fanin_ptr[g]; e < nl->fanin_ptr[g + 1]; ++e)
      l = std::max(l, level[nl->fanin[e]]);
    level[n_pi + g] = l + 1;
    for (int32_t c = cons_ptr[g]; c < cons_ptr[g + 1]; ++c)
      if (--indeg[cons[c]] == 0) queue.push_back(cons[c]);
  }
  if ((int32_t)queue.size() != G)
    return fail(DP_E_CYCLE, "dp_compile: the netlist has a combinational cycle (" +
                                std::to_string(G - (int32_t)queue.size()) +
                                " gates on or behind it)");
  int32_t depth = 0;
  for (int32_t g = 0; g < G; ++g) depth = std::max(depth, level[n_pi + g]);

  // --- counting sort by (level, kind, heavy first, cell); stable, so caller
  // id breaks ties.  Within a level the fixed cells precede the library
  // cells (each kind runs in kernels of its own).  Within each kind the
  // gates whose output has more than kHeavyFanout readers are then spread
  // one per 64 positions from the start of the range: with many columns the
  // reverse sweep sums their long fan-out ranges in several dependent load
  // rounds, which then overlap the rest of the level instead of trailing
  // it, and with few columns no wave holds more than one of them, so each
  // wave's long ranges still go out in one round.
  constexpr int32_t kHeavyFanout = kHeavyPull;
  // per level: [kind 1024][class 512][heavy 256][cell < 256]; the class of a
  // library cell is its input count above kSmallCellInputs (the simulation
  // runs the two classes in launches of their own), always 0 for fixed cells
  constexpr int32_t kSlots = 2048;
  auto big_cell = [&](int32_t op) {
    return op >= dp::kCellBase && lib[logic_cell[op - dp::kCellBase]].n_in > kSmallCellInputs;
  };
  auto key_of = [&](int32_t g) {
    const int32_t op = internal_op(nl->op[g]);
    const bool cell = op >= dp::kCellBase;
    const bool heavy = cons_ptr[g + 1] - cons_ptr[g] > kHeavyFanout;
    return level[n_pi + g] * kSlots + (cell ? 1024 : 0) + (big_cell(op) ? 512 : 0) +
           (heavy ? 0 : 256) + (cell ? op - dp::kCellBase : op);
  };
  const int32_t n_keys = (depth + 1) * kSlots;
  std::vector<int32_t> key_ptr(n_keys + 1, 0);
  for (int32_t g = 0; g < G; ++g) ++key_ptr[key_of(g) + 1];
  for (int32_t k = 0; k < n_keys; ++k) key_ptr[k + 1] += key_ptr[k];
  std::vector<int32_t> gate_of(G);  // internal -> caller gate
  {
    std::vector<int32_t> fill(key_ptr.begin(), key_ptr.end() - 1);
    for (int32_t g = 0; g < G; ++g) gate_of[fill[key_of(g)]++] = g;
    // Level by level: within each (kind, class, heavy, cell) bucket, order
    // gates by the internal id of their first fan-in net (stable), so
    // consecutive waves of the simulation read that pin's rows in address
    // order; then spread each (level, kind, class)'s heavy gates (sorted
    // first) one per 64.
    std::vector<int32_t> pos(G, 0), part;
    auto src_of = [&](int32_t g) {
      const int32_t n = nl->fanin[nl->fanin_ptr[g]];
      return n < n_pi ? n : n_pi + pos[n - n_pi];
    };
    for (int32_t l = 1; l <= depth; ++l) {
      for (int32_t k = l * kSlots; k < (l + 1) * kSlots; ++k) {
        const int32_t a = key_ptr[k], b = key_ptr[k + 1];
        if (b - a > 1)
          std::stable_sort(gate_of.begin() + a, gate_of.begin() + b,
                           [&](int32_t x, int32_t y) { return src_of(x) < src_of(y); });
      }
      for (int32_t kc = 0; kc < 4; ++kc) {  // (kind, class)
        const int32_t k0 = l * kSlots + kc * 512;
        const int32_t a = key_ptr[k0], h = key_ptr[k0 + 256] - a, b = key_ptr[k0 + 512];
        if (h == 0 || h == b - a) continue;
        part.assign(gate_of.begin() + a, gate_of.begin() + b);
        int32_t hi = 0, ni = h;  // next heavy, next other
        for (int32_t i = 0; i < b - a; ++i) {
          const bool take_heavy = hi < h && (i % 64 == 0 || ni == b - a);
          gate_of[a + i] = take_heavy ? part[hi++] : part[ni++];
        }
      }
      for (int32_t i = key_ptr[l * kSlots]; i < key_ptr[(l + 1) * kSlots]; ++i) pos[gate_of[i]] = i;
    }
  }
  auto *d = new dp_design();
  d->ctx = ctx;
  d->n_pi = n_pi;
  d->n_gates = G;
  d->n_nets = n_nets;
  d->depth = depth;
  d->n_edges = n_edges;
  d->level_ptr.assign(depth + 2, 0);
  for (int32_t l = 1; l <= depth + 1; ++l)
    d->level_ptr[l] = (l <= depth) ? key_ptr[l * kSlots] : G;
  d->level_ptr[0] = 0;
  for (int32_t l = 1; l <= depth; ++l)
    d->max_level_width = std::max(d->max_level_width, d->level_ptr[l + 1] - d->level_ptr[l]);
  d->h_level = level;
  d->h_int2ext.resize(n_nets);
  d->h_ext2int.resize(n_nets);
  for (int32_t i = 0; i < n_pi; ++i) d->h_int2ext[i] = d->h_ext2int[i] = i;
  for (int32_t gi = 0; gi < G; ++gi) {
    d->h_int2ext[n_pi + gi] = n_pi + gate_of[gi];
    d->h_ext2int[n_pi + gate_of[gi]] = n_pi + gi;
  }
  int32_t pins_max = 3;
  for (int32_t g = 0; g < G; ++g) pins_max = std::max(pins_max, arity_of_op(nl->op[g]));
  const int32_t pins_rows = pins_max;
  d->pins = pins_max;
  d->n_cells = n_logic;
  d->h_cell_logic.resize(n_cells);
  for (int32_t c = 0; c < n_cells; ++c)
    d->h_cell_logic[c] = as_fixed[c] >= 0 ? -1 - as_fixed[c] : logic[c];
  d->h_op.resize(G);
  d->h_arity_prefix.assign(G + 1, 0);
  std::vector<int32_t> in((size_t)pins_rows * G, 0);
  std::vector<int32_t> rev_ptr(n_nets + 1, 0), rev_edge(n_edges);
  for (int32_t gi = 0; gi < G; ++gi) {
    int32_t g = gate_of[gi];
    d->h_op[gi] = (uint8_t)internal_op(nl->op[g]);
    int32_t k = nl->fanin_ptr[g + 1] - nl->fanin_ptr[g];
    d->h_arity_prefix[gi + 1] = d->h_arity_prefix[gi] + k;
    // a library cell's input j comes from fan-in position perm[j] (its pin
    // list); fixed cells read their pins in order
    const int32_t *pm = nl->op[g] >= kCellBase ? perm[nl->op[g] - kCellBase].data() : nullptr;
    for (int32_t j = 0; j < pins_rows; ++j) {
      // unused pins alias pin 0 so that no index is ever out of range
      const int32_t pos = j < k ? (pm ? pm[j] : j) : (pm ? pm[0] : 0);
      in[(size_t)j * G + gi] = d->h_ext2int[nl->fanin[nl->fanin_ptr[g] + pos]];
    }
    for (int32_t j = 0; j < k; ++j) ++rev_ptr[in[(size_t)j * G + gi] + 1];
  }
  for (int32_t n = 0; n < n_nets; ++n) rev_ptr[n + 1] += rev_ptr[n];
  {
    // ascending internal gate, then pin: a fixed order for the reverse sums
    std::vector<int32_t> fill(rev_ptr.begin(), rev_ptr.end() - 1);
    for (int32_t gi = 0; gi < G; ++gi) {
      int32_t k = d->h_arity_prefix[gi + 1] - d->h_arity_prefix[gi];
      for (int32_t j = 0; j < k; ++j) {
        int32_t src = in[(size_t)j * G + gi];
        rev_edge[fill[src]++] = j * G + gi;
      }
    }
  }
  // slot[j][g'] = where pin j of gate g' sits in its source net's fan-out
  // list: the reverse sweep writes a pin's contribution there, so a net sums
  // one contiguous range
  std::vector<int32_t> slot((size_t)pins_rows * G, 0);
  for (int64_t e = 0; e < n_edges; ++e) slot[rev_edge[e]] = (int32_t)e;
  d->lvl_pins.assign(depth + 1, 0);
  d->lvl_fanout.assign(depth + 1, 0);
  d->lvl_read.assign(depth + 1, 0);
  for (int32_t l = 1; l <= depth; ++l)
    for (int32_t gi = d->level_ptr[l]; gi < d->level_ptr[l + 1]; ++gi) {
      d->lvl_pins[l] += d->h_arity_prefix[gi + 1] - d->h_arity_prefix[gi];
      d->lvl_fanout[l] += rev_ptr[n_pi + gi + 1] - rev_ptr[n_pi + gi];
      d->lvl_read[l] += rev_ptr[n_pi + gi + 1] > rev_ptr[n_pi + gi];
    }
  d->lvl_fanout[0] = rev_ptr[n_pi] - rev_ptr[0];
  // gates whose fan-out range the many-column reverse levels pull with
  // whole workgroups (ascending internal id)
  for (int32_t gi = 0; gi < G; ++gi)
    if (rev_ptr[n_pi + gi + 1] - rev_ptr[n_pi + gi] > kHeavyPull) d->h_heavy.push_back(gi);
  for (int32_t i = 0; i < n_pi; ++i)
    if (rev_ptr[i + 1] - rev_ptr[i] > kHeavyPull) d->h_heavy_pi.push_back(i);
  d->lvl_fixed.assign(depth + 1, 0);
  d->lvl_small_cells.assign(depth + 1, 0);
  for (int32_t l = 1; l <= depth; ++l) {
    const int32_t g0 = d->level_ptr[l], g1 = d->level_ptr[l + 1];
    int32_t f = g0;
    while (f < g1 && d->h_op[f] < kCellBase) ++f;
    d->lvl_fixed[l] = f - g0;
    int32_t sc = f;
    while (sc < g1 && !big_cell(d->h_op[sc])) ++sc;
    d->lvl_small_cells[l] = sc - f;
    if (f < g1) {
      d->has_cell_gates = true;
      ++d->cell_levels;
    }
    if (f > g0 && f < g1) ++d->split_levels;
  }
  // code of each logic id, padded to kCellMaxCode words (64 bytes, so a lane
  // loads it whole with four aligned 16-byte loads), and the logic table
  std::vector<uint16_t> code((size_t)std::max(n_logic, 1) * kCellMaxCode, 0);
  std::vector<int32_t> cell_tab(3 * (size_t)std::max(n_logic, 1), 0);
  std::vector<uint64_t> tt((size_t)std::max(n_logic, 1), 0);
  for (int32_t id = 0; id < n_logic; ++id) {
    const CellCode &cc = lib[logic_cell[id]];
    cell_tab[3 * id] = id * kCellMaxCode;
    cell_tab[3 * id + 1] = (int32_t)cc.code.size();
    cell_tab[3 * id + 2] = cc.n_in;
    std::copy(cc.code.begin(), cc.code.end(), code.begin() + (size_t)id * kCellMaxCode);
    tt[id] = truth_table(cc);
  }
  std::vector<uint8_t> arity(std::max(G, 1), 0);
  for (int32_t gi = 0; gi < G; ++gi)
    arity[gi] = (uint8_t)(d->h_arity_prefix[gi + 1] - d->h_arity_prefix[gi]);
  hipStream_t s = ctx->stream;
  dp_status st = DP_OK;
  if ((st = upload(d->code, code, s)) != DP_OK || (st = upload(d->cell, cell_tab, s)) != DP_OK ||
      (st = upload(d->tt, tt, s)) != DP_OK || (st = upload(d->arity, arity, s)) != DP_OK ||
      (st = upload(d->op, d->h_op, s)) != DP_OK || (st = upload(d->in, in, s)) != DP_OK ||
      (st = upload(d->rev_ptr, rev_ptr, s)) != DP_OK ||
      (st = upload(d->rev_edge, rev_edge, s)) != DP_OK ||
      (st = upload(d->slot, slot, s)) != DP_OK ||
      (st = upload(d->level_dev, d->level_ptr, s)) != DP_OK ||
      (st = upload(d->int2ext, d->h_int2ext, s)) != DP_OK ||
      (st = upload(d->ext2int, d->h_ext2int, s)) != DP_OK ||
      (st = upload(d->heavy, d->h_heavy, s)) != DP_OK ||
      (st = upload(d->heavy_pi, d->h_heavy_pi, s)) != DP_OK) {
    delete d;
    return st;
  }
  hipError_t e = hipStreamSynchronize(s);  // host vectors above go out of scope
  if (e != hipSuccess) {
    delete d;
    return fail(DP_E_HIP, std::string("dp_compile: upload failed: ") + hipGetErrorString(e));
  }
  d->device_bytes = (int64_t)(d->op.bytes + d->in.bytes + d->rev_ptr.bytes + d->rev_edge.bytes +
                              d->slot.bytes + d->int2ext.bytes + d->ext2int.bytes +
                              d->code.bytes + d->cell.bytes + d->tt.bytes + d->arity.bytes + d->heavy.bytes +
                              d->heavy_pi.bytes);
  ctx_retain(ctx);
  *out = d;
  return DP_OK;
}

}  // namespace dp
