// gfx950 kernels of the DiffPower hot path.
//
// Layouts (internal net numbering, see dp_design):
//   SP (packed, see sp_load)       float  [n_nets][B]      (query column innermost)
//   beta                           float  [n_nets][B]      (hybrid; a frozen beta is read as given)
//   contrib                        float  [n_edges][C]     (fan-out order of the reader)
//   simulation words W             uint64 [n_nets][pitch]  (one chunk of cycles)
//   ones, toggles                  uint32 [n_nets][B]
//
// Work mapping: the SP and reverse kernels give one lane to each
// (gate or net, column).  The simulation kernel gives one 64-lane wave to a
// (gate, run of word pairs): the wave's cell is uniform, so the cell switch
// is a scalar branch outside the word loop; each lane moves 16-byte word
// pairs, so every fan-in row is read as contiguous 1 KiB wave-wide accesses.

#include <algorithm>

#include "dp_kernels.h"

namespace dp {
namespace {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / 64;
// The simulation level runs in smaller workgroups: finer grains fill the
// chip's last wave of blocks more evenly (0.5% per level on MI355X against
// 256 threads; 64 threads gained nothing further).
constexpr int kSimBlock = 128;
constexpr int kSimWaves = kSimBlock / 64;
// Per-level SP and reverse launches are latency-bound gathers with few items
// (one per gate and column): one-wave workgroups spread a level over as many
// CUs as it has waves, so no CU's address unit serialises several waves'
// gathers (the one-column reverse level 0.5 us faster than with 256 threads).
constexpr int kLevelBlock = 64;

// Two consecutive simulation words as one 16-byte vector (a single
// dwordx4 access per lane).
typedef uint64_t w2 __attribute__((ext_vector_type(2)));
// A signal probability and its complement (p, q = 1 - p), one 8-byte access.
typedef float f2 __attribute__((ext_vector_type(2)));

enum : int { INV = 0, BUF, AND2, OR2, NAND2, NOR2, XOR2, AOI21, MUX2 };

__device__ __forceinline__ int arity_of(int op) { return op < AND2 ? 1 : (op < AOI21 ? 2 : 3); }

__device__ __forceinline__ float clamp01(float v) { return fminf(fmaxf(v, 0.0f), 1.0f); }

// A net's probability is stored as one float: the smaller of p and q =
// 1 - p, negated when it is q (sign bit set: p is the larger, so p = 1 is
// -0.0).  The larger is always 1 minus the smaller (settle() makes it so for
// gate outputs, and for a startpoint p >= 1/2 the difference 1 - p is exact),
// so the (p, q) pair the rules work on comes back bit for bit from 4 bytes.
__device__ __forceinline__ f2 sp_load(float s) {
  const float m = fabsf(s);
  return (__float_as_uint(s) >> 31) ? f2{1.0f - m, m} : f2{m, 1.0f - m};
}

// A startpoint probability in the stored form.
__device__ __forceinline__ float sp_pack(float p) { return p <= 0.5f ? p : -(1.0f - p); }

// Clip to [0, 1] (Alg. 2) and re-tie the pair: the smaller of p and q comes
// from its own formula (full relative accuracy), the larger is 1 minus it.
// Without this, rounding drift of p + q - 1 adds up along reconvergent
// paths and grows with the number of paths.  Returns the stored form.
__device__ __forceinline__ float settle(f2 v) {
  const float p = clamp01(v.x), q = clamp01(v.y);
  return p <= q ? p : -q;
}

// Probability that the cell output is 1, and its complement, for
// independent inputs (Sec. II-B; Alg. 2 gives AND = a0 a1 and NAND =
// 1 - a0 a1).  Inputs and outputs are (p, q = 1 - p) pairs and every
// formula is a sum of products of p's and q's, so neither output loses
// relative accuracy when the probability is close to 0 or 1.
__device__ __forceinline__ f2 sp_rule(int op, f2 a, f2 b, f2 c) {
  const float pa = a.x, qa = a.y, pb = b.x, qb = b.y, pc = c.x, qc = c.y;
  f2 r;
  switch (op) {
    case INV: r = f2{qa, pa}; break;
    case BUF: r = a; break;
    case AND2: r = f2{pa * pb, fmaf(pa, qb, qa)}; break;
    case OR2: r = f2{fmaf(qa, pb, pa), qa * qb}; break;
    case NAND2: r = f2{fmaf(pa, qb, qa), pa * pb}; break;
    case NOR2: r = f2{qa * qb, fmaf(qa, pb, pa)}; break;
    case XOR2: r = f2{fmaf(pa, qb, qa * pb), fmaf(pa, pb, qa * qb)}; break;
    case AOI21: r = f2{fmaf(pa, qb, qa) * qc, fmaf(pa * pb, qc, pc)}; break;  // !((A1&A2)|B)
    default: r = f2{fmaf(qc, pa, pc * pb), fmaf(qc, qa, pc * qb)}; break;     // MUX2 S?I1:I0
  }
  return r;
}

// Partial derivatives of the output probability with respect to each input
// probability (Sec. III-E: dAND/da = b, dOR/da = 1 - b, dXOR/da = 1 - 2b,
// dNOT = -1; the compound cells by the product rule).
__device__ __forceinline__ void sp_partials(int op, f2 a, f2 b, f2 c, float &d0, float &d1,
                                            float &d2) {
  const float pa = a.x, qa = a.y, pb = b.x, qb = b.y, pc = c.x, qc = c.y;
  d1 = 0.0f;
  d2 = 0.0f;
  switch (op) {
    case INV: d0 = -1.0f; break;
    case BUF: d0 = 1.0f; break;
    case AND2: d0 = pb; d1 = pa; break;
    case OR2: d0 = qb; d1 = qa; break;
    case NAND2: d0 = -pb; d1 = -pa; break;
    case NOR2: d0 = -qb; d1 = -qa; break;
    case XOR2: d0 = qb - pb; d1 = qa - pa; break;
    case AOI21: d0 = -pb * qc; d1 = -pa * qc; d2 = -fmaf(pa, qb, qa); break;
    default: d0 = qc; d1 = pc; d2 = pb - pa; break;  // MUX2
  }
}

// ---------------------------------------------------------------- library cells
// A library cell is post-order stack code (Alg. 1), interpreted operation by
// operation: each binary operation applies its independent-input rule to its
// two operands (Sec. III-E: AND ab, OR a + b - ab, XOR a + b - 2ab, NOT 1 - a),
// in the same cancellation-free (p, q) form as the fixed cells.
// Each cell's code sits padded to kCellMaxCode words (64 bytes) at offset
// c * kCellMaxCode, so a lane loads its whole program with four 16-byte
// loads that depend only on the opcode, in flight with its input gathers,
// and interprets it from registers.
struct LaneCode {
  uint32_t w[kCellMaxCode / 2];  // two instructions per dword
  int len, nin;
};

__device__ __forceinline__ LaneCode lane_code(const GraphView &g, int op) {
  LaneCode lc;
  const int c = op - kCellBase;
  lc.len = g.cell[3 * c + 1];
  lc.nin = g.cell[3 * c + 2];
  const uint4 *src = reinterpret_cast<const uint4 *>(g.code + (int64_t)c * kCellMaxCode);
#pragma unroll
  for (int k = 0; k < kCellMaxCode / 8; ++k) {
    const uint4 v = src[k];
    lc.w[4 * k] = v.x;
    lc.w[4 * k + 1] = v.y;
    lc.w[4 * k + 2] = v.z;
    lc.w[4 * k + 3] = v.w;
  }
  return lc;
}

__device__ __forceinline__ int code_at(const LaneCode &lc, int i) {
  return (int)((lc.w[i >> 1] >> ((i & 1) * 16)) & 0xffffu);
}

__device__ __forceinline__ f2 pair_op(int op, f2 a, f2 b) {
  if (op == kCellAnd) return f2{a.x * b.x, fmaf(a.x, b.y, a.y)};
  if (op == kCellOr) return f2{fmaf(a.y, b.x, a.x), a.y * b.y};
  return f2{fmaf(a.x, b.y, a.y * b.x), fmaf(a.x, b.x, a.y * b.y)};  // XOR
}

__device__ f2 cell_sp(const LaneCode &lc, const f2 *x) {
  f2 st[kCellMaxStack];
  int top = 0;
  for (int i = 0; i < lc.len; ++i) {
    const int w = code_at(lc, i), op = w & 0xff;
    if (op == kCellIn) {
      st[top++] = x[w >> 8];
    } else if (op == kCellZero) {
      st[top++] = f2{0.0f, 1.0f};
    } else if (op == kCellOne) {
      st[top++] = f2{1.0f, 0.0f};
    } else if (op == kCellNot) {
      st[top - 1] = f2{st[top - 1].y, st[top - 1].x};
    } else {
      const f2 b = st[--top];
      const f2 a = st[--top];
      st[top++] = pair_op(op, a, b);
    }
  }
  return st[0];
}

// Partial derivatives of a cell's probability with respect to its inputs
// (Sec. III-E, Alg. 3), by reverse mode over the code read as a tape.  The
// forward pass gives every instruction its value and records, for each
// operation, which instructions produced its operands (the stack holds
// instruction indices).  Every value feeds exactly one later instruction
// (the code is a tree), so the backward pass visits the instructions from
// the last to the first and finds each adjoint set, once, by its consumer:
// an operation sets its operands' adjoints to its own times the local
// derivative (AND: the other operand; OR: its complement; XOR: q - p of the
// other operand; NOT: -1), and an input instruction adds its adjoint to the
// input's partial.
__device__ void cell_partials(const LaneCode &lc, const f2 *x, float *d) {
  f2 val[kCellMaxCode];
  float adj[kCellMaxCode];
  uint8_t lhs[kCellMaxCode], rhs[kCellMaxCode];
  uint8_t st[kCellMaxStack];
  int top = 0;
  for (int i = 0; i < lc.len; ++i) {
    const int w = code_at(lc, i), op = w & 0xff;
    if (op == kCellIn) {
      val[i] = x[w >> 8];
    } else if (op == kCellZero) {
      val[i] = f2{0.0f, 1.0f};
    } else if (op == kCellOne) {
      val[i] = f2{1.0f, 0.0f};
    } else if (op == kCellNot) {
      lhs[i] = st[--top];
      val[i] = f2{val[lhs[i]].y, val[lhs[i]].x};
    } else {
      rhs[i] = st[--top];
      lhs[i] = st[--top];
      val[i] = pair_op(op, val[lhs[i]], val[rhs[i]]);
    }
    st[top++] = (uint8_t)i;
  }
  for (int k = 0; k < lc.nin; ++k) d[k] = 0.0f;
  adj[lc.len - 1] = 1.0f;
  for (int i = lc.len - 1; i >= 0; --i) {
    const int w = code_at(lc, i), op = w & 0xff;
    const float a = adj[i];
    if (op == kCellIn) {
      d[w >> 8] += a;
    } else if (op == kCellNot) {
      adj[lhs[i]] = -a;
    } else if (op == kCellAnd || op == kCellOr || op == kCellXor) {
      const f2 u = val[lhs[i]], v = val[rhs[i]];
      const float du = op == kCellAnd ? v.x : (op == kCellOr ? v.y : v.y - v.x);
      const float dv = op == kCellAnd ? u.x : (op == kCellOr ? u.y : u.y - u.x);
      adj[lhs[i]] = a * du;
      adj[rhs[i]] = a * dv;
    }
  }
}

// Boolean function of a cell on 64 lanes (Sec. III-C).
template <int OP>
__device__ __forceinline__ uint64_t cell_bits(uint64_t a, uint64_t b, uint64_t c) {
  if constexpr (OP == INV) return ~a;
  else if constexpr (OP == BUF) return a;
  else if constexpr (OP == AND2) return a & b;
  else if constexpr (OP == OR2) return a | b;
  else if constexpr (OP == NAND2) return ~(a & b);
  else if constexpr (OP == NOR2) return ~(a | b);
  else if constexpr (OP == XOR2) return a ^ b;
  else if constexpr (OP == AOI21) return ~((a & b) | c);
  else return (a & ~c) | (b & c);  // MUX2
}

template <int OP>
constexpr int kArity = OP < AND2 ? 1 : (OP < AOI21 ? 2 : 3);

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ int64_t gidx() {
  return (int64_t)blockIdx.x * kBlock + threadIdx.x;
}

// Launches stay below 2^32 threads in total.
constexpr int64_t kMaxBlocks = (1ll << 32) / kBlock - 1;
inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline unsigned level_blocks(int64_t n) { return (unsigned)((n + kLevelBlock - 1) / kLevelBlock); }
// SP level launches of many lanes take 256-thread workgroups: a dependent
// launch of 5,000 one-wave workgroups costs about 0.3 us more than one of
// 1,250 four-wave workgroups, while a few waves still spread over as many
// CUs as one-wave workgroups give them.
constexpr int kWideBlock = 256;
constexpr int64_t kWideLanes = 65536;
inline unsigned level_block(int64_t lanes) { return lanes >= kWideLanes ? kWideBlock : kLevelBlock; }
inline unsigned level_grid(int64_t lanes) {
  const int64_t bs = level_block(lanes);
  return (unsigned)((lanes + bs - 1) / bs);
}
inline bool too_big(int64_t items) { return (items + kBlock - 1) / kBlock > kMaxBlocks; }

// ---------------------------------------------------------------- plumbing
__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  int64_t i = gidx();
  if (i < n) p[i] = v;
}
__global__ __launch_bounds__(kBlock) void k_fill_f32(float *p, int64_t n, float v) {
  int64_t i = gidx();
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_load_pi(const float *__restrict__ p,
                                                     float *__restrict__ sp, int32_t n_pi,
                                                     int32_t B) {
  int64_t idx = gidx();
  if (idx >= (int64_t)n_pi * B) return;
  int32_t i = (int32_t)(idx / B), b = (int32_t)(idx - (int64_t)i * B);
  sp[idx] = sp_pack(p[(int64_t)b * n_pi + i]);
}

__global__ __launch_bounds__(kBlock) void k_check_range(const float *__restrict__ v, int64_t n,
                                                         float lo, float hi, int32_t *bad) {
  int64_t i = gidx();
  if (i >= n) return;
  float x = v[i];
  if (!(x >= lo && x <= hi)) *bad = 1;  // NaN fails both comparisons
}

__global__ __launch_bounds__(kBlock) void k_gather_nets(const float *__restrict__ src,
                                                         const int32_t *__restrict__ int2ext,
                                                         float *__restrict__ dst, int32_t n) {
  int64_t i = gidx();
  if (i < n) dst[i] = src[int2ext[i]];
}

__global__ __launch_bounds__(kBlock) void k_import_cols(const float *__restrict__ src,
                                                         const int32_t *__restrict__ int2ext,
                                                         float *__restrict__ dst, int32_t n_nets,
                                                         int32_t B) {
  int64_t idx = gidx();
  if (idx >= (int64_t)n_nets * B) return;
  int32_t n = (int32_t)(idx / B), b = (int32_t)(idx - (int64_t)n * B);
  dst[idx] = src[(int64_t)b * n_nets + int2ext[n]];
}

__global__ __launch_bounds__(kBlock) void k_import_sizes(const float *__restrict__ src,
                                                          const int32_t *__restrict__ int2ext,
                                                          float *__restrict__ dst, int32_t n_pi,
                                                          int32_t G, int32_t S) {
  int64_t idx = gidx();
  if (idx >= (int64_t)G * S) return;
  int32_t s = (int32_t)(idx / G), g = (int32_t)(idx - (int64_t)s * G);
  dst[idx] = src[(int64_t)s * G + (int2ext[n_pi + g] - n_pi)];
}

// ---------------------------------------------------------------- SP level
// One lane per (gate, column) of level [g0, g0 + n): gather the fan-in
// probabilities, apply the cell rule, clip to [0, 1] (Alg. 2).
// CELLS: the range holds library cells only (their own kernel instances, so
// the fixed-cell kernels keep their register budget).
// Row j of a per-pin table ([pins][G]), or row 0 where the design's widest
// gate has fewer pins: a choice of address that is uniform across the
// launch, so a gather through it waits on no other load.  (In the fan-in
// table, pins a gate does not use alias its pin 0; callers ignore them.)
__device__ __forceinline__ const int32_t *pin_row(const int32_t *tab, const GraphView &g, int j) {
  return tab + (g.pins > j ? (int64_t)j * g.G : 0);
}

// Takes loaded values at this point: every load before it is then issued
// ahead of the first wait, and none can be moved into the branch of the one
// opcode that reads it or behind a use of another (each would add a
// dependent round trip).
template <typename T>
__device__ __forceinline__ void value_taken(T v) { asm volatile("" ::"v"(v)); }
template <typename... V>
__device__ __forceinline__ void gathers_done(V... v) {
  (value_taken(v), ...);
}

template <bool CELLS>
__device__ __forceinline__ void sp_item(const GraphView &g, const SpLevel &lv, uint32_t idx) {
  const int32_t B = lv.B;
  const uint32_t gl32 = idx / (uint32_t)B;
  const int32_t gl = (int32_t)gl32;
  const int32_t b = (int32_t)(idx - gl32 * (uint32_t)B);
  const int32_t gi = lv.g0 + gl;
  const int op = g.op[gi];
  float *sp = lv.sp;
  if constexpr (CELLS) {
    // every pin row (unused pins alias pin 0), so the gathers need no count;
    // the indices arrive with the opcode, the probabilities with the cell's
    // code, and no gather waits on another
    int32_t pin[kCellMaxIn];
#pragma unroll
    for (int k = 0; k < kCellMaxIn; ++k) pin[k] = k < g.pins ? g.in[k * g.G + gi] : 0;
    value_taken(op);
#pragma unroll
    for (int k = 0; k < kCellMaxIn; ++k) value_taken(pin[k]);
    float r[kCellMaxIn];
#pragma unroll
    for (int k = 0; k < kCellMaxIn; ++k) r[k] = k < g.pins ? sp[(int64_t)pin[k] * B + b] : 0.0f;
    const LaneCode lc = lane_code(g, op);
    f2 x[kCellMaxIn];
#pragma unroll
    for (int k = 0; k < kCellMaxIn; ++k) x[k] = k < g.pins ? sp_load(r[k]) : f2{0.0f, 1.0f};
    sp[(int64_t)(g.n_pi + gi) * B + b] = settle(cell_sp(lc, x));
    return;
  }
  // the opcode and every pin's index arrive in one load round; the second
  // round gathers the probabilities of the pins the gate has
  const int32_t i0 = g.in[gi];
  const int32_t i1 = pin_row(g.in, g, 1)[gi];
  const int32_t i2 = pin_row(g.in, g, 2)[gi];
  gathers_done(op, i0, i1, i2);
  const int k = arity_of(op);
  const float sa = sp[(int64_t)i0 * B + b];
  float sb = 0.0f, sc = 0.0f;
  if (k > 1) sb = sp[(int64_t)i1 * B + b];
  if (k > 2) sc = sp[(int64_t)i2 * B + b];
  gathers_done(sa, sb, sc);
  const f2 z = f2{0.0f, 1.0f};
  sp[(int64_t)(g.n_pi + gi) * B + b] =
      settle(sp_rule(op, sp_load(sa), k > 1 ? sp_load(sb) : z, k > 2 ? sp_load(sc) : z));
}

__global__ __launch_bounds__(kWideBlock) void k_sp_level(GraphView g, SpLevel lv) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (uint32_t)lv.n * (uint32_t)lv.B) sp_item<false>(g, lv, idx);
}

__global__ __launch_bounds__(kBlock) void k_sp_cells(GraphView g, SpLevel lv) {
  const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx < (uint32_t)lv.n * (uint32_t)lv.B) sp_item<true>(g, lv, idx);
}

// The same for an even column count, two columns per lane: one 8-byte
// access moves two stored probabilities, and half as many waves cover the
// level.

__global__ __launch_bounds__(kWideBlock) void k_sp_level_x2(GraphView g, SpLevel lv) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t half = (uint32_t)lv.B / 2;
  if (idx >= (uint32_t)lv.n * half) return;
  const uint32_t gl = idx / half;
  const int32_t b = 2 * (int32_t)(idx - gl * half);
  const int32_t gi = lv.g0 + (int32_t)gl;
  const int op = g.op[gi];
  const int k = arity_of(op);
  const f2 *sp2 = reinterpret_cast<const f2 *>(lv.sp);
  const int64_t B2 = lv.B / 2;
  const f2 z = f2{0.0f, 1.0f};
  const int32_t i0 = g.in[gi];
  const int32_t i1 = pin_row(g.in, g, 1)[gi];
  const int32_t i2 = pin_row(g.in, g, 2)[gi];
  gathers_done(op, i0, i1, i2);
  const f2 a = sp2[(int64_t)i0 * B2 + b / 2];
  f2 bl = f2{0.0f, 0.0f}, cl = f2{0.0f, 0.0f};
  if (k > 1) bl = sp2[(int64_t)i1 * B2 + b / 2];
  if (k > 2) cl = sp2[(int64_t)i2 * B2 + b / 2];
  gathers_done(a.x, a.y, bl.x, bl.y, cl.x, cl.y);
  const float r0 = settle(sp_rule(op, sp_load(a.x), k > 1 ? sp_load(bl.x) : z,
                                  k > 2 ? sp_load(cl.x) : z));
  const float r1 = settle(sp_rule(op, sp_load(a.y), k > 1 ? sp_load(bl.y) : z,
                                  k > 2 ? sp_load(cl.y) : z));
  reinterpret_cast<f2 *>(lv.sp)[(int64_t)(g.n_pi + gi) * B2 + b / 2] = f2{r0, r1};
}

// ---------------------------------------------------------------- simulation
// Count ones / toggles of one word pair computed by this lane.  `prev` is the
// word before the pair's first word.
__device__ __forceinline__ void count_pair(const ChunkView &c, int32_t p, w2 y, uint64_t prev,
                                           uint32_t &ones, uint32_t &togs) {
  const int32_t u0 = 2 * p, u1 = u0 + 1;
  if (u0 >= c.u_lo && u0 < c.u_hi) ones += __popcll(y.x);
  if (u1 >= c.u_lo && u1 < c.u_hi) ones += __popcll(y.y);
  if (u0 >= c.u_tog_lo && u0 < c.u_hi) togs += __popcll(y.x ^ prev);
  if (u1 >= c.u_tog_lo && u1 < c.u_hi) togs += __popcll(y.y ^ y.x);
}

// One gate's row over pairs [p_begin, p_begin + 64*ITERS): loads of all
// iterations are issued before any store so they overlap in flight.  Rows
// are addressed as 16-byte word pairs so each lane moves one pair per access.
template <int OP, int ITERS>
__device__ __forceinline__ void sim_gate_row(const w2 *__restrict__ r0,
                                             const w2 *__restrict__ r1,
                                             const w2 *__restrict__ r2,
                                             w2 *__restrict__ out, bool keep, int32_t p_begin,
                                             const ChunkView &c, int lane, uint32_t &ones,
                                             uint32_t &togs) {
  constexpr int K = kArity<OP>;
  uint64_t carry = 0;
  if (p_begin > 0) {  // word just before this run, recomputed from its inputs
    const int32_t q = p_begin - 1;
    carry = cell_bits<OP>(r0[q].y, K > 1 ? r1[q].y : 0, K > 2 ? r2[q].y : 0);
  }
  w2 x0[ITERS], x1[ITERS], x2[ITERS];
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int32_t p = p_begin + it * 64 + lane;
    const bool ok = p < c.pairs;
    const w2 z = w2{0, 0};
    x0[it] = ok ? r0[p] : z;
    x1[it] = (ok && K > 1) ? r1[p] : z;
    x2[it] = (ok && K > 2) ? r2[p] : z;
  }
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int32_t p = p_begin + it * 64 + lane;
    w2 y;
    y.x = cell_bits<OP>(x0[it].x, x1[it].x, x2[it].x);
    y.y = cell_bits<OP>(x0[it].y, x1[it].y, x2[it].y);
    uint64_t prev = __shfl_up(y.y, 1u);
    if (lane == 0) prev = carry;
    carry = __shfl(y.y, 63);
    if (p < c.pairs) {
      // streaming store: a row's readers run in later launches, mostly on
      // other XCDs, so the words gain nothing from this XCD's L2 (measured
      // 3% faster per level than a plain store on MI355X); a row nobody
      // reads is not stored at all
      if (keep) __builtin_nontemporal_store(y, out + p);
      count_pair(c, p, y, prev, ones, togs);
    }
  }
}

// A library cell's Boolean function from its truth table (bit m = output for
// the input pattern m, input k = bit k of m), by Shannon expansion depth
// first: f = x_{N-1} ? f(x_{N-1} = 1) : f(x_{N-1} = 0), one bit select per
// node, N + 1 words live.  The simulation needs exact bits only, which the
// table gives; probabilities and partials follow the code (op by op).
template <int N>
__device__ __forceinline__ uint64_t tt_eval(const uint64_t *x, uint64_t tt, int base) {
  if constexpr (N == 1) {
    const uint64_t m0 = 0ull - ((tt >> base) & 1ull), m1 = 0ull - ((tt >> (base + 1)) & 1ull);
    return (x[0] & m1) | (~x[0] & m0);
  } else {
    const uint64_t lo = tt_eval<N - 1>(x, tt, base);
    const uint64_t hi = tt_eval<N - 1>(x, tt, base + (1 << (N - 1)));
    return (x[N - 1] & hi) | (~x[N - 1] & lo);
  }
}

// A library cell's row with N inputs: sim_gate_row with the table in place
// of the fixed rule.
template <int N, int ITERS, int NMAX>
__device__ __forceinline__ void sim_tt_row(const int32_t (&ix)[NMAX], uint64_t tt,
                                           const w2 *__restrict__ W, int64_t pp,
                                           w2 *__restrict__ out, bool keep, int32_t p_begin,
                                           const ChunkView &c, int lane, uint32_t &ones,
                                           uint32_t &togs) {
  const w2 *r[N];
#pragma unroll
  for (int k = 0; k < N; ++k) r[k] = W + (int64_t)ix[k] * pp;
  uint64_t carry = 0;
  if (p_begin > 0) {  // word just before this run, recomputed from its inputs
    uint64_t x[N];
#pragma unroll
    for (int k = 0; k < N; ++k) x[k] = r[k][p_begin - 1].y;
    carry = tt_eval<N>(x, tt, 0);
  }
  w2 v[N][ITERS];
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int32_t p = p_begin + it * 64 + lane;
    const bool ok = p < c.pairs;
#pragma unroll
    for (int k = 0; k < N; ++k) v[k][it] = ok ? r[k][p] : w2{0, 0};
  }
#pragma unroll
  for (int it = 0; it < ITERS; ++it) {
    const int32_t p = p_begin + it * 64 + lane;
    uint64_t xa[N], xb[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      xa[k] = v[k][it].x;
      xb[k] = v[k][it].y;
    }
    const w2 y = w2{tt_eval<N>(xa, tt, 0), tt_eval<N>(xb, tt, 0)};
    uint64_t prev = __shfl_up(y.y, 1u);
    if (lane == 0) prev = carry;
    carry = __shfl(y.y, 63);
    if (p < c.pairs) {
      if (keep) __builtin_nontemporal_store(y, out + p);  // see sim_gate_row
      count_pair(c, p, y, prev, ones, togs);
    }
  }
}

template <int ITERS, int NMAX>
__device__ __forceinline__ void sim_cell_row(const GraphView &g, int op, int32_t gi,
                                             const w2 *__restrict__ W, int64_t pp,
                                             w2 *__restrict__ out, bool keep, int32_t p_begin,
                                             const ChunkView &c, int lane, uint32_t &ones,
                                             uint32_t &togs) {
  // the gate's input count and every pin's input net go out with the
  // opcode (pin rows past the design's widest cell alias pin 0), so the
  // input rows load in the next round; the table rides along with them
  const int nin = __builtin_amdgcn_readfirstlane((int)g.arity[gi]);
  int32_t ix[NMAX];
#pragma unroll
  for (int k = 0; k < NMAX; ++k) ix[k] = __builtin_amdgcn_readfirstlane(pin_row(g.in, g, k)[gi]);
  const int cl = op - kCellBase;
  const uint64_t t = g.tt[cl];
  const uint64_t tt = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(t >> 32)) << 32) |
                      (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)t);
  // NMAX: the most inputs a cell of the launch has (the instance for narrow
  // cells keeps fewer registers, so more of its waves are resident)
  switch (nin) {
    case 1: sim_tt_row<1, ITERS>(ix, tt, W, pp, out, keep, p_begin, c, lane, ones, togs); break;
    case 2: sim_tt_row<2, ITERS>(ix, tt, W, pp, out, keep, p_begin, c, lane, ones, togs); break;
    case 3: sim_tt_row<3, ITERS>(ix, tt, W, pp, out, keep, p_begin, c, lane, ones, togs); break;
    default:
      if constexpr (NMAX > 3) {
        switch (nin) {
          case 4: sim_tt_row<4, ITERS>(ix, tt, W, pp, out, keep, p_begin, c, lane, ones, togs); break;
          case 5: sim_tt_row<5, ITERS>(ix, tt, W, pp, out, keep, p_begin, c, lane, ones, togs); break;
          default: sim_tt_row<6, ITERS>(ix, tt, W, pp, out, keep, p_begin, c, lane, ones, togs); break;
        }
      }
      break;
  }
}

// CELLS: 0 for fixed cells, else the most inputs a library cell of the
// launch has.
template <int ITERS, int CELLS>
__global__ __launch_bounds__(kSimBlock) void k_sim_level(GraphView g, ChunkView c, CountView cnt,
                                                      int32_t g0, int32_t n, int32_t waves_per_row,
                                                      int32_t sim_blocks, SpLevel sp) {
  if ((int32_t)blockIdx.x >= sim_blocks) {  // fused SP of the same level (and kind)
    const uint32_t idx = (blockIdx.x - (uint32_t)sim_blocks) * kSimBlock + threadIdx.x;
    if (idx < (uint32_t)sp.n * (uint32_t)sp.B) sp_item<(CELLS > 0)>(g, sp, idx);
    return;
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t task = (int64_t)blockIdx.x * kSimWaves + wave;
  // tasks: (column, gate, run of word pairs), column outermost
  const int64_t per_col = (int64_t)n * waves_per_row;
  if (task >= per_col * c.n_cols) return;
  const int32_t lc = (int32_t)(task / per_col);
  const int64_t rest = task - (int64_t)lc * per_col;
  const int32_t gl = (int32_t)(rest / waves_per_row);
  const int32_t seg = (int32_t)(rest - (int64_t)gl * waves_per_row);
  const int32_t gi = g0 + gl;
  const int op = __builtin_amdgcn_readfirstlane((int)g.op[gi]);
  const int64_t pp = c.pitch / 2;  // pairs per row
  uint64_t *Wc = c.W + (int64_t)lc * c.col_stride;
  const w2 *W = reinterpret_cast<const w2 *>(Wc);
  const w2 *r0 = W + (int64_t)__builtin_amdgcn_readfirstlane(g.in[gi]) * pp;
  const w2 *r1 = W + (int64_t)__builtin_amdgcn_readfirstlane(g.in[g.G + gi]) * pp;
  const w2 *r2 = W + (int64_t)__builtin_amdgcn_readfirstlane(g.in[2 * g.G + gi]) * pp;
  w2 *out = reinterpret_cast<w2 *>(Wc) + (int64_t)(g.n_pi + gi) * pp;
  // a net with no readers needs its counts only: its words are not stored
  const int32_t on = g.n_pi + gi;
  const bool keep = __builtin_amdgcn_readfirstlane(g.rev_ptr[on + 1]) >
                    __builtin_amdgcn_readfirstlane(g.rev_ptr[on]);
  const int32_t p_begin = seg * 64 * ITERS;
  uint32_t ones = 0, togs = 0;
  if constexpr (CELLS > 0) {
    sim_cell_row<ITERS, CELLS>(g, op, gi, W, pp, out, keep, p_begin, c, lane, ones, togs);
  } else {
  switch (op) {
    case INV: sim_gate_row<INV, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case BUF: sim_gate_row<BUF, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case AND2: sim_gate_row<AND2, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case OR2: sim_gate_row<OR2, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case NAND2: sim_gate_row<NAND2, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case NOR2: sim_gate_row<NOR2, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case XOR2: sim_gate_row<XOR2, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    case AOI21: sim_gate_row<AOI21, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
    default: sim_gate_row<MUX2, ITERS>(r0, r1, r2, out, keep, p_begin, c, lane, ones, togs); break;
  }
  }
  ones = wave_sum(ones);
  togs = wave_sum(togs);
  if (lane == 0) {
    const int64_t o = (int64_t)(g.n_pi + gi) * cnt.B + cnt.col + lc;
    if (ones) atomicAdd(cnt.ones + o, ones);
    if (togs) atomicAdd(cnt.tog + o, togs);
  }
}

// ---------------------------------------------------------------- stimulus
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of
// (c0,c1,c2,c3) -> (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)),
// key bumped by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1,
                   (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// floor(p * 2^32) of a float32 probability, exact in double.
__device__ __forceinline__ uint64_t prob_threshold(float p) {
  const double v = (double)p * 4294967296.0;
  if (!(v > 0.0)) return 0;
  if (v >= 4294967296.0) return 1ull << 32;
  return (uint64_t)v;
}

// Word t of PI i: i.i.d. Bernoulli(p) lanes, the temporal-independence case
// of the Markov stimulus of Sec. III-C; lane j = 4q + l is 1 iff lane l of
// Philox(t, i, q, 0; seed) is below the threshold.
__device__ __forceinline__ uint64_t stim_word(uint32_t pi, int64_t t, uint64_t thr, uint32_t k0,
                                              uint32_t k1) {
  uint64_t w = 0;
#pragma unroll 4
  for (uint32_t q = 0; q < 16; ++q) {
    const uint4 u = philox4x32_10(make_uint4((uint32_t)t, pi, q, 0u), k0, k1);
    const uint64_t bits = (uint64_t)((uint64_t)u.x < thr) | ((uint64_t)((uint64_t)u.y < thr) << 1) |
                          ((uint64_t)((uint64_t)u.z < thr) << 2) |
                          ((uint64_t)((uint64_t)u.w < thr) << 3);
    w |= bits << (4 * q);
  }
  return w;
}

// ---------------------------------------------------------------- paired SP levels
// Two consecutive fixed-cell levels in one launch: lanes [0, a.n B) run
// level a as k_sp_level does; lanes [a.n B, (a.n + b.n) B) run level b, and
// a pin that level a drives is recomputed from that gate's own inputs (its
// structure in the second load round, its inputs in the third) with the
// arithmetic level a's lane performs, so the value is bit for bit the one
// that lane stores.  One dependent round more than a level launch, one
// launch boundary less: for a few columns, where a level's launch is
// latency-bound, two levels cost about what one did.
__device__ __forceinline__ f2 sp_recomputed(int op, float u0, float u1, float u2) {
  const int k = arity_of(op);
  const f2 z = f2{0.0f, 1.0f};
  return sp_load(settle(sp_rule(op, sp_load(u0), k > 1 ? sp_load(u1) : z, k > 2 ? sp_load(u2) : z)));
}

__device__ __forceinline__ void sp_pair_item(const GraphView &g, const SpLevel &a,
                                             const SpLevel &b, uint32_t idx) {
  const uint32_t na = (uint32_t)a.n * (uint32_t)a.B;
  if (idx < na) {
    sp_item<false>(g, a, idx);
    return;
  }
  const uint32_t t = idx - na;
  const int32_t B = b.B;
  if (t >= (uint32_t)b.n * (uint32_t)B) return;
  const uint32_t gl = t / (uint32_t)B;
  const int32_t col = (int32_t)(t - gl * (uint32_t)B);
  const int32_t gi = b.g0 + (int32_t)gl;
  float *sp = b.sp;
  // first load round: the gate's opcode and pins
  const int op = g.op[gi];
  const int32_t i0 = g.in[gi];
  const int32_t i1 = pin_row(g.in, g, 1)[gi];
  const int32_t i2 = pin_row(g.in, g, 2)[gi];
  gathers_done(op, i0, i1, i2);
  const int k = arity_of(op);
  const int32_t lo = g.n_pi + a.g0, hi = lo + a.n;  // the nets level a drives
  const bool r0 = i0 >= lo && i0 < hi, r1 = k > 1 && i1 >= lo && i1 < hi,
             r2 = k > 2 && i2 >= lo && i2 < hi;
  // second load round: a pin level a drives gives that gate's structure, any other
  // pin its stored probability
  int32_t po[3] = {0, 0, 0}, pj[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  float v[3] = {0.0f, 0.0f, 0.0f};
  const int32_t pin[3] = {i0, i1, i2};
  const bool rec[3] = {r0, r1, r2};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j >= k) continue;
    if (rec[j]) {
      const int32_t pg = pin[j] - g.n_pi;
      po[j] = g.op[pg];
      pj[j][0] = g.in[pg];
      pj[j][1] = pin_row(g.in, g, 1)[pg];
      pj[j][2] = pin_row(g.in, g, 2)[pg];
    } else {
      v[j] = sp[(int64_t)pin[j] * B + col];
    }
  }
  gathers_done(po[0], po[1], po[2], pj[0][0], pj[0][1], pj[0][2], pj[1][0], pj[1][1], pj[1][2],
               pj[2][0], pj[2][1], pj[2][2], v[0], v[1], v[2]);
  // third load round: the recomputed gates' inputs (levels below a: stored)
  float u[3][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j >= k || !rec[j]) continue;
    const int kp = arity_of(po[j]);
    u[j][0] = sp[(int64_t)pj[j][0] * B + col];
    if (kp > 1) u[j][1] = sp[(int64_t)pj[j][1] * B + col];
    if (kp > 2) u[j][2] = sp[(int64_t)pj[j][2] * B + col];
  }
  f2 x[3];
  const f2 z = f2{0.0f, 1.0f};
#pragma unroll
  for (int j = 0; j < 3; ++j)
    x[j] = j >= k ? z : (rec[j] ? sp_recomputed(po[j], u[j][0], u[j][1], u[j][2]) : sp_load(v[j]));
  sp[(int64_t)(g.n_pi + gi) * B + col] = settle(sp_rule(op, x[0], x[1], x[2]));
}

__global__ __launch_bounds__(kWideBlock) void k_sp_pair(GraphView g, SpLevel a, SpLevel b) {
  sp_pair_item(g, a, b, blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------- Markov stimulus
// Startpoints with a target transition rate tau (Sec. III-C): each lane is a
// two-state chain with stationary law Bernoulli(p); a lane at 1 stays with
// probability 1 - tau / (2p), a lane at 0 rises with probability
// tau / (2 (1 - p)), each cycle's draw being the same Philox uniform as the
// independent stimulus (counter (t, stream, lane / 4)); cycle 0 is the
// stationary draw.  Probabilities in double, clamped to [0, 1].
__device__ __forceinline__ uint64_t threshold_d(double x) {
  const double v = x * 4294967296.0;
  if (!(v > 0.0)) return 0;
  if (v >= 4294967296.0) return 1ull << 32;
  return (uint64_t)v;
}

__device__ __forceinline__ void markov_probs(float p, float tau, double &rise, double &stay) {
  const double pd = (double)p, td = (double)tau;
  if (pd <= 0.0) {
    rise = 0.0;
    stay = 0.0;
  } else if (pd >= 1.0) {
    rise = 1.0;
    stay = 1.0;
  } else {
    rise = td / (2.0 * (1.0 - pd));
    stay = 1.0 - td / (2.0 * pd);
  }
  if (rise > 1.0) rise = 1.0;
  if (stay < 0.0) stay = 0.0;
}

// A lane's next bit as a map of its previous bit: x -> (x & s) | (~x & u),
// 64 lanes at once.  Maps compose associatively.
struct BitMap {
  uint64_t s, u;
};
__device__ __forceinline__ BitMap bitmap_then(BitMap first, BitMap then) {
  return BitMap{(first.s & then.s) | (~first.s & then.u), (first.u & then.s) | (~first.u & then.u)};
}
__device__ __forceinline__ uint64_t bitmap_apply(BitMap m, uint64_t x) {
  return (x & m.s) | (~x & m.u);
}

constexpr int kMarkovK = 4;  // consecutive words per lane and tile

// Words [B][n_pi][T] of every (column, startpoint), one wave each.  A tile of
// 64 K words: each lane draws the maps of its K words and composes them, an
// inclusive scan over the lanes composes the prefixes, and each lane applies
// its exclusive prefix to the word carried in from the previous tile, then
// its own maps in order.
__global__ __launch_bounds__(kBlock) void k_markov_words(const float *__restrict__ sp,
                                                         const float *__restrict__ tau,
                                                         const int32_t *__restrict__ stream,
                                                         int32_t n_pi, int32_t B, int64_t T,
                                                         uint32_t k0, uint32_t k1,
                                                         uint64_t *__restrict__ out) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * kWavesPerBlock + wave;  // b * n_pi + i
  if (row >= (int64_t)B * n_pi) return;
  const int32_t b = (int32_t)(row / n_pi), i = (int32_t)(row - (int64_t)b * n_pi);
  const float p = sp_load(sp[(int64_t)i * B + b]).x;
  double rise, stay;
  markov_probs(p, tau[(int64_t)b * n_pi + i], rise, stay);
  const uint64_t thr_p = prob_threshold(p), thr_rise = threshold_d(rise),
                 thr_stay = threshold_d(stay);
  const uint32_t si = stream ? (uint32_t)stream[i] : (uint32_t)i;
  uint64_t *orow = out + row * T;
  const BitMap id = BitMap{~0ull, 0ull};
  uint64_t carry = 0;  // cycle 0's map is constant, so the first carry is moot
  for (int64_t t0 = 0; t0 < T; t0 += 64 * kMarkovK) {
    BitMap m[kMarkovK];
    BitMap f = id;
#pragma unroll
    for (int k = 0; k < kMarkovK; ++k) {
      const int64_t t = t0 + (int64_t)lane * kMarkovK + k;
      m[k] = id;
      if (t < T) {
        const uint64_t ts = t == 0 ? thr_p : thr_stay, tr = t == 0 ? thr_p : thr_rise;
        uint64_t ms = 0, mu = 0;
        for (uint32_t q = 0; q < 16; ++q) {
          const uint4 u = philox4x32_10(make_uint4((uint32_t)t, si, q, 0u), k0, k1);
          const uint64_t s4 = (uint64_t)((uint64_t)u.x < ts) | ((uint64_t)((uint64_t)u.y < ts) << 1) |
                              ((uint64_t)((uint64_t)u.z < ts) << 2) |
                              ((uint64_t)((uint64_t)u.w < ts) << 3);
          const uint64_t u4 = (uint64_t)((uint64_t)u.x < tr) | ((uint64_t)((uint64_t)u.y < tr) << 1) |
                              ((uint64_t)((uint64_t)u.z < tr) << 2) |
                              ((uint64_t)((uint64_t)u.w < tr) << 3);
          ms |= s4 << (4 * q);
          mu |= u4 << (4 * q);
        }
        m[k] = BitMap{ms, mu};
      }
      f = bitmap_then(f, m[k]);
    }
    for (int d = 1; d < 64; d <<= 1) {  // inclusive scan: earlier lanes' maps first
      const BitMap g = BitMap{__shfl_up(f.s, (unsigned)d), __shfl_up(f.u, (unsigned)d)};
      if (lane >= d) f = bitmap_then(g, f);
    }
    BitMap e = BitMap{__shfl_up(f.s, 1u), __shfl_up(f.u, 1u)};
    if (lane == 0) e = id;
    uint64_t x = bitmap_apply(e, carry);
#pragma unroll
    for (int k = 0; k < kMarkovK; ++k) {
      const int64_t t = t0 + (int64_t)lane * kMarkovK + k;
      x = bitmap_apply(m[k], x);
      if (t < T) orow[t] = x;
    }
    carry = __shfl(x, 63);
  }
}

template <int ITERS>
__global__ __launch_bounds__(kBlock) void k_stimulus(int32_t n_pi, ChunkView c, CountView cnt,
                                                     const float *__restrict__ p_rows,
                                                     const uint64_t *__restrict__ stim, int64_t T,
                                                     const int32_t *__restrict__ stream,
                                                     uint32_t k0, uint32_t k1,
                                                     int32_t waves_per_row) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t task = (int64_t)blockIdx.x * kWavesPerBlock + wave;
  // tasks: (column, PI, run of word pairs), column outermost
  const int64_t per_col = (int64_t)n_pi * waves_per_row;
  if (task >= per_col * c.n_cols) return;
  const int32_t lc = (int32_t)(task / per_col);
  const int64_t rest = task - (int64_t)lc * per_col;
  const int32_t i = (int32_t)(rest / waves_per_row);
  const int32_t seg = (int32_t)(rest - (int64_t)i * waves_per_row);
  const int32_t col = cnt.col + lc;
  const uint64_t thr = prob_threshold(sp_load(p_rows[(int64_t)i * cnt.B + col]).x);
  const uint64_t *srow = stim ? stim + ((int64_t)lc * n_pi + i) * T : nullptr;
  const uint32_t si = stream ? (uint32_t)stream[i] : (uint32_t)i;  // shared stream
  auto word = [&](int64_t u) -> uint64_t {
    const int64_t t = c.t_first + u;
    if (t < 0 || t >= T) return 0;
    return srow ? srow[t] : stim_word(si, t, thr, k0, k1);
  };
  uint64_t *out = c.W + (int64_t)lc * c.col_stride + (int64_t)i * c.pitch;
  const int32_t p_begin = seg * 64 * ITERS;
  uint64_t carry = p_begin > 0 ? word(2 * (int64_t)p_begin - 1) : 0;
  uint32_t ones = 0, togs = 0;
  for (int it = 0; it < ITERS; ++it) {
    const int32_t p = p_begin + it * 64 + lane;
    w2 y = w2{0, 0};
    if (p < c.pairs) {
      y.x = word(2 * (int64_t)p);
      y.y = word(2 * (int64_t)p + 1);
    }
    uint64_t prev = __shfl_up(y.y, 1u);
    if (lane == 0) prev = carry;
    carry = __shfl(y.y, 63);
    if (p < c.pairs) {
      reinterpret_cast<w2 *>(out)[p] = y;
      count_pair(c, p, y, prev, ones, togs);
    }
  }
  ones = wave_sum(ones);
  togs = wave_sum(togs);
  if (lane == 0) {
    const int64_t o = (int64_t)i * cnt.B + col;
    if (ones) atomicAdd(cnt.ones + o, ones);
    if (togs) atomicAdd(cnt.tog + o, togs);
  }
}

// ---------------------------------------------------------------- beta and terms
// The hybrid beta of a net whose TR_model is tm and whose simulation counted
// tog toggles: clip(TR_acc / TR_model) with TR_acc = toggles / (64 (T - 1))
// (Eq. 4-5; 0/0 -> 1, x/0 -> beta_max).
__device__ __forceinline__ float hybrid_beta(const PowerArgs &a, uint32_t tog, float tm) {
  const float ta = (float)((double)tog / (64.0 * (double)(a.T - 1)));
  const float beta = tm == 0.0f ? (ta == 0.0f ? 1.0f : a.beta_max) : ta / tm;
  return fminf(fmaxf(beta, a.beta_min), a.beta_max);
}

// beta of net n in column b (idx = n B + b) with TR_model = tm: 1 in modeled
// mode, the frozen value, or the hybrid value.
__device__ __forceinline__ float beta_of(const PowerArgs &a, int64_t idx, int32_t n, float tm) {
  if (a.mode == 1) return hybrid_beta(a, a.tog[idx], tm);
  if (a.mode == 2) return a.beta_shared ? a.beta_frozen[n] : a.beta_frozen[idx];
  return 1.0f;
}

// The hybrid beta of every (net, column), for the contraction with many
// size vectors (the sum over nets with one or paired sizes takes it in the
// same pass, k_power_sp).
__global__ __launch_bounds__(kBlock) void k_beta(PowerArgs a) {
  const int64_t idx = gidx();
  if (idx >= (int64_t)a.n_nets * a.B) return;
  const int32_t n = (int32_t)(idx / a.B);
  const f2 pq = sp_load(a.sp[idx]);
  a.beta[idx] = beta_of(a, idx, n, 2.0f * pq.x * pq.y);
}

__global__ __launch_bounds__(kBlock) void k_export(ExportArgs a) {
  const int64_t idx = gidx();
  if (idx >= (int64_t)a.n_nets * a.B) return;
  const int32_t n = (int32_t)(idx / a.B), b = (int32_t)(idx - (int64_t)n * a.B);
  const int64_t o = (int64_t)b * a.n_nets + a.int2ext[n];
  const f2 pq = sp_load(a.sp[idx]);
  const float tm = 2.0f * pq.x * pq.y;
  if (a.o_sp) a.o_sp[o] = pq.x;
  if (a.o_tr) a.o_tr[o] = tm;
  const float beta = a.beta ? a.beta[idx] : 1.0f;
  if (a.o_beta) a.o_beta[o] = beta;
  if (a.o_tr_hyb) a.o_tr_hyb[o] = beta * tm;
  if (a.o_sp_acc) a.o_sp_acc[o] = (float)((double)a.ones[idx] / (64.0 * (double)a.T));
  if (a.o_tr_acc) a.o_tr_acc[o] = (float)((double)a.tog[idx] / (64.0 * (double)(a.T - 1)));
  if (a.o_ones) a.o_ones[o] = a.ones[idx];
  if (a.o_tog) a.o_tog[o] = a.tog[idx];
}

// ---------------------------------------------------------------- power
// P[b] = sum_n x[n][b] C_n s_b(drv n) with x = kappa beta TR_model, one or
// paired sizes, accumulated in double in an order fixed by the net index
// alone, so a column's power does not depend on the launch it rides in:
// nets in chunks of kPowerChunk; lane j of kPowerLanes sums the chunk's
// nets j, j + kPowerLanes, ... in increasing order; the lane sums are added
// by a fixed pairwise tree (stride 32, 16, ..., 1); the chunks by
// k_power_final.  A block takes one chunk for a tile of tb columns (tb a
// power of two up to 64), the column innermost, so a wave's SP loads are
// whole row segments of tb columns; with tb = 64 a thread keeps the sums
// of several lanes.  Each term is computed where it is summed, and in
// hybrid mode beta is stored on the way.  The column tiles of one chunk go
// to blocks of one XCD (blocks are dealt to the XCDs in turn), which then
// share the chunk's capacitance and size lines in their L2.
constexpr int32_t kPowerChunk = 2048;
constexpr int32_t kPowerLanes = 64;
constexpr int32_t kPowerCols = 64;       // columns per block at most
constexpr int32_t kPowerThreads = 1024;  // threads per block at most
constexpr int32_t kPowerBatch = 8;       // terms per thread whose loads go out together
constexpr int32_t kXcds = 8;

// NQ lanes per thread (1 for tb <= 16 columns, 2 for 32, 4 for 64); MODE
// is the beta mode (0 modeled, 1 hybrid, 2 frozen).  Every operand of a
// round's eight terms is loaded (at a clamped, valid address) before the
// first term is formed; a term past the chunk's end is dropped.
template <int NQ, int MODE>
__global__ __launch_bounds__(kPowerThreads) void k_power_sp(PowerArgs a, int32_t tb,
                                                           int32_t col_tiles) {
  constexpr int U = kPowerBatch / NQ;  // nets of each lane per round
  constexpr int32_t jper = kPowerLanes / NQ;
  __shared__ double lds[kPowerLanes * kPowerCols];
  const int32_t xcd = (int32_t)(blockIdx.x % kXcds), slot = (int32_t)(blockIdx.x / kXcds);
  const int32_t chunk = (slot / col_tiles) * kXcds + xcd;
  const int32_t tile = slot - (slot / col_tiles) * col_tiles;
  if (chunk >= a.n_chunks) return;  // the grid's round-up to whole XCD rounds
  const int32_t c = (int32_t)threadIdx.x % tb, j0 = (int32_t)threadIdx.x / tb;
  const int32_t b = tile * tb + c;
  const int32_t n_lo = chunk * kPowerChunk, n_hi = min(n_lo + kPowerChunk, a.n_nets);
  const bool sized = a.size && a.paired;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (b < a.B) {
    for (int32_t i0 = 0; n_lo + i0 * kPowerLanes < n_hi; i0 += U) {
      // aux: the toggle count (hybrid) or the frozen beta's bits
      float v[kPowerBatch], cv[kPowerBatch], sv[kPowerBatch];
      uint32_t aux[kPowerBatch];
#pragma unroll
      for (int k = 0; k < kPowerBatch; ++k) {
        const int32_t n = min(n_lo + j0 + (k / U) * jper + (i0 + k % U) * kPowerLanes, n_hi - 1);
        const int64_t idx = (int64_t)n * a.B + b;
        v[k] = a.sp[idx];
        cv[k] = a.cap[n];
        if constexpr (MODE == 1) aux[k] = a.tog[idx];
        if constexpr (MODE == 2)
          aux[k] = __float_as_uint(a.beta_frozen[a.beta_shared ? (int64_t)n : idx]);
        sv[k] = (sized && n >= a.n_pi) ? a.size[(int64_t)b * a.G + max(n - a.n_pi, 0)] : 1.0f;
      }
#pragma unroll
      for (int k = 0; k < kPowerBatch; ++k) {
        const int32_t n = n_lo + j0 + (k / U) * jper + (i0 + k % U) * kPowerLanes;
        if (n < n_hi) {
          const f2 pq = sp_load(v[k]);
          const float tm = 2.0f * pq.x * pq.y;
          float beta = 1.0f;
          if constexpr (MODE == 2) beta = __uint_as_float(aux[k]);
          if constexpr (MODE == 1) {
            beta = hybrid_beta(a, aux[k], tm);
            a.beta[(int64_t)n * a.B + b] = beta;
          }
          acc[k / U] += (double)(a.kappa * beta * tm) * (double)(cv[k] * sv[k]);
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) lds[(j0 + q * jper) * tb + c] = acc[q];
  __syncthreads();
  for (int32_t stride = kPowerLanes / 2; stride > 0; stride >>= 1) {
    for (int32_t e = threadIdx.x; e < stride * tb; e += blockDim.x)
      lds[e] += lds[e + stride * tb];
    __syncthreads();
  }
  if (threadIdx.x < tb && b < a.B) a.partial[(int64_t)chunk * a.B + b] = lds[c];
}

__device__ __forceinline__ double block_sum_d(double v, double *lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kWavesPerBlock; ++i) r += lds[i];
  return r;
}

// Many size vectors (S > 0, not paired): P[b][s] = sum_n X[n][b] Y[n][s]
// with X[n][b] = kappa beta TR_model and Y[n][s] = C_n s_s(drv n) is a small dense product
// (B x N) (N x S).  A block owns a 32 x 64 (b, s) tile and one slab of nets;
// X and Y slabs are staged through LDS and each thread accumulates 8 outputs
// in double.  Partials [slab][b][s] are summed over slabs in a fixed order.
constexpr int32_t kTileB = 32, kTileS = 64, kSlabNets = 2048, kStage = 64;

__global__ __launch_bounds__(kBlock) void k_power_tiled(PowerArgs a, int32_t n_slabs) {
  __shared__ float xs[kStage][kTileB];
  __shared__ float ys[kStage][kTileS + 1];
  const int32_t tiles_s = (a.S + kTileS - 1) / kTileS;
  const int32_t tile = blockIdx.x % tiles_s;
  const int32_t rest = blockIdx.x / tiles_s;
  const int32_t tiles_b = (a.B + kTileB - 1) / kTileB;
  const int32_t tb = rest % tiles_b;
  const int32_t slab = rest / tiles_b;
  const int32_t b0 = tb * kTileB, s0 = tile * kTileS;
  const int32_t n_lo = slab * kSlabNets, n_hi = min(n_lo + kSlabNets, a.n_nets);
  const int tid = threadIdx.x;
  const int bl = tid % kTileB;          // this thread's b
  const int sg = tid / kTileB;          // 8 groups of 8 s values
  double acc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = 0.0;
  for (int32_t base = n_lo; base < n_hi; base += kStage) {
    // stage X[n][b0..b0+31] (x = kappa beta TR_model from SP and beta) and
    // Y[n][s0..s0+63] for kStage nets
    for (int e = tid; e < kStage * kTileB; e += kBlock) {
      const int cb = e % kTileB, r = e / kTileB;  // consecutive lanes walk columns
      const int32_t n = base + r, b = b0 + cb;
      float x = 0.0f;
      if (n < n_hi && b < a.B) {
        const int64_t idx = (int64_t)n * a.B + b;
        const f2 pq = sp_load(a.sp[idx]);
        const float tm = 2.0f * pq.x * pq.y;
        const float beta = a.mode == 1 ? a.beta[idx] : beta_of(a, idx, n, tm);
        x = a.kappa * beta * tm;
      }
      xs[r][cb] = x;
    }
    for (int e = tid; e < kStage * kTileS; e += kBlock) {
      const int cs = e / kStage, r = e % kStage;  // consecutive lanes walk nets
      const int32_t n = base + r, s = s0 + cs;
      float y = 0.0f;
      if (n < n_hi && s < a.S) {
        const float sz = n >= a.n_pi ? a.size[(int64_t)s * a.G + (n - a.n_pi)] : 1.0f;
        y = a.cap[n] * sz;
      }
      ys[r][cs] = y;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kStage; ++r) {
      const double x = (double)xs[r][bl];
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = fma(x, (double)ys[r][sg * 8 + j], acc[j]);
    }
    __syncthreads();
  }
  const int32_t b = b0 + bl;
  if (b < a.B)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int32_t s = s0 + sg * 8 + j;
      if (s < a.S) a.partial[((int64_t)slab * a.B + b) * a.S + s] = acc[j];
    }
}

// One block per column: thread t sums chunks t, t + 256, ... in order, then
// a fixed tree over the block.
__global__ __launch_bounds__(kBlock) void k_power_final(PowerArgs a, int32_t n_cols) {
  __shared__ double lds[kWavesPerBlock];
  const int32_t col = blockIdx.x;
  double acc = 0.0;
  for (int32_t k = threadIdx.x; k < a.n_chunks; k += kBlock)
    acc += a.partial[(int64_t)k * n_cols + col];
  const double r = block_sum_d(acc, lds);
  if (threadIdx.x == 0) a.power[col] = (float)r;
}

// ---------------------------------------------------------------- reverse sweep
// Local adjoint seed of net n in reverse column c (SP column b): the
// derivative of the net's own power term, kappa C 2 (1 - 2P) (Eq. 2 and
// Eq. 7), times beta (unless STE), the upstream weight and the driver's size
// factor (per column, paired, or summed over the size vectors).
__device__ __forceinline__ float seed_of(const BwdArgs &a, int32_t n, int32_t c, int32_t b,
                                         f2 pq, float beta, float cap) {
  const float local = a.kappa * cap * 2.0f * (pq.y - pq.x);
  const float base = a.ste ? local : beta * local;
  const bool gate = n >= a.n_pi && a.size;
  const int64_t g = (int64_t)(n - a.n_pi);
  if (a.per_column) {
    const int32_t s = c - b * a.cdiv;
    const float w = a.w ? a.w[c] : 1.0f;
    const float sz = gate ? a.size[(int64_t)s * a.G + g] : 1.0f;
    return base * w * sz;
  }
  if (a.paired) {
    const float w = a.w ? a.w[b] : 1.0f;
    const float sz = gate ? a.size[(int64_t)b * a.G + g] : 1.0f;
    return base * (w * sz);
  }
  const int32_t Sp = a.S > 0 ? a.S : 1;
  float ws = 0.0f;
  for (int32_t s = 0; s < Sp; ++s) {
    const float w = a.w ? a.w[(int64_t)b * Sp + s] : 1.0f;
    const float sz = gate ? a.size[(int64_t)s * a.G + g] : 1.0f;
    ws = fmaf(w, sz, ws);
  }
  return base * ws;
}

// Sum of the contributions the readers of a net left for it.  Readers write
// into the net's own contiguous range [e0, e1) of the contribution buffer
// (fan-out order), so the sum needs no index indirection.  Its order is fixed
// by the graph alone (not by the column, its lane or the batch): the range is
// cut into strands of kStrand consecutive entries, each strand is summed
// serially, and the strand sums are added in strand order.  Two ways reach
// that same sum bit for bit:
//  * lane-serial: a lane walks its own (net, column) strands.  With many
//    columns the wave's lanes are the columns of one net, so every load is a
//    contiguous row;
//  * wave-cooperative, for nets with more than one strand when columns are
//    few: lane j sums strand j of one (net, column) and the strand sums are
//    then added in order through lane shuffles.
// Every lane of the wave must call this (inactive lanes pass e0 == e1 and
// active == false); `serial` must be uniform across the wave.
constexpr int32_t kStrand = 8;
// C at which every pull is lane-serial (nets with more than kHeavyPull entries
// pulled by whole workgroups); below it a wave's lanes share its nets' long
// ranges.  Measured on the 1M-gate design (modeled fwd+bwd): the shared pull
// wins at 1 and 2 columns (0.65 against 0.81 ms, 0.71 against 0.82 ms), the
// lane-serial one from 3 (0.83 against 0.88 ms; 0.83 against 1.06 ms at 4, and
// 3.2x at 16).
constexpr int32_t kSerialColumns = 3;
// The same switch for launches without heavy-net workgroups (library cells,
// merged launches of several designs, the persistent kernel), where a
// lane-serial pull of a long range costs one lane several dependent rounds.
constexpr int32_t kSerialColumnsNoHeavy = 32;

// The entries [e, min(e + kStrand, e1)) of one strand into v (zeros past e1).
__device__ __forceinline__ void strand_load(const float *__restrict__ contrib, int32_t e,
                                            int32_t e1, int32_t C, int32_t c,
                                            float (&v)[kStrand]) {
#pragma unroll
  for (int i = 0; i < kStrand; ++i) v[i] = e + i < e1 ? contrib[(int64_t)(e + i) * C + c] : 0.0f;
}

// A strand's sum in entry order; m = entries left from the strand's start.
__device__ __forceinline__ float strand_fold(const float (&v)[kStrand], int32_t m) {
  float acc = v[0];
#pragma unroll
  for (int i = 1; i < kStrand; ++i)
    if (i < m) acc += v[i];
  return acc;
}

__device__ __forceinline__ float strand_sum(const float *__restrict__ contrib, int32_t e,
                                            int32_t e1, int32_t C, int32_t c) {
  float v[kStrand];
  strand_load(contrib, e, e1, C, c, v);
  return strand_fold(v, e1 - e);
}

// The canonical sum by one lane: a single strand directly; longer ranges four
// strands (32 loads in flight) at a time, their sums folded in strand order.
__device__ __forceinline__ float serial_pull(const float *__restrict__ contrib, int32_t e0,
                                             int32_t e1, int32_t C, int32_t c) {
  if (e1 - e0 <= kStrand) return e1 > e0 ? strand_sum(contrib, e0, e1, C, c) : 0.0f;
  float acc = 0.0f;
  for (int32_t e = e0; e < e1; e += 4 * kStrand) {
    float v[4 * kStrand];
#pragma unroll
    for (int i = 0; i < 4 * kStrand; ++i) v[i] = e + i < e1 ? contrib[(int64_t)(e + i) * C + c] : 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t es = e + q * kStrand;
      if (es < e1) {
        float sum = v[q * kStrand];
#pragma unroll
        for (int i = 1; i < kStrand; ++i)
          if (es + i < e1) sum += v[q * kStrand + i];
        acc = (es == e0) ? sum : acc + sum;
      }
    }
  }
  return acc;
}

__device__ __forceinline__ float pull_sum(const float *__restrict__ contrib, int32_t e0,
                                          int32_t e1, int32_t C, int32_t c, bool active,
                                          int lane, bool serial) {
  if (serial) return active ? serial_pull(contrib, e0, e1, C, c) : 0.0f;
  const bool light = active && e1 - e0 <= kStrand;
  // the light ranges' loads go out before the heavy batching's shuffles
  float lv[kStrand];
  if (light) strand_load(contrib, e0, e1, C, c, lv);
  uint64_t heavy = __ballot(active && !light);
  // the wave's heavy nets take consecutive strand positions (lane order);
  // when they fit in 64, their strands load in the same round as the light
  // ranges
  // (A wave holds few heavy nets, so their offsets are a short uniform loop
  // over the heavy lanes; lane values are read with readlane, a register
  // read, rather than cross-lane shuffles through LDS.)
  bool batched = false;
  int32_t cnt = 0, my_h = -1, my_j = 0;
  if (heavy) {
    cnt = ((heavy >> lane) & 1) ? (e1 - e0 + kStrand - 1) / kStrand : 0;
    int32_t run = 0;
    for (uint64_t hh = heavy; hh; hh &= hh - 1) {
      const int h = __builtin_ctzll(hh);
      const int32_t hc = __builtin_amdgcn_readlane(cnt, h);
      if (lane >= run && lane < run + hc) {
        my_h = h;
        my_j = lane - run;
      }
      run += hc;
    }
    batched = run <= 64;
    if (!batched) my_h = -1;
  }
  int32_t hbeg = 0, hend = 0, hcol = 0;
  if (batched) {
    const int src = my_h < 0 ? lane : my_h;
    hbeg = __shfl(e0, src) + my_j * kStrand;
    hend = __shfl(e1, src);
    hcol = __shfl(c, src);
  }
  float hv[kStrand];
  if (my_h >= 0) strand_load(contrib, hbeg, hend, C, hcol, hv);
  float acc = light ? strand_fold(lv, e1 - e0) : 0.0f;
  if (!heavy) return acc;
  if (batched) {
    const float v = my_h >= 0 ? strand_fold(hv, hend - hbeg) : 0.0f;
    const int32_t vbits = __float_as_int(v);
    // each heavy net folds its strand sums in strand order
    int32_t run = 0;
    for (uint64_t hh = heavy; hh; hh &= hh - 1) {
      const int h = __builtin_ctzll(hh);
      const int32_t hc = __builtin_amdgcn_readlane(cnt, h);
      float total = __int_as_float(__builtin_amdgcn_readlane(vbits, run));
      for (int32_t t = 1; t < hc; ++t)
        total = total + __int_as_float(__builtin_amdgcn_readlane(vbits, run + t));
      if (lane == h) acc = total;
      run += hc;
    }
    return acc;
  }
  while (heavy) {
    const int src = __builtin_ctzll(heavy);
    heavy &= heavy - 1;
    const int32_t h0 = __shfl(e0, src), h1 = __shfl(e1, src), hc = __shfl(c, src);
    const int32_t strands = (h1 - h0 + kStrand - 1) / kStrand;
    float total = 0.0f;
    for (int32_t base = 0; base < strands; base += 64) {
      const int32_t j = base + lane;
      const float v = j < strands ? strand_sum(contrib, h0 + j * kStrand, h1, C, hc) : 0.0f;
      const int32_t m = min(64, strands - base);
      for (int32_t t = 0; t < m; ++t) {
        const float u = __shfl(v, t);
        total = (base == 0 && t == 0) ? u : total + u;
      }
    }
    if (lane == src) acc = total;
  }
  return acc;
}

// Eq. 7 for one level: a gate's output adjoint is its seed plus the
// contributions its readers left on their fan-in slots (pulled in a fixed
// order, so the sum is deterministic); it then leaves lambda * dR/dx_j on
// each of its own fan-in slots.  Items are (gate, column) pairs, column
// innermost; item counts stay below 2^31.
// One (gate, column) item of a reverse level; every lane of the wave calls
// it (pull_sum needs the whole wave), lanes past the end pass active = false.
// WIDE (fixed cells): the launch's column count is at least kSerialColumns
// (pulls are lane-serial); a choice per launch, so each form keeps its own
// registers.  Library cells decide the pull per launch at run time.
// skip_heavy (WIDE only): items of gates with more than kHeavyPull fan-out
// entries are left to the launch's cooperative blocks (bwd_heavy).
// UNI (WIDE, a multiple of 64 columns): every wave holds one gate, so the
// gate's values are made wave-uniform once loaded (scalar branches, scalar
// row addresses, loops with scalar bounds).
template <bool CELLS, bool WIDE, bool UNI = false>
__device__ __forceinline__ void bwd_item(const GraphView &g, const BwdArgs &a, int32_t g0,
                                         int32_t n, uint32_t idx, int lane,
                                         bool skip_heavy = false) {
  const bool active = idx < (uint32_t)n * (uint32_t)a.C;
  // lanes past the end read row g0 (a level has at least one gate) and
  // store nothing, so no load needs a guard for them
  const uint32_t gl = active ? idx / (uint32_t)a.C : 0;
  const int32_t c = active ? (int32_t)(idx - gl * (uint32_t)a.C) : 0;
  const int32_t gi = g0 + (int32_t)gl;
  const int32_t out = g.n_pi + gi;
  const int32_t b = c / a.cdiv;
  const float *sp = a.sp;
  const f2 z = f2{0.0f, 1.0f};
  // first round: the item's structure and its own net's values; nothing here
  // waits on another load
  int32_t e0 = g.rev_ptr[out];
  int32_t e1r = g.rev_ptr[out + 1];
  int op = g.op[gi];
  const float sp_out = sp[(int64_t)out * a.B + b];
  const float beta = a.beta ? a.beta[a.beta_shared ? (int64_t)out : (int64_t)out * a.B + b] : 1.0f;
  const float cap = a.cap[out];
  if constexpr (CELLS) {  // library cell: partials over its code
    // the first round also takes every pin's index and slot; the second
    // every pin's probability, the cell's code and the pull, none of them
    // waiting on another
    int32_t pin[kCellMaxIn], sl[kCellMaxIn];
#pragma unroll
    for (int j = 0; j < kCellMaxIn; ++j) {
      pin[j] = j < g.pins ? g.in[j * g.G + gi] : 0;
      sl[j] = j < g.pins ? g.slot[j * g.G + gi] : 0;
    }
#pragma unroll
    for (int j = 0; j < kCellMaxIn; ++j) value_taken(pin[j]);
    float r[kCellMaxIn];
#pragma unroll
    for (int j = 0; j < kCellMaxIn; ++j) r[j] = j < g.pins ? sp[(int64_t)pin[j] * a.B + b] : 0.0f;
    const LaneCode lc = lane_code(g, op);
    const int32_t e1 = active ? e1r : e0;  // lanes past the end pull nothing
    const float pulled =
        pull_sum(a.contrib, e0, e1, a.C, c, active, lane, a.C >= kSerialColumnsNoHeavy);
    if (!active) return;
    float lam = seed_of(a, out, c, b, sp_load(sp_out), beta, cap) + pulled;
    if (a.ste) lam *= beta;
    if (a.lam) a.lam[(int64_t)c * (a.n_pi + a.G) + out] = lam;
    f2 x[kCellMaxIn];
    float d[kCellMaxIn];
#pragma unroll
    for (int j = 0; j < kCellMaxIn; ++j) x[j] = j < g.pins ? sp_load(r[j]) : z;
    cell_partials(lc, x, d);
#pragma unroll
    for (int j = 0; j < kCellMaxIn; ++j)
      if (j < lc.nin) a.contrib[(int64_t)sl[j] * a.C + c] = lam * d[j];
    return;
  }
  // every pin's index and slot go out with the opcode and the fan-out range
  // (unused pin rows alias pin 0); taken here, so none of them is moved
  // into the branch of the arity that reads it (each would add a dependent
  // round trip)
  int32_t i0 = g.in[gi];
  int32_t i1 = pin_row(g.in, g, 1)[gi];
  int32_t i2 = pin_row(g.in, g, 2)[gi];
  int32_t s0 = g.slot[gi];
  int32_t s1 = pin_row(g.slot, g, 1)[gi];
  int32_t s2 = pin_row(g.slot, g, 2)[gi];
  gathers_done(op, e0, e1r, i0, i1, i2, s0, s1, s2);
  if constexpr (UNI) {
    e0 = __builtin_amdgcn_readfirstlane(e0);
    e1r = __builtin_amdgcn_readfirstlane(e1r);
    op = __builtin_amdgcn_readfirstlane(op);
    i0 = __builtin_amdgcn_readfirstlane(i0);
    i1 = __builtin_amdgcn_readfirstlane(i1);
    i2 = __builtin_amdgcn_readfirstlane(i2);
    s0 = __builtin_amdgcn_readfirstlane(s0);
    s1 = __builtin_amdgcn_readfirstlane(s1);
    s2 = __builtin_amdgcn_readfirstlane(s2);
  }
  // second round: every pin's probability, whatever the opcode (a pin the
  // gate lacks reads pin 0's row again, a cache hit), beside the pull's
  // loads; the values are unpacked only after the pull, so no load waits
  // on another
  const float r0 = sp[(int64_t)i0 * a.B + b];
  const float r1 = sp[(int64_t)i1 * a.B + b];
  const float r2 = sp[(int64_t)i2 * a.B + b];
  if (WIDE && skip_heavy && e1r - e0 > kHeavyPull) return;
  const int32_t e1 = active ? e1r : e0;  // lanes past the end pull nothing
  const float pulled = pull_sum(a.contrib, e0, e1, a.C, c, active, lane, WIDE);
  if (!active) return;
  float lam = seed_of(a, out, c, b, sp_load(sp_out), beta, cap) + pulled;
  if (a.ste) lam *= beta;
  if (a.lam) a.lam[(int64_t)c * (a.n_pi + a.G) + out] = lam;
  const int k = arity_of(op);
  float d0, d1, d2;
  sp_partials(op, sp_load(r0), k > 1 ? sp_load(r1) : z, k > 2 ? sp_load(r2) : z, d0, d1, d2);
  a.contrib[(int64_t)s0 * a.C + c] = lam * d0;
  if (k > 1) a.contrib[(int64_t)s1 * a.C + c] = lam * d1;
  if (k > 2) a.contrib[(int64_t)s2 * a.C + c] = lam * d2;
}

// One gate with a long fan-out range, for 64 columns of a many-column
// reverse level, by a whole workgroup.  Lane-serially, one lane would pull a
// net's entries 32 at a time, one dependent round each (a 200-reader net:
// seven rounds, the level's critical path).  Here the waves share the
// strands: wave w sums strand groups w, w + waves, ... (four strands, 32
// loads, per group) into LDS, and wave 0 folds the strand sums in strand
// order: the canonical sum, bit for bit.  Wave 0 then finishes the item as
// bwd_item does; its own values and fan-in gathers go out before the pull.
constexpr int32_t kHeavyPass = 64;  // strand sums held in LDS at a time

// The canonical sum of [e0, e1) for column c by the whole workgroup; the
// result is meaningful in wave 0 (every thread must call it).
__device__ __forceinline__ float heavy_pull(const float *__restrict__ contrib, int32_t e0,
                                            int32_t e1, int32_t C, int32_t c) {
  __shared__ float ss[kHeavyPass][64];
  const int w = (int)(threadIdx.x >> 6), nw = (int)(blockDim.x >> 6), lane = threadIdx.x & 63;
  const int32_t strands = (e1 - e0 + kStrand - 1) / kStrand;
  float pulled = 0.0f;
  for (int32_t p0 = 0; p0 < strands; p0 += kHeavyPass) {
    const int32_t np = min(kHeavyPass, strands - p0);
    for (int32_t q = 4 * w; q < np; q += 4 * nw) {
      const int32_t es = e0 + (p0 + q) * kStrand;
      float v[4 * kStrand];
#pragma unroll
      for (int i = 0; i < 4 * kStrand; ++i)
        v[i] = es + i < e1 ? contrib[(int64_t)(es + i) * C + c] : 0.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int32_t st = es + t * kStrand;
        if (q + t < np) {
          float sum = v[t * kStrand];
#pragma unroll
          for (int i = 1; i < kStrand; ++i)
            if (st + i < e1) sum += v[t * kStrand + i];
          ss[q + t][lane] = sum;
        }
      }
    }
    __syncthreads();
    if (w == 0)
      for (int32_t t = 0; t < np; ++t) pulled = (p0 == 0 && t == 0) ? ss[0][lane] : pulled + ss[t][lane];
    __syncthreads();
  }
  return pulled;
}

__device__ __forceinline__ void bwd_heavy(const GraphView &g, const BwdArgs &a,
                                          const int32_t *__restrict__ heavy, uint32_t hb) {
  const int32_t cgroups = (a.C + 63) / 64;
  const int32_t gi = heavy[hb / (uint32_t)cgroups];
  const int32_t cg = (int32_t)(hb % (uint32_t)cgroups);
  const int w = (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const bool active = cg * 64 + lane < a.C;
  const int32_t c = active ? cg * 64 + lane : cg * 64;  // idle lanes load in-row
  const int32_t out = g.n_pi + gi;
  const int32_t b = c / a.cdiv;
  const float *sp = a.sp;
  const f2 z = f2{0.0f, 1.0f};
  const int32_t e0 = g.rev_ptr[out], e1 = g.rev_ptr[out + 1];
  const int op = g.op[gi];
  const int k = arity_of(op);
  const f2 pq = sp_load(sp[(int64_t)out * a.B + b]);
  const float beta = a.beta ? a.beta[a.beta_shared ? (int64_t)out : (int64_t)out * a.B + b] : 1.0f;
  const float cap = a.cap[out];
  // every pin's index and slot in the first round (unused pin rows alias
  // pin 0), every pin's probability beside the pull's first loads
  const int32_t i0 = g.in[gi], s0 = g.slot[gi];
  const int32_t i1 = pin_row(g.in, g, 1)[gi], s1 = pin_row(g.slot, g, 1)[gi];
  const int32_t i2 = pin_row(g.in, g, 2)[gi], s2 = pin_row(g.slot, g, 2)[gi];
  gathers_done(i0, i1, i2);
  const float r0 = sp[(int64_t)i0 * a.B + b];
  const float r1 = sp[(int64_t)i1 * a.B + b];
  const float r2 = sp[(int64_t)i2 * a.B + b];
  const float pulled = heavy_pull(a.contrib, e0, e1, a.C, c);
  if (w != 0 || !active) return;
  float lam = seed_of(a, out, c, b, pq, beta, cap) + pulled;
  if (a.ste) lam *= beta;
  if (a.lam) a.lam[(int64_t)c * (a.n_pi + a.G) + out] = lam;
  float d0, d1, d2;
  sp_partials(op, sp_load(r0), k > 1 ? sp_load(r1) : z, k > 2 ? sp_load(r2) : z, d0, d1, d2);
  a.contrib[(int64_t)s0 * a.C + c] = lam * d0;
  if (k > 1) a.contrib[(int64_t)s1 * a.C + c] = lam * d1;
  if (k > 2) a.contrib[(int64_t)s2 * a.C + c] = lam * d2;
}

// With many columns the first heavy_blocks blocks take the level's heavy
// gates (heavy[0, n_heavy), in groups of 64 columns; first, so their longer
// pulls start first), and the blocks after them the (gate, column) items,
// skipping the heavy gates.
template <bool CELLS, bool WIDE, bool UNI = false>
__global__ __launch_bounds__(kWideBlock) void k_bwd_level(GraphView g, BwdArgs a, int32_t g0,
                                                           int32_t n, const int32_t *heavy,
                                                           int32_t n_heavy, uint32_t heavy_blocks) {
  if constexpr (WIDE && !CELLS) {
    if (blockIdx.x < heavy_blocks) {
      bwd_heavy(g, a, heavy, blockIdx.x);
      return;
    }
  }
  bwd_item<CELLS, WIDE, UNI>(g, a, g0, n, (blockIdx.x - heavy_blocks) * blockDim.x + threadIdx.x,
                             threadIdx.x & 63, n_heavy > 0);
}

// skip_heavy: PIs with more than kHeavyPull fan-out entries are left to the
// launch's cooperative blocks (bwd_pi_heavy).
// serial_cols: the column count from which pulls are lane-serial (the
// launch's choice: with or without heavy-PI workgroups).
__device__ __forceinline__ void bwd_pi_item(const GraphView &g, const BwdArgs &a, float *out,
                                            uint32_t idx, int lane, bool skip_heavy = false,
                                            int32_t serial_cols = kSerialColumns) {
  const bool active = idx < (uint32_t)g.n_pi * (uint32_t)a.C;
  const uint32_t i = active ? idx / (uint32_t)a.C : 0;
  const int32_t c = active ? (int32_t)(idx - i * (uint32_t)a.C) : 0;
  const int32_t e0 = g.rev_ptr[i];  // lanes past the end read PI 0 and store nothing
  const int32_t e1r = g.rev_ptr[i + 1];
  const int32_t e1 = active ? e1r : e0;
  const int32_t b = c / a.cdiv;
  const f2 pq = sp_load(a.sp[(int64_t)i * a.B + b]);
  const float beta = a.beta ? a.beta[a.beta_shared ? (int64_t)i : (int64_t)i * a.B + b] : 1.0f;
  const float cap = a.cap[i];
  const bool serial = a.C >= serial_cols;
  if (serial && skip_heavy && e1r - e0 > kHeavyPull) return;  // (lane-serial pulls only)
  const float pulled = pull_sum(a.contrib, e0, e1, a.C, c, active, lane, serial);
  if (!active) return;
  float lam = seed_of(a, (int32_t)i, c, b, pq, beta, cap) + pulled;
  if (a.ste) lam *= beta;
  if (a.fixed && a.fixed[i]) lam = 0.0f;  // excluded from the gradients
  out[(int64_t)c * g.n_pi + i] = lam;
  if (a.lam) a.lam[(int64_t)c * (a.n_pi + a.G) + i] = lam;
}

// A PI with a long fan-out range, for 64 columns, by a whole workgroup (as
// bwd_heavy for gates).
__device__ __forceinline__ void bwd_pi_heavy(const GraphView &g, const BwdArgs &a, float *out,
                                             const int32_t *__restrict__ heavy, uint32_t hb) {
  const int32_t cgroups = (a.C + 63) / 64;
  const int32_t i = heavy[hb / (uint32_t)cgroups];
  const int32_t cg = (int32_t)(hb % (uint32_t)cgroups);
  const int w = (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const bool active = cg * 64 + lane < a.C;
  const int32_t c = active ? cg * 64 + lane : cg * 64;
  const int32_t b = c / a.cdiv;
  const int32_t e0 = g.rev_ptr[i], e1 = g.rev_ptr[i + 1];
  const f2 pq = sp_load(a.sp[(int64_t)i * a.B + b]);
  const float beta = a.beta ? a.beta[a.beta_shared ? (int64_t)i : (int64_t)i * a.B + b] : 1.0f;
  const float cap = a.cap[i];
  const float pulled = heavy_pull(a.contrib, e0, e1, a.C, c);
  if (w != 0 || !active) return;
  float lam = seed_of(a, i, c, b, pq, beta, cap) + pulled;
  if (a.ste) lam *= beta;
  if (a.fixed && a.fixed[i]) lam = 0.0f;
  out[(int64_t)c * g.n_pi + i] = lam;
  if (a.lam) a.lam[(int64_t)c * (a.n_pi + a.G) + i] = lam;
}

// The first heavy_blocks blocks take the heavy PIs (many columns only).
__global__ __launch_bounds__(kBlock) void k_bwd_pi(GraphView g, BwdArgs a, float *out,
                                                   const int32_t *heavy, int32_t n_heavy,
                                                   uint32_t heavy_blocks) {
  if (blockIdx.x < heavy_blocks) {
    bwd_pi_heavy(g, a, out, heavy, blockIdx.x);
    return;
  }
  bwd_pi_item(g, a, out, (blockIdx.x - heavy_blocks) * kBlock + threadIdx.x, threadIdx.x & 63,
              n_heavy > 0);
}

// ---------------------------------------------------------------- adjoints and scores
__global__ __launch_bounds__(kBlock) void k_grad_lambda_export(
    const float *__restrict__ lam, const float *__restrict__ sp, const int32_t *__restrict__ int2ext,
    int32_t n_pi, int32_t n_nets, int32_t B, int32_t C, int32_t cdiv, float eps, float *lam_out,
    float *score) {
  const int64_t idx = gidx();
  if (idx >= (int64_t)n_nets * C) return;
  const int32_t c = (int32_t)(idx / n_nets), n = (int32_t)(idx - (int64_t)c * n_nets);
  const float l = lam[idx];
  const int32_t e = int2ext[n];
  if (lam_out) lam_out[(int64_t)c * n_nets + e] = l;
  if (score && n >= n_pi) {
    const f2 pq = sp_load(sp[(int64_t)n * B + c / cdiv]);
    const float slope = fmaxf(fabsf(pq.y - pq.x), eps);  // |1 - 2P| from the pair
    score[(int64_t)c * (n_nets - n_pi) + (e - n_pi)] = fabsf(l) * (pq.x * pq.y) / slope;
  }
}

// ---------------------------------------------------------------- power virus
// One ascent step of Alg. 4 on the startpoints, kept as (p, 1 - p) pairs.
__global__ __launch_bounds__(kBlock) void k_virus_step(float *sp, const float *__restrict__ grad,
                                                       float eta, int32_t n_pi, int32_t B) {
  const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (uint32_t)n_pi * (uint32_t)B) return;
  const int32_t i = (int32_t)(idx / (uint32_t)B), b = (int32_t)(idx - (uint32_t)i * B);
  const float p = clamp01(fmaf(eta, grad[(int64_t)b * n_pi + i], sp_load(sp[idx]).x));
  sp[idx] = sp_pack(p);
}

// Threshold at 1/2 and spell out the two-cycle stimulus (v0, 1 - v0).
__global__ __launch_bounds__(kBlock) void k_virus_vectors(const float *__restrict__ sp,
                                                          uint64_t *stim, uint8_t *v0,
                                                          float *p_out, int32_t n_pi, int32_t B) {
  const uint32_t idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (uint32_t)n_pi * (uint32_t)B) return;
  const int32_t b = (int32_t)(idx / (uint32_t)n_pi), i = (int32_t)(idx - (uint32_t)b * n_pi);
  const float p = sp_load(sp[(int64_t)i * B + b]).x;
  const bool one = p >= 0.5f;
  v0[idx] = one ? 1 : 0;
  if (p_out) p_out[idx] = p;
  const uint64_t w0 = one ? ~0ull : 0ull;
  stim[2 * (int64_t)idx] = w0;
  stim[2 * (int64_t)idx + 1] = ~w0;
}

// One block per column: thread t adds nets t, t + 256, ... in order, then a
// fixed tree over the block.
__global__ __launch_bounds__(kBlock) void k_virus_power(const uint32_t *__restrict__ tog,
                                                        const float *__restrict__ cap,
                                                        int32_t n_nets, int32_t B, double *out) {
  __shared__ double lds[kWavesPerBlock];
  const int32_t b = blockIdx.x;
  double acc = 0.0;
  for (int32_t n = threadIdx.x; n < n_nets; n += kBlock)
    if (tog[(int64_t)n * B + b] != 0u) acc += (double)cap[n];
  const double r = block_sum_d(acc, lds);
  if (threadIdx.x == 0) out[b] = r;
}

// ---------------------------------------------------------------- several designs
// The segment of this block (uniform over the block: a short scalar scan).
template <class Seg>
__device__ __forceinline__ int32_t seg_of(const Seg *__restrict__ segs, int32_t n_segs) {
  int32_t k = 0;
  while (k + 1 < n_segs && segs[k + 1].block0 <= blockIdx.x) ++k;
  return k;
}

template <bool CELLS>
__global__ __launch_bounds__(kMergedBlock) void k_sp_multi(const SpSeg *__restrict__ segs,
                                                           int32_t n_segs) {
  const SpSeg sg = segs[seg_of(segs, n_segs)];
  const uint32_t idx = (blockIdx.x - sg.block0) * kMergedBlock + threadIdx.x;
  if (!CELLS && sg.lv2.n > 0) {  // two levels of this design: launch_sp_pair's items
    sp_pair_item(sg.g, sg.lv, sg.lv2, idx);
    return;
  }
  if (idx < (uint32_t)sg.lv.n * (uint32_t)sg.lv.B) sp_item<CELLS>(sg.g, sg.lv, idx);
}

template <bool CELLS>
__global__ __launch_bounds__(kMergedBlock) void k_bwd_multi(const BwdSeg *__restrict__ segs,
                                                            int32_t n_segs) {
  const BwdSeg sg = segs[seg_of(segs, n_segs)];
  const uint32_t idx = (blockIdx.x - sg.block0) * kMergedBlock + threadIdx.x;
  if (!CELLS && sg.a.C >= kSerialColumnsNoHeavy)  // segments differ in width: chosen per block
    bwd_item<CELLS, true>(sg.g, sg.a, sg.g0, sg.n, idx, threadIdx.x & 63);
  else
    bwd_item<CELLS, false>(sg.g, sg.a, sg.g0, sg.n, idx, threadIdx.x & 63);
}

// ---------------------------------------------------------------- persistent sweeps
// One cooperative launch runs every level: a grid-stride loop over the
// level's items, then a grid barrier.  Whole waves step together so the
// wave-wide pull of the reverse sweep sees all its lanes.
//
// The barrier: at barrier k every block, once all its threads have stored
// their results, publishes k in its own arrival flag (a release store at
// device scope, which makes the block's stores visible beyond its XCD's L2);
// then the block's first wave reads all the flags, 64 at a time (lane i
// reads flags i, i + 64, ...), until every flag reads k or more, and takes
// one acquire fence.  No block waits on another's atomic: a barrier costs
// one release, the store's trip and the reads that see the last one.
// Cooperative launch keeps every block resident, so every wait ends; as a
// guard, a wait that sees no new arrival for limit_ticks ticks of the
// 100 MHz real-time counter sets the timeout flag and stops, a wait that
// finds the flag set stops at once, and the sweep's outputs are then written
// as NaN.  The wait that gives up also sets the report word, which the host
// reads at its next synchronization, so a broken sweep is reported and
// cannot pass for a result.
__device__ __forceinline__ bool barrier_timed_out(const GridBarrier &bar) {
  return __hip_atomic_load(bar.words + kBarrierTimeout, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

__device__ __forceinline__ void grid_barrier(const GridBarrier &bar, uint32_t k) {
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x, blocks = gridDim.x;
    if (lane == 0)
      __hip_atomic_store(bar.words + blockIdx.x, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t seen = 0;
    uint64_t since = __builtin_amdgcn_s_memrealtime();
    for (uint32_t it = 0;; ++it) {
      uint32_t arrived = 0;
      for (uint32_t b = lane; b < blocks; b += 64)
        arrived += __hip_atomic_load(bar.words + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= k;
      arrived = wave_sum(arrived);
      if (arrived == blocks) break;
      if ((it & 15u) == 0u && barrier_timed_out(bar)) break;
      const uint64_t now = __builtin_amdgcn_s_memrealtime();
      if (arrived != seen) {  // a new arrival restarts the clock
        seen = arrived;
        since = now;
      }
      if (now - since >= bar.limit_ticks) {  // at a limit of 0: the first poll that waits
        if (lane == 0) {
          __hip_atomic_store(bar.words + kBarrierTimeout, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(bar.words + kBarrierReport, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// A level item's structure (opcode and pin indices), loaded apart from its
// gathers so the persistent sweep can fetch the next level's before it
// waits at the barrier: the indices do not depend on any level's results.
struct SpFetch {
  int32_t op, i0, i1, i2;
};

__device__ __forceinline__ SpFetch sp_fetch(const GraphView &g, int32_t gi) {
  SpFetch f;
  f.op = g.op[gi];
  f.i0 = g.in[gi];
  f.i1 = pin_row(g.in, g, 1)[gi];
  f.i2 = pin_row(g.in, g, 2)[gi];
  return f;
}

__device__ __forceinline__ void sp_finish(const GraphView &g, const SpLevel &lv, int32_t gi,
                                          int32_t b, const SpFetch &f) {
  const int32_t B = lv.B;
  float *sp = lv.sp;
  const int k = arity_of(f.op);
  const float sa = sp[(int64_t)f.i0 * B + b];
  float sb = 0.0f, sc = 0.0f;
  if (k > 1) sb = sp[(int64_t)f.i1 * B + b];
  if (k > 2) sc = sp[(int64_t)f.i2 * B + b];
  gathers_done(sa, sb, sc);
  const f2 z = f2{0.0f, 1.0f};
  sp[(int64_t)(g.n_pi + gi) * B + b] =
      settle(sp_rule(f.op, sp_load(sa), k > 1 ? sp_load(sb) : z, k > 2 ? sp_load(sc) : z));
}

__global__ __launch_bounds__(kBlock) void k_sp_persistent(GraphView g, SpLevel lv,
                                                          const int32_t *__restrict__ level_ptr,
                                                          int32_t depth, GridBarrier bar) {
  const uint32_t stride = gridDim.x * kBlock;
  const uint32_t first = blockIdx.x * kBlock + threadIdx.x;
  const uint32_t B = (uint32_t)lv.B;
  // this thread's first item of the coming level, fetched ahead
  int32_t g0 = level_ptr[1], n = level_ptr[2] - g0;
  SpFetch ahead{};
  if (first < (uint32_t)n * B) ahead = sp_fetch(g, g0 + (int32_t)(first / B));
  for (int32_t l = 1; l <= depth; ++l) {
    SpLevel cur = lv;
    cur.g0 = g0;
    cur.n = n;
    const uint32_t items = (uint32_t)n * B;
    for (uint32_t idx = first; idx < items; idx += stride) {
      const uint32_t gl = idx / B;
      const int32_t gi = g0 + (int32_t)gl;
      const SpFetch f = idx == first ? ahead : sp_fetch(g, gi);
      if (idx != first) gathers_done(f.op, f.i0, f.i1, f.i2);
      sp_finish(g, cur, gi, (int32_t)(idx - gl * B), f);
    }
    if (l < depth) {  // the next level's structure loads go out before the wait
      g0 = level_ptr[l + 1];
      n = level_ptr[l + 2] - g0;
      if (first < (uint32_t)n * B) ahead = sp_fetch(g, g0 + (int32_t)(first / B));
    }
    grid_barrier(bar, (uint32_t)l);
  }
  if (barrier_timed_out(bar)) {  // every gate's probability becomes NaN
    const int64_t nn = (int64_t)g.G * lv.B;
    float *out = lv.sp + (int64_t)g.n_pi * lv.B;
    for (int64_t i = first; i < nn; i += stride) out[i] = __builtin_nanf("");
  }
}

template <bool WIDE>
__global__ __launch_bounds__(kBlock) void k_bwd_persistent(GraphView g, BwdArgs a,
                                                           const int32_t *__restrict__ level_ptr,
                                                           int32_t depth, float *pi_out,
                                                           GridBarrier bar) {
  const uint32_t stride = gridDim.x * kBlock;
  const int lane = threadIdx.x & 63;
  const uint32_t first = blockIdx.x * kBlock + threadIdx.x;
  for (int32_t l = depth; l >= 1; --l) {
    const int32_t g0 = level_ptr[l], n = level_ptr[l + 1] - g0;
    const uint32_t items = (uint32_t)n * (uint32_t)a.C;
    // round the trip count up to whole waves
    for (uint32_t base = first - lane; base < items; base += stride)
      bwd_item<false, WIDE>(g, a, g0, n, base + lane, lane);
    grid_barrier(bar, (uint32_t)(depth - l + 1));
  }
  const uint32_t items = (uint32_t)g.n_pi * (uint32_t)a.C;
  if (barrier_timed_out(bar)) {  // the gradient becomes NaN
    for (uint32_t i = first; i < items; i += stride) pi_out[i] = __builtin_nanf("");
    return;
  }
  for (uint32_t base = first - lane; base < items; base += stride)
    bwd_pi_item(g, a, pi_out, base + lane, lane, false, kSerialColumnsNoHeavy);
}

// dP/dC_n = sum_{b,s} w[b][s] kappa beta TR_model s_s(drv n);
// dP/ds[s][g] = sum_b w[b][s] kappa beta TR_model C of g's output net.
// x = kappa beta TR_model of net n in column b, recomputed as the forward's
// power sum computed it.
__device__ __forceinline__ float x_of(const GradExportArgs &a, int64_t n, int32_t b) {
  const int64_t idx = n * a.B + b;
  const f2 pq = sp_load(a.sp[idx]);
  const float tm = 2.0f * pq.x * pq.y;
  const float beta = a.beta ? a.beta[a.beta_shared ? n : idx] : 1.0f;
  return a.kappa * beta * tm;
}

// One wave per 64 nets.  The x values of the nets' rows are staged through
// LDS a tile of up to 32 columns at a time (consecutive lanes read
// consecutive (net, column) entries, so the loads are whole row segments;
// sixteen go out before the first store), then lane r sums its net's
// columns in order.
constexpr int32_t kCapRows = 64, kCapCols = 32, kCapBatch = 16;

template <bool BETA>  // BETA: a beta array is present
__global__ __launch_bounds__(kCapRows) void k_grad_cap(GradExportArgs a) {
  __shared__ float xs[kCapRows][kCapCols + 1];
  __shared__ float wcol[kCapCols];  // without sizes a column's weight is the net's
  const int32_t r = (int32_t)threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * kCapRows;
  const int64_t n = n0 + r;
  const int32_t rows = (int32_t)min<int64_t>(kCapRows, a.n_nets - n0);
  const int32_t Sp = (a.S > 0 && !a.paired) ? a.S : 1;
  const bool gate = n >= a.n_pi && a.size;
  auto weight = [&](int32_t b) {
    float ws = 0.0f;
    for (int32_t s = 0; s < Sp; ++s) {
      const int32_t row = a.paired ? b : s;
      const float w = a.w ? a.w[(int64_t)b * Sp + s] : 1.0f;
      const float sz = gate ? a.size[(int64_t)row * a.G + (n - a.n_pi)] : 1.0f;
      ws = fmaf(w, sz, ws);
    }
    return ws;
  };
  double acc = 0.0;
  for (int32_t b0 = 0; b0 < a.B; b0 += kCapCols) {
    const int32_t tw = min(kCapCols, a.B - b0), total = rows * tw;
    for (int32_t e0 = r; e0 < total; e0 += kCapBatch * kCapRows) {
      float v[kCapBatch];
      float bt[kCapBatch];
      // (row, column) of entry e: shifts for a whole tile, else a division
      const bool full = tw == kCapCols;
#pragma unroll
      for (int u = 0; u < kCapBatch; ++u) {  // clamped: every load is valid
        const int32_t e = min(e0 + u * kCapRows, total - 1);
        const int32_t rr = full ? e / kCapCols : e / tw;
        const int64_t nn = n0 + rr, idx = nn * a.B + b0 + (e - rr * tw);
        v[u] = a.sp[idx];
        bt[u] = BETA ? a.beta[a.beta_shared ? nn : idx] : 1.0f;
      }
#pragma unroll
      for (int u = 0; u < kCapBatch; ++u) {  // x as x_of forms it
        const f2 pq = sp_load(v[u]);
        v[u] = a.kappa * bt[u] * (2.0f * pq.x * pq.y);
      }
#pragma unroll
      for (int u = 0; u < kCapBatch; ++u) {
        const int32_t e = e0 + u * kCapRows, rr = full ? e / kCapCols : e / tw;
        if (e < total) xs[rr][e - rr * tw] = v[u];
      }
    }
    // without sizes the weight of column b is the same for every net: one
    // lane per column forms it (as weight() would), the row loop reads it
    if (!a.size && r < tw) wcol[r] = weight(b0 + r);
    __syncthreads();
    if (r < rows) {
      if (!a.size)
        for (int32_t cc = 0; cc < tw; ++cc) acc += (double)xs[r][cc] * (double)wcol[cc];
      else
        for (int32_t cc = 0; cc < tw; ++cc) acc += (double)xs[r][cc] * (double)weight(b0 + cc);
    }
    __syncthreads();
  }
  if (r < rows) a.dcap[a.int2ext[n]] = (float)acc;
}

// Few columns: one thread per net, its columns in order (the same sum as
// k_grad_cap); consecutive threads read consecutive rows, which at few
// columns are already whole lines, and no LDS pass is needed.
constexpr int32_t kCapRowsMinCols = 16;  // from this many columns k_grad_cap stages rows

__global__ __launch_bounds__(kBlock) void k_grad_cap_narrow(GradExportArgs a) {
  const int64_t n = gidx();
  if (n >= a.n_nets) return;
  const int32_t Sp = (a.S > 0 && !a.paired) ? a.S : 1;
  const bool gate = n >= a.n_pi && a.size;
  double acc = 0.0;
  for (int32_t b = 0; b < a.B; ++b) {
    float ws = 0.0f;
    for (int32_t s = 0; s < Sp; ++s) {
      const int32_t row = a.paired ? b : s;
      const float w = a.w ? a.w[(int64_t)b * Sp + s] : 1.0f;
      const float sz = gate ? a.size[(int64_t)row * a.G + (n - a.n_pi)] : 1.0f;
      ws = fmaf(w, sz, ws);
    }
    acc += (double)x_of(a, n, b) * (double)ws;
  }
  a.dcap[a.int2ext[n]] = (float)acc;
}

__global__ __launch_bounds__(kBlock) void k_grad_size(GradExportArgs a) {
  const int64_t idx = gidx();
  if (idx >= (int64_t)a.G * a.S) return;
  const int32_t s = (int32_t)(idx / a.G), g = (int32_t)(idx - (int64_t)s * a.G);
  const int32_t n = a.n_pi + g;
  double acc = 0.0;
  if (a.paired) {  // size row s belongs to column s only
    acc = (double)x_of(a, n, s) * (double)(a.w ? a.w[s] : 1.0f);
  } else {
    for (int32_t b = 0; b < a.B; ++b) {
      const float w = a.w ? a.w[(int64_t)b * a.S + s] : 1.0f;
      acc += (double)x_of(a, n, b) * (double)w;
    }
  }
  a.dsize[(int64_t)s * a.G + (a.int2ext[n] - a.n_pi)] = (float)(acc * (double)a.cap[n]);
}

}  // namespace

// ==================================================================== launchers
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_fill_u32<<<blocks_for(n), kBlock, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_fill_f32<<<blocks_for(n), kBlock, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_load_pi(const float *p, float *sp, int32_t n_pi, int32_t B, hipStream_t s) {
  const int64_t n = (int64_t)n_pi * B;
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_load_pi<<<blocks_for(n), kBlock, 0, s>>>(p, sp, n_pi, B);
  return hipGetLastError();
}

hipError_t launch_check_range(const float *v, int64_t n, float lo, float hi, int32_t *bad,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_check_range<<<blocks_for(n), kBlock, 0, s>>>(v, n, lo, hi, bad);
  return hipGetLastError();
}

hipError_t launch_gather_nets_f32(const float *src_ext, const int32_t *int2ext, float *dst_int,
                                  int32_t n_nets, hipStream_t s) {
  if (n_nets <= 0) return hipSuccess;
  k_gather_nets<<<blocks_for(n_nets), kBlock, 0, s>>>(src_ext, int2ext, dst_int, n_nets);
  return hipGetLastError();
}

hipError_t launch_import_cols_f32(const float *src, const int32_t *int2ext, float *dst,
                                  int32_t n_nets, int32_t B, hipStream_t s) {
  const int64_t n = (int64_t)n_nets * B;
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_import_cols<<<blocks_for(n), kBlock, 0, s>>>(src, int2ext, dst, n_nets, B);
  return hipGetLastError();
}

hipError_t launch_import_sizes(const float *src, const int32_t *int2ext, float *dst, int32_t n_pi,
                               int32_t G, int32_t S, hipStream_t s) {
  const int64_t n = (int64_t)G * S;
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_import_sizes<<<blocks_for(n), kBlock, 0, s>>>(src, int2ext, dst, n_pi, G, S);
  return hipGetLastError();
}

hipError_t launch_grad_lambda_export(const float *lam, const float *sp, const int32_t *int2ext,
                                     int32_t n_pi, int32_t n_nets, int32_t B, int32_t C,
                                     int32_t cdiv, float eps, float *lam_out, float *score,
                                     hipStream_t s) {
  const int64_t n = (int64_t)n_nets * C;
  if (n <= 0 || (!lam_out && !score)) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_grad_lambda_export<<<blocks_for(n), kBlock, 0, s>>>(lam, sp, int2ext, n_pi, n_nets, B, C,
                                                        cdiv, eps, lam_out, score);
  return hipGetLastError();
}

hipError_t launch_virus_step(float *sp, const float *grad, float eta, int32_t n_pi, int32_t B,
                             hipStream_t s) {
  const int64_t n = (int64_t)n_pi * B;
  if (n <= 0) return hipSuccess;
  if (n >= (1ll << 31)) return hipErrorInvalidValue;
  k_virus_step<<<blocks_for(n), kBlock, 0, s>>>(sp, grad, eta, n_pi, B);
  return hipGetLastError();
}

hipError_t launch_virus_vectors(const float *sp, uint64_t *stim, uint8_t *v0, float *p_out,
                                int32_t n_pi, int32_t B, hipStream_t s) {
  const int64_t n = (int64_t)n_pi * B;
  if (n <= 0) return hipSuccess;
  if (n >= (1ll << 31)) return hipErrorInvalidValue;
  k_virus_vectors<<<blocks_for(n), kBlock, 0, s>>>(sp, stim, v0, p_out, n_pi, B);
  return hipGetLastError();
}

hipError_t launch_virus_power(const uint32_t *tog, const float *cap, int32_t n_nets, int32_t B,
                              double *out, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  k_virus_power<<<(unsigned)B, kBlock, 0, s>>>(tog, cap, n_nets, B, out);
  return hipGetLastError();
}

hipError_t launch_sp_multi(const SpSeg *segs, int32_t n_segs, uint32_t blocks, bool cells,
                           hipStream_t s) {
  if (n_segs <= 0 || blocks == 0) return hipSuccess;
  if (cells)
    k_sp_multi<true><<<blocks, kMergedBlock, 0, s>>>(segs, n_segs);
  else
    k_sp_multi<false><<<blocks, kMergedBlock, 0, s>>>(segs, n_segs);
  return hipGetLastError();
}

hipError_t launch_bwd_multi(const BwdSeg *segs, int32_t n_segs, uint32_t blocks, bool cells,
                            hipStream_t s) {
  if (n_segs <= 0 || blocks == 0) return hipSuccess;
  if (cells)
    k_bwd_multi<true><<<blocks, kMergedBlock, 0, s>>>(segs, n_segs);
  else
    k_bwd_multi<false><<<blocks, kMergedBlock, 0, s>>>(segs, n_segs);
  return hipGetLastError();
}

hipError_t launch_sp_pair(const GraphView &g, const SpLevel &a, const SpLevel &b, hipStream_t s) {
  const int64_t n = ((int64_t)a.n + b.n) * a.B;
  if (n <= 0) return hipSuccess;
  if (n >= (1ll << 31) || a.B != b.B || a.sp != b.sp || b.g0 != a.g0 + a.n)
    return hipErrorInvalidValue;
  k_sp_pair<<<level_grid(n), level_block(n), 0, s>>>(g, a, b);
  return hipGetLastError();
}

hipError_t launch_sp_level(const GraphView &g, const SpLevel &lv, bool cells, hipStream_t s) {
  const int64_t n = (int64_t)lv.n * lv.B;
  if (n <= 0) return hipSuccess;
  if (n >= (1ll << 31)) return hipErrorInvalidValue;
  if (cells)
    k_sp_cells<<<blocks_for(n), kBlock, 0, s>>>(g, lv);
  else if (lv.B % 2 == 0)
    k_sp_level_x2<<<level_grid(n / 2), level_block(n / 2), 0, s>>>(g, lv);
  else
    k_sp_level<<<level_grid(n), level_block(n), 0, s>>>(g, lv);
  return hipGetLastError();
}

static int32_t waves_per_row(const ChunkView &c, int iters) {
  return (c.pairs + 64 * iters - 1) / (64 * iters);
}

hipError_t launch_stimulus(const GraphView &g, const ChunkView &c, const CountView &cnt,
                           const float *p_col, const uint64_t *stim, int64_t T,
                           const int32_t *stream, uint64_t seed, const SimTune &tune,
                           hipStream_t s) {
  if (g.n_pi <= 0 || c.pairs <= 0) return hipSuccess;
  if (c.n_cols <= 0) return hipSuccess;
  const int iters = tune.iters;
  const int32_t wpr = waves_per_row(c, iters);
  const int64_t tasks = (int64_t)g.n_pi * wpr * c.n_cols;
  if ((tasks + kWavesPerBlock - 1) / kWavesPerBlock > kMaxBlocks) return hipErrorInvalidValue;
  const unsigned grid = (unsigned)((tasks + kWavesPerBlock - 1) / kWavesPerBlock);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  switch (iters) {
    case 1: k_stimulus<1><<<grid, kBlock, 0, s>>>(g.n_pi, c, cnt, p_col, stim, T, stream, k0, k1, wpr); break;
    case 2: k_stimulus<2><<<grid, kBlock, 0, s>>>(g.n_pi, c, cnt, p_col, stim, T, stream, k0, k1, wpr); break;
    case 4: k_stimulus<4><<<grid, kBlock, 0, s>>>(g.n_pi, c, cnt, p_col, stim, T, stream, k0, k1, wpr); break;
    default: k_stimulus<8><<<grid, kBlock, 0, s>>>(g.n_pi, c, cnt, p_col, stim, T, stream, k0, k1, wpr); break;
  }
  return hipGetLastError();
}

hipError_t launch_markov_words(const float *sp, const float *tau, const int32_t *stream,
                               int32_t n_pi, int32_t B, int64_t T, uint64_t seed, uint64_t *out,
                               hipStream_t s) {
  const int64_t rows = (int64_t)n_pi * B;
  if (rows <= 0 || T <= 0) return hipSuccess;
  const int64_t blocks = (rows + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > kMaxBlocks) return hipErrorInvalidValue;
  k_markov_words<<<(unsigned)blocks, kBlock, 0, s>>>(sp, tau, stream, n_pi, B, T, (uint32_t)seed,
                                                     (uint32_t)(seed >> 32), out);
  return hipGetLastError();
}

hipError_t launch_sim_level(const GraphView &g, const ChunkView &c, const CountView &cnt,
                            int32_t g0, int32_t n, const SpLevel *sp, bool cells,
                            const SimTune &tune, hipStream_t s, int cell_inputs) {
  if (n <= 0 || c.n_cols <= 0) return hipSuccess;
  const bool narrow = cells && cell_inputs <= kSmallCellInputs;
  // cells: up to 2 pairs per lane (up to 6 input rows each), narrow cells up to 4
  const int iters = cells ? min(tune.iters, narrow ? 4 : 2) : tune.iters;
  const int32_t wpr = waves_per_row(c, iters);
  const int64_t tasks = (int64_t)n * wpr * c.n_cols;
  const int64_t sim_blocks64 = (tasks + kSimWaves - 1) / kSimWaves;
  SpLevel spl{};
  int64_t sp_blocks = 0;
  if (sp) {
    spl = *sp;
    if ((int64_t)spl.n * spl.B >= (1ll << 31)) return hipErrorInvalidValue;
    sp_blocks = ((int64_t)spl.n * spl.B + kSimBlock - 1) / kSimBlock;
  }
  if (sim_blocks64 + sp_blocks > kMaxBlocks || sim_blocks64 > INT32_MAX) return hipErrorInvalidValue;
  const int32_t sim_blocks = (int32_t)sim_blocks64;
  const unsigned grid = (unsigned)(sim_blocks + sp_blocks);
  if (narrow) {
    switch (iters) {
      case 1: k_sim_level<1, 3><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
      case 2: k_sim_level<2, 3><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
      default: k_sim_level<4, 3><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
    }
    return hipGetLastError();
  }
  if (cells) {
    if (iters == 1)
      k_sim_level<1, 6><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl);
    else
      k_sim_level<2, 6><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl);
    return hipGetLastError();
  }
  switch (iters) {
    case 1: k_sim_level<1, 0><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
    case 2: k_sim_level<2, 0><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
    case 4: k_sim_level<4, 0><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
    default: k_sim_level<8, 0><<<grid, kSimBlock, 0, s>>>(g, c, cnt, g0, n, wpr, sim_blocks, spl); break;
  }
  return hipGetLastError();
}

hipError_t launch_export(const ExportArgs &a, hipStream_t s) {
  const int64_t n = (int64_t)a.n_nets * a.B;
  if (n <= 0) return hipSuccess;
  if (too_big(n)) return hipErrorInvalidValue;
  k_export<<<blocks_for(n), kBlock, 0, s>>>(a);
  return hipGetLastError();
}

int32_t power_chunks(int32_t n_nets) {
  return n_nets <= 0 ? 1 : (n_nets + kPowerChunk - 1) / kPowerChunk;
}

int32_t power_partial_doubles(int32_t n_nets, int32_t B, int32_t S, int32_t paired) {
  const int64_t cols = (int64_t)B * ((S > 0 && !paired) ? S : 1);
  int64_t slabs = power_chunks(n_nets);
  if (S > 0 && !paired) slabs = std::max<int64_t>(slabs, (n_nets + kSlabNets - 1) / kSlabNets);
  return (int32_t)(slabs * cols);
}

hipError_t launch_power(const PowerArgs &a, hipStream_t s) {
  const int32_t Sp = (a.S > 0 && !a.paired) ? a.S : 1;
  const int32_t n_cols = a.B * Sp;
  if ((int64_t)a.n_nets * a.B <= 0) return hipSuccess;
  if (a.S > 0 && !a.paired && a.size) {
    if (a.mode == 1) {  // the hybrid beta first: the contraction reads it
      if (!a.beta || too_big((int64_t)a.n_nets * a.B)) return hipErrorInvalidValue;
      k_beta<<<blocks_for((int64_t)a.n_nets * a.B), kBlock, 0, s>>>(a);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    const int32_t n_slabs = (a.n_nets + kSlabNets - 1) / kSlabNets;
    const int64_t blocks = (int64_t)n_slabs * ((a.B + kTileB - 1) / kTileB) *
                           ((a.S + kTileS - 1) / kTileS);
    if (blocks > kMaxBlocks) return hipErrorInvalidValue;
    k_power_tiled<<<(unsigned)blocks, kBlock, 0, s>>>(a, n_slabs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    PowerArgs f = a;
    f.n_chunks = n_slabs;
    k_power_final<<<(unsigned)n_cols, kBlock, 0, s>>>(f, n_cols);
    return hipGetLastError();
  }
  if (a.mode == 1 && !a.beta) return hipErrorInvalidValue;
  if (a.n_chunks != power_chunks(a.n_nets)) return hipErrorInvalidValue;
  int32_t tb = 1;
  while (tb < a.B && tb < kPowerCols) tb *= 2;
  const int32_t col_tiles = (a.B + tb - 1) / tb;
  const int64_t blocks = (int64_t)kXcds * col_tiles * ((a.n_chunks + kXcds - 1) / kXcds);
  if (blocks > kMaxBlocks) return hipErrorInvalidValue;
  if (a.mode < 0 || a.mode > 2) return hipErrorInvalidValue;
  const unsigned threads = (unsigned)std::min(kPowerLanes * tb, kPowerThreads);
  using K = void (*)(PowerArgs, int32_t, int32_t);
  static const K table[3][3] = {{k_power_sp<1, 0>, k_power_sp<1, 1>, k_power_sp<1, 2>},
                                {k_power_sp<2, 0>, k_power_sp<2, 1>, k_power_sp<2, 2>},
                                {k_power_sp<4, 0>, k_power_sp<4, 1>, k_power_sp<4, 2>}};
  const K kern = table[tb == 64 ? 2 : tb == 32 ? 1 : 0][a.mode];
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(threads), 0, s, a, tb, col_tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_power_final<<<(unsigned)n_cols, kBlock, 0, s>>>(a, n_cols);
  return hipGetLastError();
}


hipError_t launch_bwd_level(const GraphView &g, const BwdArgs &a, int32_t g0, int32_t n,
                            bool cells, hipStream_t s, const int32_t *heavy, int32_t n_heavy) {
  const int64_t items = (int64_t)n * a.C;
  if (items <= 0) return hipSuccess;
  if (items >= (1ll << 31)) return hipErrorInvalidValue;
  if (cells) {
    k_bwd_level<true, false><<<level_blocks(items), kLevelBlock, 0, s>>>(g, a, g0, n, nullptr,
                                                                          0, 0);
  } else if (a.C >= kSerialColumns) {
    if (n_heavy < 0 || (n_heavy > 0 && !heavy)) return hipErrorInvalidValue;
    // 256-thread workgroups at every size: the instance holds 16 KiB of LDS
    // for its heavy-net blocks, so one-wave workgroups would leave a CU ten
    // waves (8 columns: 0.87 ms fwd+bwd against 1.18 ms at 6 with one-wave
    // groups on the 1M-gate design)
    const int64_t hb = (int64_t)n_heavy * ((a.C + 63) / 64);
    const int64_t blocks = hb + blocks_for(items);
    if (blocks > kMaxBlocks) return hipErrorInvalidValue;
    if (a.C % 64 == 0)  // one gate per wave
      k_bwd_level<false, true, true><<<(unsigned)blocks, kWideBlock, 0, s>>>(
          g, a, g0, n, heavy, n_heavy, (uint32_t)hb);
    else
      k_bwd_level<false, true><<<(unsigned)blocks, kWideBlock, 0, s>>>(
          g, a, g0, n, heavy, n_heavy, (uint32_t)hb);
  } else {
    k_bwd_level<false, false><<<level_grid(items), level_block(items), 0, s>>>(g, a, g0, n,
                                                                              nullptr, 0, 0);
  }
  return hipGetLastError();
}

hipError_t launch_bwd_pi(const GraphView &g, const BwdArgs &a, float *out, hipStream_t s,
                         const int32_t *heavy, int32_t n_heavy) {
  const int64_t items = (int64_t)g.n_pi * a.C;
  if (items <= 0) return hipSuccess;
  if (items >= (1ll << 31)) return hipErrorInvalidValue;
  if (n_heavy < 0 || (n_heavy > 0 && !heavy)) return hipErrorInvalidValue;
  if (a.C < kSerialColumns) n_heavy = 0;
  const int64_t hb = (int64_t)n_heavy * ((a.C + 63) / 64);
  const int64_t blocks = hb + blocks_for(items);
  if (blocks > kMaxBlocks) return hipErrorInvalidValue;
  k_bwd_pi<<<(unsigned)blocks, kBlock, 0, s>>>(g, a, out, heavy, n_heavy, (uint32_t)hb);
  return hipGetLastError();
}

// Blocks of a cooperative launch: enough for the widest level, at most what
// stays resident on the device.
// One block per compute unit at most (and never more than stays resident):
// the barrier's cost grows with its block count, and a wider level is
// covered by the grid-stride loop.
static hipError_t persistent_grid(const void *kernel, int64_t max_items, unsigned *grid) {
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0);
  if (e != hipSuccess) return e;
  // one block per CU at most, and no more blocks than the barrier has flags
  const int64_t resident = std::min<int64_t>({(int64_t)per_cu * ncu, ncu, kBarrierFlags});
  if (resident < 1) return hipErrorInvalidValue;
  const int64_t want = std::max<int64_t>(1, (max_items + kBlock - 1) / kBlock);
  *grid = (unsigned)std::min(resident, want);
  return hipSuccess;
}

hipError_t launch_sp_persistent(const GraphView &g, const SpLevel &lv, const int32_t *level_ptr,
                                int32_t depth, int64_t max_items, GridBarrier bar,
                                hipStream_t s) {
  if (depth <= 0) return hipSuccess;
  if (max_items >= (1ll << 31) || !bar.words) return hipErrorInvalidValue;
  unsigned grid = 0;
  hipError_t e = persistent_grid(reinterpret_cast<const void *>(&k_sp_persistent), max_items, &grid);
  if (e != hipSuccess) return e;
  k_fill_u32<<<blocks_for(kBarrierWords), kBlock, 0, s>>>(bar.words, kBarrierWords, 0u);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  GraphView gv = g;
  SpLevel l = lv;
  const int32_t *lp = level_ptr;
  int32_t d = depth;
  GridBarrier gb = bar;
  void *args[] = {&gv, &l, &lp, &d, &gb};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_sp_persistent), dim3(grid),
                                    dim3(kBlock), args, 0, s);
}

hipError_t launch_bwd_persistent(const GraphView &g, const BwdArgs &a, const int32_t *level_ptr,
                                 int32_t depth, int64_t max_items, float *pi_out,
                                 GridBarrier bar, hipStream_t s) {
  max_items = std::max<int64_t>(max_items, (int64_t)g.n_pi * a.C);
  if (max_items >= (1ll << 31) || !bar.words) return hipErrorInvalidValue;
  const void *kernel = a.C >= kSerialColumnsNoHeavy
                           ? reinterpret_cast<const void *>(&k_bwd_persistent<true>)
                           : reinterpret_cast<const void *>(&k_bwd_persistent<false>);
  unsigned grid = 0;
  hipError_t e = persistent_grid(kernel, max_items, &grid);
  if (e != hipSuccess) return e;
  k_fill_u32<<<blocks_for(kBarrierWords), kBlock, 0, s>>>(bar.words, kBarrierWords, 0u);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  GraphView gv = g;
  BwdArgs ba = a;
  const int32_t *lp = level_ptr;
  int32_t d = depth;
  float *po = pi_out;
  GridBarrier gb = bar;
  void *args[] = {&gv, &ba, &lp, &d, &po, &gb};
  return hipLaunchCooperativeKernel(kernel, dim3(grid), dim3(kBlock), args, 0, s);
}

hipError_t launch_grad_export(const GradExportArgs &a, hipStream_t s) {
  if (a.dcap && a.n_nets > 0) {
    const unsigned blocks = (unsigned)((a.n_nets + kCapRows - 1) / kCapRows);
    if (a.B < kCapRowsMinCols)
      k_grad_cap_narrow<<<blocks_for(a.n_nets), kBlock, 0, s>>>(a);
    else if (a.beta)
      k_grad_cap<true><<<blocks, kCapRows, 0, s>>>(a);
    else
      k_grad_cap<false><<<blocks, kCapRows, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.dsize && a.S > 0 && a.G > 0) {
    k_grad_size<<<blocks_for((int64_t)a.G * a.S), kBlock, 0, s>>>(a);
    return hipGetLastError();
  }
  return hipSuccess;
}

}  // namespace dp
