/*
 * DiffPower FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded and obviously correct evaluation of what the
 * GPU hot path computes: static probability (SP) propagation, toggle rate
 * (TR) under temporal independence, bit-packed logic simulation of a seeded
 * stimulus, the hybrid beta calibration, switching power and its reverse-mode
 * adjoint (DiffPower, arXiv 2608.03778, Sec. II and III).
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the HIP library: it has its
 * own netlist walk (Kahn topological order), its own gate rules, its own
 * Philox4x32-10 and its own reductions.  Everything is evaluated in
 * topological order, one gate and one cycle at a time, in double precision
 * (uint64 words for the simulation).
 *
 * Readings of the paper taken where it is silent (all listed in the design
 * notes): fixed cells use their exact single-cell probability rule; a
 * simulated word t holds cycle t of 64 independent stimulus lanes; the
 * stimulus is i.i.d. Bernoulli(p) per cycle from Philox4x32-10 with an
 * integer threshold; TR_acc is normalised per transition, 64 (T-1); beta's
 * 0/0 is 1 and x/0 is beta_max; the power terms use C_eff = C * s_driver;
 * the power-virus proxy and P_virus sum over nets, since every sink pin
 * carries its driver's value.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Opcodes of the nine fixed cells (pin order in brackets). */
enum {
  ORC_INV = 0,   /* A         : !A                */
  ORC_BUF = 1,   /* A         : A                 */
  ORC_AND2 = 2,  /* A, B      : A & B             */
  ORC_OR2 = 3,   /* A, B      : A | B             */
  ORC_NAND2 = 4, /* A, B      : !(A & B)          */
  ORC_NOR2 = 5,  /* A, B      : !(A | B)          */
  ORC_XOR2 = 6,  /* A, B      : A ^ B             */
  ORC_AOI21 = 7, /* A1, A2, B : !((A1 & A2) | B)  */
  ORC_MUX2 = 8   /* I0, I1, S : S ? I1 : I0       */
};

/* ------------------------------------------------------------------------ */
/* Library cells given as Boolean expressions (Sec. III-A, Alg. 1): each is
 * parsed (NOT binds tightest, then AND, XOR, OR), compiled in post-order to
 * a zero-address stack code, and evaluated operation by operation.  A gate
 * whose opcode is ORC_CELL_BASE + c is an instance of library cell c; its
 * inputs are the expression's identifiers in order of first appearance. */
#define ORC_CELL_BASE 16
#define ORC_MAX_IN 6
#define ORC_MAX_CODE 64
#define ORC_MAX_CELLS 240
enum { OC_IN = 0, OC_NOT = 1, OC_AND = 2, OC_OR = 3, OC_XOR = 4, OC_ZERO = 5, OC_ONE = 6 };

static int g_n_cells = 0;
static uint16_t g_code[ORC_MAX_CELLS][ORC_MAX_CODE]; /* op | arg << 8 */
static int g_len[ORC_MAX_CELLS], g_nin[ORC_MAX_CELLS];

/* recursive-descent parser over a NUL-terminated expression */
typedef struct {
  const char *s;
  int pos, n_ids, len, err;
  char ids[ORC_MAX_IN][32];
  uint16_t *code;
} orc_parser;

static void ps_skip(orc_parser *ps) {
  while (ps->s[ps->pos] == ' ' || ps->s[ps->pos] == '\t') ps->pos++;
}
static void ps_emit(orc_parser *ps, int op, int arg) {
  if (ps->len >= ORC_MAX_CODE) { ps->err = 1; return; }
  ps->code[ps->len++] = (uint16_t)(op | (arg << 8));
}
static int is_id0(char c) { return (c >= 'A' && c <= 'Z') || (c >= 'a' && c <= 'z') || c == '_'; }
static int is_id(char c) { return is_id0(c) || (c >= '0' && c <= '9'); }
static void ps_or(orc_parser *ps);
static void ps_unary(orc_parser *ps) {
  ps_skip(ps);
  char c = ps->s[ps->pos];
  if (c == '!' || c == '~') {
    ps->pos++;
    ps_unary(ps);
    ps_emit(ps, OC_NOT, 0);
  } else if (c == '(') {
    ps->pos++;
    ps_or(ps);
    ps_skip(ps);
    if (ps->s[ps->pos] != ')') { ps->err = 1; return; }
    ps->pos++;
  } else if (c == '0' || c == '1') {
    ps->pos++;
    ps_emit(ps, c == '0' ? OC_ZERO : OC_ONE, 0);
  } else if (is_id0(c)) {
    char name[32];
    int n = 0;
    while (is_id(ps->s[ps->pos]) && n < 31) name[n++] = ps->s[ps->pos++];
    name[n] = 0;
    if (is_id(ps->s[ps->pos])) { ps->err = 1; return; }
    int k = 0;
    while (k < ps->n_ids && strcmp(ps->ids[k], name) != 0) ++k;
    if (k == ps->n_ids) {
      if (ps->n_ids == ORC_MAX_IN) { ps->err = 1; return; }
      strcpy(ps->ids[ps->n_ids++], name);
    }
    ps_emit(ps, OC_IN, k);
  } else {
    ps->err = 1;
  }
}
static void ps_and(orc_parser *ps) {
  ps_unary(ps);
  for (;;) {
    ps_skip(ps);
    char c = ps->s[ps->pos];
    if (ps->err || (c != '&' && c != '*')) return;
    ps->pos++;
    ps_unary(ps);
    ps_emit(ps, OC_AND, 0);
  }
}
static void ps_xor(orc_parser *ps) {
  ps_and(ps);
  for (;;) {
    ps_skip(ps);
    if (ps->err || ps->s[ps->pos] != '^') return;
    ps->pos++;
    ps_and(ps);
    ps_emit(ps, OC_XOR, 0);
  }
}
static void ps_or(orc_parser *ps) {
  ps_xor(ps);
  for (;;) {
    ps_skip(ps);
    char c = ps->s[ps->pos];
    if (ps->err || (c != '|' && c != '+')) return;
    ps->pos++;
    ps_xor(ps);
    ps_emit(ps, OC_OR, 0);
  }
}

/* Compile one expression; returns the code length, or -1 on a syntax error
 * (or more than ORC_MAX_IN inputs / ORC_MAX_CODE instructions). */
int orc_cell_compile(const char *expr, uint16_t *code, int *n_inputs) {
  orc_parser ps;
  memset(&ps, 0, sizeof ps);
  ps.s = expr;
  ps.code = code;
  ps_or(&ps);
  ps_skip(&ps);
  if (ps.err || ps.s[ps.pos] != 0 || ps.len == 0) return -1;
  *n_inputs = ps.n_ids;
  return ps.len;
}

/* Register the cell library for later calls: 0, or -(1 + c) if cell c does
 * not compile. */
int orc_set_cells(int n_cells, const char *const *exprs) {
  if (n_cells < 0 || n_cells > ORC_MAX_CELLS) return -1;
  for (int c = 0; c < n_cells; ++c) {
    int n = orc_cell_compile(exprs[c], g_code[c], &g_nin[c]);
    if (n < 0) return -(1 + c);
    g_len[c] = n;
  }
  g_n_cells = n_cells;
  return 0;
}

/* Op-by-op probability of a cell's code (each operation applies its
 * independent-input rule to its operands). */
static double cell_sp(int c, const double *x) {
  double st[ORC_MAX_CODE];
  int top = 0;
  for (int i = 0; i < g_len[c]; ++i) {
    int op = g_code[c][i] & 0xff, arg = g_code[c][i] >> 8;
    double a, b;
    switch (op) {
      case OC_IN: st[top++] = x[arg]; break;
      case OC_ZERO: st[top++] = 0.0; break;
      case OC_ONE: st[top++] = 1.0; break;
      case OC_NOT: st[top - 1] = 1.0 - st[top - 1]; break;
      default:
        b = st[--top];
        a = st[--top];
        st[top++] = op == OC_AND ? a * b : (op == OC_OR ? a + b - a * b : a + b - 2.0 * a * b);
    }
  }
  return st[0];
}

static double complex cell_sp_c(int c, const double complex *x) {
  double complex st[ORC_MAX_CODE];
  int top = 0;
  for (int i = 0; i < g_len[c]; ++i) {
    int op = g_code[c][i] & 0xff, arg = g_code[c][i] >> 8;
    double complex a, b;
    switch (op) {
      case OC_IN: st[top++] = x[arg]; break;
      case OC_ZERO: st[top++] = 0.0; break;
      case OC_ONE: st[top++] = 1.0; break;
      case OC_NOT: st[top - 1] = 1.0 - st[top - 1]; break;
      default:
        b = st[--top];
        a = st[--top];
        st[top++] = op == OC_AND ? a * b : (op == OC_OR ? a + b - a * b : a + b - 2.0 * a * b);
    }
  }
  return st[0];
}

/* Partial derivatives of cell_sp with respect to each input (Sec. III-E),
 * by forward-mode differentiation: for input k the code is evaluated on
 * (value, derivative with respect to x_k) pairs, each operation applying
 * the chain rule to its independent-operand rule:
 *   NOT  1 - a        ->  -a'
 *   AND  a b          ->  a' b + a b'
 *   OR   a + b - a b  ->  a' + b' - (a' b + a b')
 *   XOR  a + b - 2ab  ->  a' + b' - 2 (a' b + a b')
 * an input contributes 1 for x_k and 0 otherwise, a constant 0. */
static void cell_partials(int c, const double *x, double *d) {
  for (int k = 0; k < g_nin[c]; ++k) {
    double v[ORC_MAX_CODE], dv[ORC_MAX_CODE];
    int top = 0;
    for (int i = 0; i < g_len[c]; ++i) {
      int op = g_code[c][i] & 0xff, arg = g_code[c][i] >> 8;
      if (op == OC_IN || op == OC_ZERO || op == OC_ONE) {
        v[top] = op == OC_IN ? x[arg] : (op == OC_ONE ? 1.0 : 0.0);
        dv[top] = (op == OC_IN && arg == k) ? 1.0 : 0.0;
        ++top;
      } else if (op == OC_NOT) {
        v[top - 1] = 1.0 - v[top - 1];
        dv[top - 1] = -dv[top - 1];
      } else {
        --top;
        double b = v[top], db = dv[top];
        --top;
        double a = v[top], da = dv[top];
        double prod = da * b + a * db;
        if (op == OC_AND) {
          v[top] = a * b;
          dv[top] = prod;
        } else if (op == OC_OR) {
          v[top] = a + b - a * b;
          dv[top] = da + db - prod;
        } else {
          v[top] = a + b - 2.0 * a * b;
          dv[top] = da + db - 2.0 * prod;
        }
        ++top;
      }
    }
    d[k] = dv[0];
  }
}

static uint64_t cell_bits(int c, const uint64_t *w) {
  uint64_t st[ORC_MAX_CODE];
  int top = 0;
  for (int i = 0; i < g_len[c]; ++i) {
    int op = g_code[c][i] & 0xff, arg = g_code[c][i] >> 8;
    uint64_t a, b;
    switch (op) {
      case OC_IN: st[top++] = w[arg]; break;
      case OC_ZERO: st[top++] = 0; break;
      case OC_ONE: st[top++] = ~0ull; break;
      case OC_NOT: st[top - 1] = ~st[top - 1]; break;
      default:
        b = st[--top];
        a = st[--top];
        st[top++] = op == OC_AND ? (a & b) : (op == OC_OR ? (a | b) : (a ^ b));
    }
  }
  return st[0];
}

static const int orc_arity[9] = {1, 1, 2, 2, 2, 2, 2, 3, 3};

int orc_op_arity(int op) {
  if (op >= 0 && op < 9) return orc_arity[op];
  if (op >= ORC_CELL_BASE && op - ORC_CELL_BASE < g_n_cells) return g_nin[op - ORC_CELL_BASE];
  return -1;
}

/* ------------------------------------------------------------------------ */
/* Netlist check and topological order (Sec. III-A: the graph is levelized so
 * that a node depends only on nodes of lower levels; any topological order
 * gives the same values).  Returns 0, -1 for a malformed netlist, -2 for a
 * combinational cycle. */
int orc_topo_order(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                   const int32_t *fanin_ptr, const int32_t *fanin,
                   int32_t *order) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  if (n_pi < 0 || n_gates < 0 || fanin_ptr[0] != 0) return -1;
  for (int32_t g = 0; g < n_gates; ++g) {
    if (orc_op_arity(op[g]) < 0) return -1;
    if (fanin_ptr[g + 1] - fanin_ptr[g] != orc_op_arity(op[g])) return -1;
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
      if (fanin[e] < 0 || fanin[e] >= n_nets) return -1;
  }
  /* indeg[g] = number of input pins of g driven by a gate */
  int32_t *indeg = calloc((size_t)n_gates + 1, sizeof(int32_t));
  int32_t *cnt = calloc((size_t)n_gates + 1, sizeof(int32_t));
  int32_t *cptr = calloc((size_t)n_gates + 2, sizeof(int32_t));
  int32_t n_edges = fanin_ptr[n_gates];
  int32_t *cons = malloc(sizeof(int32_t) * ((size_t)n_edges + 1));
  for (int32_t g = 0; g < n_gates; ++g)
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
      if (fanin[e] >= n_pi) {
        indeg[g]++;
        cnt[fanin[e] - n_pi]++;
      }
  for (int32_t d = 0; d < n_gates; ++d) cptr[d + 1] = cptr[d] + cnt[d];
  memset(cnt, 0, sizeof(int32_t) * ((size_t)n_gates + 1));
  for (int32_t g = 0; g < n_gates; ++g)
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
      if (fanin[e] >= n_pi) {
        int32_t d = fanin[e] - n_pi;
        cons[cptr[d] + cnt[d]++] = g;
      }
  int32_t head = 0, tail = 0;
  for (int32_t g = 0; g < n_gates; ++g)
    if (indeg[g] == 0) order[tail++] = g;
  while (head < tail) {
    int32_t d = order[head++];
    for (int32_t c = cptr[d]; c < cptr[d + 1]; ++c)
      if (--indeg[cons[c]] == 0) order[tail++] = cons[c];
  }
  free(indeg);
  free(cnt);
  free(cptr);
  free(cons);
  return tail == n_gates ? 0 : -2;
}

/* Level of every net: PIs 0, a gate one more than its deepest input. */
void orc_levels(int32_t n_pi, int32_t n_gates, const int32_t *fanin_ptr,
                const int32_t *fanin, const int32_t *order, int32_t *level) {
  for (int32_t i = 0; i < n_pi; ++i) level[i] = 0;
  for (int32_t k = 0; k < n_gates; ++k) {
    int32_t g = order[k], l = 0;
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
      if (level[fanin[e]] > l) l = level[fanin[e]];
    level[n_pi + g] = l + 1;
  }
}

/* ------------------------------------------------------------------------ */
/* Gate probability rules.  Under the independence assumption of Sec. II-B
 * the probability that a gate output is 1 is the sum, over the input
 * minterms that make the output 1, of the product of the input
 * probabilities; for these read-once cells that sum collapses to the closed
 * forms below (the paper gives AND = a0 a1 and NAND = 1 - a0 a1 as examples
 * in Alg. 2, and the OR/XOR/NOT forms in Sec. III-E). */
static double sp_rule(int op, const double *x) {
  if (op >= ORC_CELL_BASE) return cell_sp(op - ORC_CELL_BASE, x);
  switch (op) {
    case ORC_INV: return 1.0 - x[0];
    case ORC_BUF: return x[0];
    case ORC_AND2: return x[0] * x[1];
    case ORC_OR2: return 1.0 - (1.0 - x[0]) * (1.0 - x[1]);
    case ORC_NAND2: return 1.0 - x[0] * x[1];
    case ORC_NOR2: return (1.0 - x[0]) * (1.0 - x[1]);
    case ORC_XOR2: return x[0] + x[1] - 2.0 * x[0] * x[1];
    case ORC_AOI21: return (1.0 - x[0] * x[1]) * (1.0 - x[2]);
    case ORC_MUX2: return (1.0 - x[2]) * x[0] + x[2] * x[1];
  }
  return 0.0;
}

/* Partial derivatives of sp_rule with respect to each input (Sec. III-E:
 * d(ab)/da = b, d(OR)/da = 1-b, d(XOR)/da = 1-2b, d(NOT)/dx = -1; the
 * compound cells follow by the product rule). */
static void sp_partials(int op, const double *x, double *d) {
  if (op >= ORC_CELL_BASE) {
    cell_partials(op - ORC_CELL_BASE, x, d);
    return;
  }
  switch (op) {
    case ORC_INV: d[0] = -1.0; break;
    case ORC_BUF: d[0] = 1.0; break;
    case ORC_AND2: d[0] = x[1]; d[1] = x[0]; break;
    case ORC_OR2: d[0] = 1.0 - x[1]; d[1] = 1.0 - x[0]; break;
    case ORC_NAND2: d[0] = -x[1]; d[1] = -x[0]; break;
    case ORC_NOR2: d[0] = -(1.0 - x[1]); d[1] = -(1.0 - x[0]); break;
    case ORC_XOR2: d[0] = 1.0 - 2.0 * x[1]; d[1] = 1.0 - 2.0 * x[0]; break;
    case ORC_AOI21:
      d[0] = -x[1] * (1.0 - x[2]);
      d[1] = -x[0] * (1.0 - x[2]);
      d[2] = -(1.0 - x[0] * x[1]);
      break;
    case ORC_MUX2: d[0] = 1.0 - x[2]; d[1] = x[2]; d[2] = x[1] - x[0]; break;
  }
}

/* Boolean function of each cell on 64 parallel lanes (Sec. III-C). */
static uint64_t bit_rule(int op, const uint64_t *w) {
  if (op >= ORC_CELL_BASE) return cell_bits(op - ORC_CELL_BASE, w);
  switch (op) {
    case ORC_INV: return ~w[0];
    case ORC_BUF: return w[0];
    case ORC_AND2: return w[0] & w[1];
    case ORC_OR2: return w[0] | w[1];
    case ORC_NAND2: return ~(w[0] & w[1]);
    case ORC_NOR2: return ~(w[0] | w[1]);
    case ORC_XOR2: return w[0] ^ w[1];
    case ORC_AOI21: return ~((w[0] & w[1]) | w[2]);
    case ORC_MUX2: return (w[0] & ~w[2]) | (w[1] & w[2]);
  }
  return 0;
}

static double clamp01(double v) { return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v); }

/* Exported single-gate rules, for tests that enumerate truth tables (a
 * library cell's opcode is ORC_CELL_BASE + its index). */
double orc_gate_sp(int op, const double *x) { return sp_rule(op, x); }
void orc_gate_partials(int op, const double *x, double *d) { sp_partials(op, x, d); }
uint64_t orc_gate_bits(int op, const uint64_t *w) { return bit_rule(op, w); }

/* ------------------------------------------------------------------------ */
/* Pass 1 (Sec. III-B, Alg. 2): P of every net.  PIs take the given
 * probabilities (the callers promote float32 inputs exactly); each gate, in
 * topological order, gathers its input probabilities, applies its rule and
 * clips to [0, 1]. */
void orc_sp(int32_t n_pi, int32_t n_gates, const uint8_t *op,
            const int32_t *fanin_ptr, const int32_t *fanin,
            const int32_t *order, const double *p_pi, double *P) {
  for (int32_t i = 0; i < n_pi; ++i) P[i] = p_pi[i];
  for (int32_t k = 0; k < n_gates; ++k) {
    int32_t g = order[k];
    double x[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
      x[e - fanin_ptr[g]] = P[fanin[e]];
    P[n_pi + g] = clamp01(sp_rule(op[g], x));
  }
}

/* Same propagation with the PI probabilities given in double precision and
 * one PI shifted by a complex step i*h: every rule is a polynomial, so
 * Im(F(p + i h e_k)) / h is the derivative of F with respect to p_k with no
 * subtractive cancellation.  Used only to check the adjoint. */
static double complex sp_rule_c(int op, const double complex *x) {
  if (op >= ORC_CELL_BASE) return cell_sp_c(op - ORC_CELL_BASE, x);
  switch (op) {
    case ORC_INV: return 1.0 - x[0];
    case ORC_BUF: return x[0];
    case ORC_AND2: return x[0] * x[1];
    case ORC_OR2: return 1.0 - (1.0 - x[0]) * (1.0 - x[1]);
    case ORC_NAND2: return 1.0 - x[0] * x[1];
    case ORC_NOR2: return (1.0 - x[0]) * (1.0 - x[1]);
    case ORC_XOR2: return x[0] + x[1] - 2.0 * x[0] * x[1];
    case ORC_AOI21: return (1.0 - x[0] * x[1]) * (1.0 - x[2]);
    case ORC_MUX2: return (1.0 - x[2]) * x[0] + x[2] * x[1];
  }
  return 0.0;
}

/* Complex-step derivative of modeled power sum_n k*beta_n*Ceff_n*2P(1-P)
 * with respect to PI `pi`, beta given (frozen). */
double orc_power_complex_step(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                              const int32_t *fanin_ptr, const int32_t *fanin,
                              const int32_t *order, const double *p_pi,
                              const double *beta, const double *ceff,
                              double kappa, int32_t pi, double h) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  double complex *P = malloc(sizeof(double complex) * (size_t)n_nets);
  for (int32_t i = 0; i < n_pi; ++i) P[i] = p_pi[i] + (i == pi ? I * h : 0.0);
  for (int32_t k = 0; k < n_gates; ++k) {
    int32_t g = order[k];
    double complex x[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
      x[e - fanin_ptr[g]] = P[fanin[e]];
    P[n_pi + g] = sp_rule_c(op[g], x); /* values stay inside [0,1]: no clip */
  }
  double complex s = 0.0;
  for (int64_t n = 0; n < n_nets; ++n)
    s += kappa * beta[n] * ceff[n] * 2.0 * P[n] * (1.0 - P[n]);
  free(P);
  return cimag(s) / h;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror and Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11).  One round maps
 * (c0, c1, c2, c3) with key (k0, k1) to
 *   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
 * with M0 = 0xD2511F53 and M1 = 0xCD9E8D57; the key is bumped by the Weyl
 * constants (0x9E3779B9, 0xBB67AE85) between rounds; ten rounds. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Integer threshold of a float32 probability: floor(p * 2^32), exact because
 * a float32 times a power of two is exact in double; p = 1 gives 2^32. */
uint64_t orc_threshold(float p) {
  double v = (double)p * 4294967296.0;
  if (!(v > 0.0)) return 0;
  if (v >= 4294967296.0) return 4294967296ull;
  return (uint64_t)floor(v);
}

/* Stimulus (Sec. III-C: 64-bit input words from Markov chains calibrated to a
 * target SP and TR).  With the target TR of the temporal-independence model,
 * 2p(1-p), the chain's 0->1 probability is p and its 1->0 probability is
 * 1-p, i.e. every cycle is an independent Bernoulli(p) draw.  Bit j of word t
 * of PI i is 1 iff u < floor(p_i 2^32), with u lane (j mod 4) of
 * Philox4x32-10(counter = (t, i, j div 4, 0), key = (seed lo, seed hi)). */
uint64_t orc_stimulus_word(int32_t pi, int64_t t, float p, uint64_t seed) {
  uint64_t thr = orc_threshold(p);
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint64_t w = 0;
  for (int q = 0; q < 16; ++q) {
    uint32_t ctr[4] = {(uint32_t)t, (uint32_t)pi, (uint32_t)q, 0u};
    uint32_t u[4];
    orc_philox4x32_10(ctr, key, u);
    for (int l = 0; l < 4; ++l)
      if ((uint64_t)u[l] < thr) w |= (uint64_t)1 << (4 * q + l);
  }
  return w;
}

/* Words [t0, t0 + n_words) of every PI, laid out [n_pi][n_words]. */
void orc_stimulus(int32_t n_pi, const float *p_pi, uint64_t seed, int64_t t0,
                  int64_t n_words, uint64_t *words) {
  for (int32_t i = 0; i < n_pi; ++i)
    for (int64_t t = 0; t < n_words; ++t)
      words[(int64_t)i * n_words + t] = orc_stimulus_word(i, t0 + t, p_pi[i], seed);
}

/* Integer threshold of a double probability: floor(x 2^32), 0 below 0 and
 * 2^32 from 1 up (x 2^32 is exact; floor then rounds down). */
uint64_t orc_threshold_d(double x) {
  double v = x * 4294967296.0;
  if (!(v > 0.0)) return 0;
  if (v >= 4294967296.0) return 4294967296ull;
  return (uint64_t)floor(v);
}

/* The chain of a startpoint with stationary probability p and target
 * transition rate tau (Sec. III-C): a two-state Markov chain whose
 * stationary law is Bernoulli(p) and whose probability of a change per cycle
 * is tau, so P(0 -> 1) = a = tau / (2 (1 - p)) and P(1 -> 0) = b =
 * tau / (2 p).  Returned as the rise probability a and the stay-at-one
 * probability 1 - b, clamped into [0, 1] (tau beyond 2 min(p, 1 - p) gives
 * the fastest chain there is); p = 0 never leaves 0 and p = 1 never leaves 1.
 * With tau = 2 p (1 - p) both equal p: every cycle is then an independent
 * Bernoulli(p) draw, the temporal-independence model. */
void orc_markov_probs(float p, float tau, double *rise, double *stay) {
  double pd = (double)p, td = (double)tau, a, st;
  if (pd <= 0.0) {
    a = 0.0;
    st = 0.0;
  } else if (pd >= 1.0) {
    a = 1.0;
    st = 1.0;
  } else {
    a = td / (2.0 * (1.0 - pd));
    st = 1.0 - td / (2.0 * pd);
  }
  if (a > 1.0) a = 1.0;
  if (st < 0.0) st = 0.0;
  *rise = a;
  *stay = st;
}

/* Startpoint stimulus with a target transition rate and shared streams
 * (Sec. III-C).  Startpoint i draws its uniforms from stream s_i = stream[i]
 * (i when stream is NULL), so startpoints that share a stream and a
 * (p, tau) get the same words: u(t, j) is lane (j mod 4) of
 * Philox4x32-10(counter = (t, s_i, j div 4, 0), key = (seed lo, seed hi)).
 * Lane j of startpoint i is its own chain: at cycle 0 it is 1 iff
 * u(0, j) < floor(p_i 2^32) (the stationary law, the same bit as the
 * independent stimulus); at cycle t >= 1 a lane at 1 stays at 1 iff
 * u(t, j) < floor((1 - b) 2^32) and a lane at 0 rises iff
 * u(t, j) < floor(a 2^32).  tau == NULL: every cycle draws like cycle 0
 * (independent cycles).  Words [n_pi][T]. */
void orc_stimulus_model(int32_t n_pi, const float *p_pi, const float *tau,
                        const int32_t *stream, uint64_t seed, int64_t T,
                        uint64_t *words) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int32_t i = 0; i < n_pi; ++i) {
    uint32_t si = stream ? (uint32_t)stream[i] : (uint32_t)i;
    uint64_t thr_p = orc_threshold(p_pi[i]);
    uint64_t thr_rise = thr_p, thr_stay = thr_p;
    if (tau) {
      double a, st;
      orc_markov_probs(p_pi[i], tau[i], &a, &st);
      thr_rise = orc_threshold_d(a);
      thr_stay = orc_threshold_d(st);
    }
    uint64_t prev = 0;
    for (int64_t t = 0; t < T; ++t) {
      uint64_t w = 0;
      for (int q = 0; q < 16; ++q) {
        uint32_t ctr[4] = {(uint32_t)t, si, (uint32_t)q, 0u};
        uint32_t u[4];
        orc_philox4x32_10(ctr, key, u);
        for (int l = 0; l < 4; ++l) {
          int j = 4 * q + l;
          uint64_t thr;
          if (t == 0) thr = thr_p;
          else thr = ((prev >> j) & 1u) ? thr_stay : thr_rise;
          if ((uint64_t)u[l] < thr) w |= (uint64_t)1 << j;
        }
      }
      words[(int64_t)i * T + t] = w;
      prev = w;
    }
  }
}

static int popcount64(uint64_t x) {
  int c = 0;
  while (x) {
    x &= x - 1;
    ++c;
  }
  return c;
}

/* Pass 2 (Sec. III-C): cycle-by-cycle bit-parallel simulation of T words.
 * For each cycle t every PI takes its stimulus word, every gate (in
 * topological order) evaluates its Boolean function on its input words;
 * ones[n] adds popcount(w_n(t)) and, for t >= 1, toggles[n] adds
 * popcount(w_n(t) ^ w_n(t-1)).  The stimulus is read from `pi_words`
 * ([n_pi][T]) when given, otherwise generated from (p_pi, seed). */
/* Counts restricted to the cycles [t_begin, t_end): ones over those cycles,
 * toggles for the transitions into them (cycle t_begin - 1 is simulated
 * too when t_begin > 0).  Counts of disjoint ranges add up to the counts of
 * their union.  Generated stimulus only. */
void orc_sim_range(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                   const int32_t *fanin_ptr, const int32_t *fanin,
                   const int32_t *order, int64_t t_begin, int64_t t_end,
                   const float *p_pi, uint64_t seed, uint64_t *ones,
                   uint64_t *toggles);

void orc_sim(int32_t n_pi, int32_t n_gates, const uint8_t *op,
             const int32_t *fanin_ptr, const int32_t *fanin,
             const int32_t *order, int64_t T, const uint64_t *pi_words,
             const float *p_pi, uint64_t seed, uint64_t *ones,
             uint64_t *toggles) {
  if (!pi_words) {
    orc_sim_range(n_pi, n_gates, op, fanin_ptr, fanin, order, 0, T, p_pi, seed,
                  ones, toggles);
    return;
  }
  int64_t n_nets = (int64_t)n_pi + n_gates;
  uint64_t *cur = calloc((size_t)n_nets, sizeof(uint64_t));
  uint64_t *prev = calloc((size_t)n_nets, sizeof(uint64_t));
  for (int64_t n = 0; n < n_nets; ++n) ones[n] = toggles[n] = 0;
  for (int64_t t = 0; t < T; ++t) {
    for (int32_t i = 0; i < n_pi; ++i) cur[i] = pi_words[(int64_t)i * T + t];
    for (int32_t k = 0; k < n_gates; ++k) {
      int32_t g = order[k];
      uint64_t w[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
      for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
        w[e - fanin_ptr[g]] = cur[fanin[e]];
      cur[n_pi + g] = bit_rule(op[g], w);
    }
    for (int64_t n = 0; n < n_nets; ++n) {
      ones[n] += (uint64_t)popcount64(cur[n]);
      if (t > 0) toggles[n] += (uint64_t)popcount64(cur[n] ^ prev[n]);
    }
    uint64_t *tmp = prev;
    prev = cur;
    cur = tmp;
  }
  free(cur);
  free(prev);
}

void orc_sim_range(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                   const int32_t *fanin_ptr, const int32_t *fanin,
                   const int32_t *order, int64_t t_begin, int64_t t_end,
                   const float *p_pi, uint64_t seed, uint64_t *ones,
                   uint64_t *toggles) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  uint64_t *cur = calloc((size_t)n_nets, sizeof(uint64_t));
  uint64_t *prev = calloc((size_t)n_nets, sizeof(uint64_t));
  for (int64_t n = 0; n < n_nets; ++n) ones[n] = toggles[n] = 0;
  int64_t t_first = t_begin > 0 ? t_begin - 1 : 0;
  for (int64_t t = t_first; t < t_end; ++t) {
    for (int32_t i = 0; i < n_pi; ++i) cur[i] = orc_stimulus_word(i, t, p_pi[i], seed);
    for (int32_t k = 0; k < n_gates; ++k) {
      int32_t g = order[k];
      uint64_t w[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
      for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
        w[e - fanin_ptr[g]] = cur[fanin[e]];
      cur[n_pi + g] = bit_rule(op[g], w);
    }
    for (int64_t n = 0; n < n_nets; ++n) {
      if (t >= t_begin) ones[n] += (uint64_t)popcount64(cur[n]);
      if (t > t_first) toggles[n] += (uint64_t)popcount64(cur[n] ^ prev[n]);
    }
    uint64_t *tmp = prev;
    prev = cur;
    cur = tmp;
  }
  free(cur);
  free(prev);
}

/* ------------------------------------------------------------------------ */
/* Activity, beta and power.
 *   TR_model = 2P(1-P)                                   (Eq. 2)
 *   SP_acc = ones / (64 T), TR_acc = toggles / (64 (T-1)) (Eq. 4, per transition)
 *   beta = clip(TR_acc / TR_model, beta_min, beta_max)   (Eq. 5), 1 when modeled
 *   TR_hyb = beta * TR_model
 *   C_eff = C * s_driver (s = 1 for PIs and when no sizes are given)
 *   P_sw = kappa * sum_n beta_n * C_eff,n * TR_model,n,  kappa = ef * Vdd^2 * f (Eq. 1)
 * hybrid = 0 gives the modeled pipeline.  `beta_in`, when given, replaces the
 * computed beta (a frozen calibration).  Output arrays may be NULL. */
double orc_power(int32_t n_pi, int32_t n_gates, const double *P,
                 const uint64_t *ones, const uint64_t *toggles, int64_t T,
                 const float *cap, const float *size, double kappa, int hybrid,
                 double beta_min, double beta_max, const double *beta_in,
                 double *tr_model, double *sp_acc, double *tr_acc,
                 double *beta_out, double *tr_hyb, double *ceff_out) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  double total = 0.0;
  for (int64_t n = 0; n < n_nets; ++n) {
    double tm = 2.0 * P[n] * (1.0 - P[n]);
    double b = 1.0, sa = 0.0, ta = 0.0;
    if (hybrid) {
      sa = (double)ones[n] / (64.0 * (double)T);
      ta = (double)toggles[n] / (64.0 * (double)(T - 1));
      if (tm == 0.0)
        b = (ta == 0.0) ? 1.0 : beta_max;
      else
        b = ta / tm;
      if (b < beta_min) b = beta_min;
      if (b > beta_max) b = beta_max;
    }
    if (beta_in) b = beta_in[n];
    double s = (size && n >= n_pi) ? (double)size[n - n_pi] : 1.0;
    double ce = (double)cap[n] * s;
    total += kappa * b * ce * tm;
    if (tr_model) tr_model[n] = tm;
    if (sp_acc) sp_acc[n] = sa;
    if (tr_acc) tr_acc[n] = ta;
    if (beta_out) beta_out[n] = b;
    if (tr_hyb) tr_hyb[n] = b * tm;
    if (ceff_out) ceff_out[n] = ce;
  }
  return total;
}

/* ------------------------------------------------------------------------ */
/* Reverse-mode adjoint (Sec. III-E, Eq. 7): with beta, C, s and the stimulus
 * held fixed,
 *   lambda_n = local_n + sum over the gates j reading n of lambda_out(j) *
 *              dR_j/dx_pin,
 *   local_n  = kappa * beta_n * C_eff,n * 2 (1 - 2 P_n)   (d TR_model / dP)
 * evaluated in reverse topological order.  The clip of Alg. 2 passes the
 * gradient straight through.  beta_ste = 1 applies Eq. 6 literally instead:
 * lambda_n = beta_n * (sum over readers + kappa * C_eff,n * 2 (1 - 2 P_n)).
 * Outputs: lambda [n_nets]; dP/dC_n = kappa beta_n s_drv(n) TR_model,n;
 * dP/ds_g = kappa beta_out C_out TR_model,out (arrays may be NULL). */
void orc_adjoint(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                 const int32_t *fanin_ptr, const int32_t *fanin,
                 const int32_t *order, const double *P, const double *beta,
                 const float *cap, const float *size, double kappa,
                 int beta_ste, double *lambda, double *dcap, double *dsize) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  double *acc = calloc((size_t)n_nets, sizeof(double));
  for (int64_t n = 0; n < n_nets; ++n) acc[n] = 0.0;
  for (int32_t k = n_gates - 1; k >= -n_pi; --k) {
    /* visit gates in reverse topological order, then the PIs */
    int64_t n = (k >= 0) ? (int64_t)n_pi + order[k] : (int64_t)(-k - 1);
    double s = (n >= n_pi && size) ? (double)size[n - n_pi] : 1.0;
    double ce = (double)cap[n] * s;
    double lam;
    if (beta_ste)
      lam = beta[n] * (acc[n] + kappa * ce * 2.0 * (1.0 - 2.0 * P[n]));
    else
      lam = acc[n] + kappa * beta[n] * ce * 2.0 * (1.0 - 2.0 * P[n]);
    lambda[n] = lam;
    if (n >= n_pi) {
      int32_t g = (int32_t)(n - n_pi);
      double x[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0}, d[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
      for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
        x[e - fanin_ptr[g]] = P[fanin[e]];
      sp_partials(op[g], x, d);
      for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e)
        acc[fanin[e]] += lam * d[e - fanin_ptr[g]];
    }
  }
  for (int64_t n = 0; n < n_nets; ++n) {
    double s = (n >= n_pi && size) ? (double)size[n - n_pi] : 1.0;
    double tm = 2.0 * P[n] * (1.0 - P[n]);
    if (dcap) dcap[n] = kappa * beta[n] * s * tm;
    if (dsize && n >= n_pi) dsize[n - n_pi] = kappa * beta[n] * (double)cap[n] * tm;
  }
  free(acc);
}

/* ------------------------------------------------------------------------ */
/* Power virus by gradient ascent (Sec. IV-B, Alg. 4).
 * The startpoint SPs p [n_pi] (in/out) are ascended `steps` times on the
 * proxy of Eq. 9 at net level (a sink pin carries its driver's value),
 *   P_proxy = sum_n beta_n * C_n * 2 P_n (1 - P_n),
 * whose gradient is the adjoint of orc_adjoint with kappa = 1 and the frozen
 * beta (beta = NULL means 1):  p_i <- clip(p_i + eta * dP_proxy/dp_i, 0, 1).
 * Then v0_i = [p_i >= 1/2], v1_i = 1 - v0_i, and the transition-weighted
 * power of Eq. 3 at net level,
 *   P_virus = sum_n C_n * [value of net n under v0 != value under v1],
 * is returned (v0 [n_pi] out). */
double orc_virus_power(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                       const int32_t *fanin_ptr, const int32_t *fanin,
                       const int32_t *order, const float *cap, const uint8_t *v0) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  uint64_t *w0 = calloc((size_t)n_nets, sizeof(uint64_t));
  uint64_t *w1 = calloc((size_t)n_nets, sizeof(uint64_t));
  for (int32_t i = 0; i < n_pi; ++i) {
    w0[i] = v0[i] ? ~0ull : 0ull;
    w1[i] = ~w0[i];
  }
  for (int32_t k = 0; k < n_gates; ++k) {
    int32_t g = order[k];
    uint64_t a0[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0}, a1[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e) {
      a0[e - fanin_ptr[g]] = w0[fanin[e]];
      a1[e - fanin_ptr[g]] = w1[fanin[e]];
    }
    w0[n_pi + g] = bit_rule(op[g], a0);
    w1[n_pi + g] = bit_rule(op[g], a1);
  }
  double total = 0.0;
  for (int64_t n = 0; n < n_nets; ++n)
    if ((w0[n] & 1ull) != (w1[n] & 1ull)) total += (double)cap[n];
  free(w0);
  free(w1);
  return total;
}

double orc_power_virus(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                       const int32_t *fanin_ptr, const int32_t *fanin,
                       const int32_t *order, const float *cap, const double *beta,
                       int32_t steps, double eta, double *p, uint8_t *v0) {
  int64_t n_nets = (int64_t)n_pi + n_gates;
  double *P = calloc((size_t)n_nets, sizeof(double));
  double *b = calloc((size_t)n_nets, sizeof(double));
  double *lam = calloc((size_t)n_nets, sizeof(double));
  for (int64_t n = 0; n < n_nets; ++n) b[n] = beta ? beta[n] : 1.0;
  for (int32_t t = 0; t < steps; ++t) {
    orc_sp(n_pi, n_gates, op, fanin_ptr, fanin, order, p, P);
    orc_adjoint(n_pi, n_gates, op, fanin_ptr, fanin, order, P, b, cap, NULL, 1.0, 0, lam,
                NULL, NULL);
    for (int32_t i = 0; i < n_pi; ++i) p[i] = clamp01(p[i] + eta * lam[i]);
  }
  for (int32_t i = 0; i < n_pi; ++i) v0[i] = p[i] >= 0.5 ? 1 : 0;
  free(P);
  free(b);
  free(lam);
  return orc_virus_power(n_pi, n_gates, op, fanin_ptr, fanin, order, cap, v0);
}

/* ------------------------------------------------------------------------ */
/* SP with one net overridden: P[net] += delta after its own rule, and the
 * change propagates to everything downstream (a hook for finite
 * differences of the adjoint of an internal net). */
void orc_sp_override(int32_t n_pi, int32_t n_gates, const uint8_t *op,
                     const int32_t *fanin_ptr, const int32_t *fanin,
                     const int32_t *order, const double *p_pi, int64_t net,
                     double delta, double *P) {
  for (int32_t i = 0; i < n_pi; ++i) P[i] = p_pi[i];
  if (net >= 0 && net < n_pi) P[net] += delta;
  for (int32_t k = 0; k < n_gates; ++k) {
    int32_t g = order[k];
    double x[ORC_MAX_IN] = {0, 0, 0, 0, 0, 0};
    for (int32_t e = fanin_ptr[g]; e < fanin_ptr[g + 1]; ++e) x[e - fanin_ptr[g]] = P[fanin[e]];
    P[n_pi + g] = clamp01(sp_rule(op[g], x));
    if ((int64_t)n_pi + g == net) P[net] += delta;
  }
}

/* Sizing score (Sec. IV-A, Eq. 8) of every gate, from its output net n:
 *   alpha_n = TR_model,n = 2 P_n (1 - P_n)              (Eq. 2)
 *   dP/dalpha_n = lambda_n / (d alpha_n / d P_n) = lambda_n / (2 (1 - 2 P_n))
 *   P_sw,n = kappa beta_n C_n alpha_n  (its local power), so
 *   dP/dP_sw,n = dP/dalpha_n / (kappa beta_n C_n) and
 *   S_g = |dP/dP_sw,n| * P_sw,n = |lambda_n| P_n (1 - P_n) / |1 - 2 P_n|.
 * Where |1 - 2 P_n| < eps (the activity is flat in P) eps stands in for it. */
void orc_sizing_score(int32_t n_pi, int32_t n_gates, const double *P, const double *lambda,
                      double eps, double *score) {
  for (int32_t g = 0; g < n_gates; ++g) {
    int64_t n = (int64_t)n_pi + g;
    double slope = fabs(1.0 - 2.0 * P[n]);
    if (slope < eps) slope = eps;
    score[g] = fabs(lambda[n]) * P[n] * (1.0 - P[n]) / slope;
  }
}
