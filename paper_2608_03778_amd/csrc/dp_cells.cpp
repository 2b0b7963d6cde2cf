// Library cells given as Boolean expressions (Sec. III-A, Alg. 1): each
// expression is compiled to post-order code for a zero-address stack
// machine, which the level kernels interpret for probabilities, bits and
// partial derivatives.
//
// Grammar (NOT binds tightest, then AND, XOR, OR; binary operators are left
// associative):  expr := term (op term)* ;  term := ('!'|'~') term | '(' expr
// ')' | identifier | '0' | '1' ;  AND is '&' or '*', XOR '^', OR '|' or '+'.
// A cell's inputs are its distinct identifiers in order of first
// appearance; a gate's fan-in list follows that order.
#include <algorithm>
#include <cctype>
#include <cstring>
#include <initializer_list>
#include <string>
#include <vector>

#include "dp_internal.h"

namespace dp {

namespace {

enum Tok { T_END, T_ID, T_ZERO, T_ONE, T_NOT, T_AND, T_XOR, T_OR, T_LP, T_RP, T_BAD };

struct Lexer {
  const char *s;
  size_t i = 0;
  std::string id;
  Tok next() {
    while (s[i] == ' ' || s[i] == '\t') ++i;
    const char c = s[i];
    if (!c) return T_END;
    ++i;
    switch (c) {
      case '!': case '~': return T_NOT;
      case '&': case '*': return T_AND;
      case '^': return T_XOR;
      case '|': case '+': return T_OR;
      case '(': return T_LP;
      case ')': return T_RP;
      case '0': case '1':
        if (std::isalnum((unsigned char)s[i]) || s[i] == '_') return T_BAD;
        return c == '0' ? T_ZERO : T_ONE;
      default: break;
    }
    if (std::isalpha((unsigned char)c) || c == '_') {
      id.assign(1, c);
      while (std::isalnum((unsigned char)s[i]) || s[i] == '_') id += s[i++];
      return T_ID;
    }
    return T_BAD;
  }
};

// Precedence climbing, emitting code as operands complete.
struct Compiler {
  Lexer lx;
  Tok tok = T_END;
  std::vector<std::string> inputs;
  std::vector<uint16_t> code;
  std::string err;
  int depth = 0, max_depth = 0;

  void advance() { tok = lx.next(); }
  void emit(int op, int arg) {
    code.push_back((uint16_t)(op | (arg << 8)));
    if (op == kCellIn || op == kCellZero || op == kCellOne) depth += 1;
    else if (op != kCellNot) depth -= 1;
    if (depth > max_depth) max_depth = depth;
  }
  static int bind(Tok t) { return t == T_OR ? 1 : t == T_XOR ? 2 : t == T_AND ? 3 : 0; }
  static int op_of(Tok t) { return t == T_OR ? kCellOr : t == T_XOR ? kCellXor : kCellAnd; }

  void term() {
    if (!err.empty()) return;
    switch (tok) {
      case T_NOT:
        advance();
        term();
        emit(kCellNot, 0);
        return;
      case T_LP:
        advance();
        expr(1);
        if (tok != T_RP) {
          err = "missing ')'";
          return;
        }
        advance();
        return;
      case T_ZERO: emit(kCellZero, 0); advance(); return;
      case T_ONE: emit(kCellOne, 0); advance(); return;
      case T_ID: {
        size_t k = 0;
        while (k < inputs.size() && inputs[k] != lx.id) ++k;
        if (k == inputs.size()) inputs.push_back(lx.id);
        emit(kCellIn, (int)k);
        advance();
        return;
      }
      default: err = "operand expected"; return;
    }
  }
  // operators binding at least min_bind; a right operand takes only tighter
  // ones, which makes the binary operators left associative
  void expr(int min_bind) {
    term();
    while (err.empty() && bind(tok) >= min_bind) {
      const Tok op = tok;
      advance();
      expr(bind(op) + 1);
      emit(op_of(op), 0);
    }
  }
};

}  // namespace

std::string compile_cell(const char *text, CellCode *out) {
  if (!text) return "NULL expression";
  Compiler c;
  c.lx.s = text;
  c.advance();
  c.expr(1);
  if (c.err.empty() && c.tok == T_BAD) c.err = "unknown character";
  if (c.err.empty() && c.tok != T_END) c.err = "unexpected text after the expression";
  if (!c.err.empty()) return c.err;
  if (c.inputs.empty()) return "no inputs (a cell reads at least one pin)";
  if (c.inputs.size() > (size_t)kCellMaxIn) return "more than 6 inputs";
  if (c.code.size() > (size_t)kCellMaxCode) return "more than 32 operations";
  if (c.max_depth > kCellMaxStack) return "deeper than 8 stack entries";
  out->code = c.code;
  out->n_in = (int32_t)c.inputs.size();
  out->inputs = c.inputs;
  return "";
}

// Alg. 1's perm: the fan-in position of each input of a compiled cell given
// its pin list (names separated by commas or blanks, in the order a gate
// lists its fan-in).  perm[k] = pin position of input k (identifier k in
// order of first appearance).  Returns an error message, or "".
std::string pin_permutation(const CellCode &cc, const char *pins, std::vector<int32_t> *perm) {
  std::vector<std::string> names;
  std::string cur;
  for (const char *q = pins;; ++q) {
    const char ch = *q;
    if (ch == ',' || ch == ' ' || ch == '\t' || ch == 0) {
      if (!cur.empty()) names.push_back(cur);
      cur.clear();
      if (!ch) break;
    } else if (std::isalnum((unsigned char)ch) || ch == '_') {
      cur += ch;
    } else {
      return std::string("bad character '") + ch + "' in the pin list";
    }
  }
  if ((int32_t)names.size() != cc.n_in)
    return "the pin list names " + std::to_string(names.size()) + " pins; the function reads " +
           std::to_string(cc.n_in);
  perm->assign(cc.n_in, -1);
  for (int32_t j = 0; j < (int32_t)names.size(); ++j) {
    const auto it = std::find(cc.inputs.begin(), cc.inputs.end(), names[j]);
    if (it == cc.inputs.end()) return "pin " + names[j] + " is not read by the function";
    int32_t &slot = (*perm)[it - cc.inputs.begin()];
    if (slot >= 0) return "pin " + names[j] + " is listed twice";
    slot = j;
  }
  return "";
}

// The fixed cell a compiled expression is, if any (its code equals that
// cell's own; every such cell reads each input once, in pin order).
int fixed_op_of(const CellCode &cc) {
  auto is = [&](std::initializer_list<uint16_t> want) {
    return cc.code.size() == want.size() && std::equal(want.begin(), want.end(), cc.code.begin());
  };
  const uint16_t I0 = kCellIn, I1 = kCellIn | (1 << 8), I2 = kCellIn | (2 << 8);
  if (is({I0, kCellNot})) return DP_INV;
  if (is({I0})) return DP_BUF;
  if (is({I0, I1, kCellAnd})) return DP_AND2;
  if (is({I0, I1, kCellOr})) return DP_OR2;
  if (is({I0, I1, kCellAnd, kCellNot})) return DP_NAND2;
  if (is({I0, I1, kCellOr, kCellNot})) return DP_NOR2;
  if (is({I0, I1, kCellXor})) return DP_XOR2;
  if (is({I0, I1, kCellAnd, I2, kCellOr, kCellNot})) return DP_AOI21;
  return -1;
}

// The code run on 64 lanes at once, lane m carrying input pattern m.
uint64_t truth_table(const CellCode &cc) {
  uint64_t in[kCellMaxIn];
  for (int k = 0; k < kCellMaxIn; ++k) {
    uint64_t w = 0;
    for (int m = 0; m < 64; ++m)
      if ((m >> k) & 1) w |= 1ull << m;
    in[k] = w;
  }
  uint64_t st[kCellMaxStack];
  int top = 0;
  for (uint16_t word : cc.code) {
    const int op = word & 0xff, arg = word >> 8;
    if (op == kCellIn) {
      st[top++] = in[arg];
    } else if (op == kCellZero) {
      st[top++] = 0;
    } else if (op == kCellOne) {
      st[top++] = ~0ull;
    } else if (op == kCellNot) {
      st[top - 1] = ~st[top - 1];
    } else {
      const uint64_t b = st[--top];
      const uint64_t a = st[--top];
      st[top++] = op == kCellAnd ? (a & b) : (op == kCellOr ? (a | b) : (a ^ b));
    }
  }
  return st[0];
}

}  // namespace dp
