"""Pins of the oracle's library-cell path (Alg. 1-3: expressions compiled to
stack code, evaluated operation by operation, differentiated in reverse),
each against something other than the oracle: hand-written post-order
code, Python's own evaluation of the expression, exact minterm sums, closed
forms, finite differences and the complex-step derivative."""
from __future__ import annotations

import itertools
import re

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import synth
from tests import brute

LIB = synth.LIBRARY


def _py_eval(expr, values):
    """The expression evaluated by Python on booleans (an independent route)."""
    names = list(dict.fromkeys(re.findall(r"[A-Za-z_][A-Za-z0-9_]*", expr)))
    py = expr.replace("!", " not ").replace("~", " not ").replace("&", " and ")
    py = py.replace("*", " and ").replace("|", " or ").replace("+", " or ").replace("^", " != ")
    env = dict(zip(names, (bool(v) for v in values)))
    py = re.sub(r"(?<![A-Za-z0-9_])1(?![A-Za-z0-9_])", "True", py)
    py = re.sub(r"(?<![A-Za-z0-9_])0(?![A-Za-z0-9_])", "False", py)
    # Python's 'not' binds looser than '!=': parenthesize each negated operand
    py = re.sub(r"not\s+([A-Za-z_][A-Za-z0-9_]*)", r"(not \1)", py)
    return bool(eval(py, {}, env))


def test_parser_precedence_and_input_order():
    code, n = oracle.cell_code("A|B&C")
    assert code == [("IN", 0), ("IN", 1), ("IN", 2), ("AND", 0), ("OR", 0)] and n == 3
    assert oracle.cell_code("A^B&C")[0] == [("IN", 0), ("IN", 1), ("IN", 2), ("AND", 0),
                                            ("XOR", 0)]
    assert oracle.cell_code("A|B^C")[0] == [("IN", 0), ("IN", 1), ("IN", 2), ("XOR", 0),
                                            ("OR", 0)]
    assert oracle.cell_code("!A&B")[0] == [("IN", 0), ("NOT", 0), ("IN", 1), ("AND", 0)]
    assert oracle.cell_code("(A|B)&C")[0] == [("IN", 0), ("IN", 1), ("OR", 0), ("IN", 2),
                                              ("AND", 0)]
    assert oracle.cell_code("A&B&C")[0] == [("IN", 0), ("IN", 1), ("AND", 0), ("IN", 2),
                                            ("AND", 0)]
    assert oracle.cell_code("B & A")[0] == [("IN", 0), ("IN", 1), ("AND", 0)]
    assert oracle.cell_code("~(A+B)*C")[0] == [("IN", 0), ("IN", 1), ("OR", 0), ("NOT", 0),
                                               ("IN", 2), ("AND", 0)]
    assert oracle.cell_code("A^1")[0] == [("IN", 0), ("CONST1", 0), ("XOR", 0)]
    assert oracle.cell_code("A&B|A")[1] == 2
    for bad in ("", "A&", "(A", "A B", "A&&B", "A|B)", "A&B&C&D&E&F&G"):
        with pytest.raises(ValueError):
            oracle.cell_code(bad)


@pytest.mark.parametrize("c", range(len(LIB)))
def test_cell_bits_equal_python_truth_table(c):
    oracle.set_cells(LIB)
    expr = LIB[c]
    k = synth.cell_arity(expr)
    words = np.zeros(6, dtype=np.uint64)
    words[:k] = brute.pack_minterm_words(k)
    got = oracle.gate_bits(synth.CELL_BASE + c, words)
    for m, vals in enumerate(itertools.product((0, 1), repeat=k)):
        bits = [(m >> i) & 1 for i in range(k)]
        assert ((got >> m) & 1) == int(_py_eval(expr, bits)), (expr, bits)


READ_ONCE = [c for c, e in enumerate(LIB)
             if len(re.findall(r"[A-Za-z_][A-Za-z0-9_]*", e)) == synth.cell_arity(e)]


@pytest.mark.parametrize("c", READ_ONCE)
def test_read_once_cells_are_exact(c):
    """Operation-by-operation evaluation is exact on read-once expressions:
    it equals the minterm sum of the truth table."""
    oracle.set_cells(LIB)
    expr = LIB[c]
    k = synth.cell_arity(expr)
    rng = np.random.default_rng(c)
    for _ in range(20):
        p = rng.uniform(0, 1, k)
        exact = 0.0
        for vals in itertools.product((0, 1), repeat=k):
            if _py_eval(expr, vals):
                exact += np.prod([pi if v else 1 - pi for pi, v in zip(p, vals)])
        assert oracle.gate_sp(synth.CELL_BASE + c, p) == pytest.approx(exact, abs=1e-14)


def test_read_many_cells_follow_op_by_op_semantics():
    """The multiplexer written out reads S twice: the op-by-op value is the
    exact (1-s) i0 + s i1 minus i0 i1 s (1 - s); the majority reads each
    input twice: OR(OR(ab, ac), bc) with independent operands.  (The
    expression's inputs in order of first appearance are I0, S, I1.)"""
    oracle.set_cells(LIB)
    mux = synth.CELL_BASE + LIB.index("(I0&!S)|(I1&S)")
    maj = synth.CELL_BASE + LIB.index("A&B|A&C|B&C")
    rng = np.random.default_rng(3)
    for _ in range(20):
        i0, i1, s = rng.uniform(0, 1, 3)
        want = (1 - s) * i0 + s * i1 - i0 * i1 * s * (1 - s)
        assert oracle.gate_sp(mux, [i0, s, i1]) == pytest.approx(want, abs=1e-15)
        assert oracle.gate_sp(synth.MUX2, [i0, i1, s]) - want == pytest.approx(
            i0 * i1 * s * (1 - s), abs=1e-15)
        a, b, c = rng.uniform(0, 1, 3)
        ab, ac, bc = a * b, a * c, b * c
        o1 = ab + ac - ab * ac
        assert oracle.gate_sp(maj, [a, b, c]) == pytest.approx(o1 + bc - o1 * bc, abs=1e-15)


def test_common_gates_as_expressions_equal_fixed_cells():
    exprs = ("!A", "A", "A&B", "A|B", "!(A&B)", "!(A|B)", "A^B", "!((A&B)|C)")
    fixed = (synth.INV, synth.BUF, synth.AND2, synth.OR2, synth.NAND2, synth.NOR2,
             synth.XOR2, synth.AOI21)
    oracle.set_cells(exprs)
    rng = np.random.default_rng(4)
    for c, op in enumerate(fixed):
        for _ in range(10):
            x = rng.uniform(0, 1, 3)
            assert oracle.gate_sp(synth.CELL_BASE + c, x) == pytest.approx(
                oracle.gate_sp(op, x), abs=1e-15)
            np.testing.assert_allclose(oracle.gate_partials(synth.CELL_BASE + c, x),
                                       oracle.gate_partials(op, x), atol=1e-15)


@pytest.mark.parametrize("c", range(len(LIB)))
def test_cell_partials_equal_finite_differences(c):
    oracle.set_cells(LIB)
    op = synth.CELL_BASE + c
    k = synth.cell_arity(LIB[c])
    rng = np.random.default_rng(10 + c)
    h = 1e-6
    for _ in range(10):
        x = rng.uniform(0.05, 0.95, k)
        d = oracle.gate_partials(op, x)
        for j in range(k):
            e = np.zeros(k)
            e[j] = h
            fd = (oracle.gate_sp(op, x + e) - oracle.gate_sp(op, x - e)) / (2 * h)
            assert d[j] == pytest.approx(fd, abs=1e-8)


def _cell_spec(n_gates, n_pi, depth):
    ops = tuple(range(9)) + tuple(synth.CELL_BASE + c for c in range(len(LIB)))
    return synth.DagSpec(n_gates=n_gates, n_pi=n_pi, depth=depth, ops=ops, cells=LIB)


@pytest.mark.parametrize("seed", range(6))
def test_tree_of_read_once_cells_is_exact(seed):
    ops = tuple(range(8)) + tuple(synth.CELL_BASE + c for c in READ_ONCE)
    nl = synth.random_tree(10, seed, ops=ops, cells=LIB)
    o = oracle.Netlist.of(nl)
    p = np.random.default_rng(seed).uniform(0.05, 0.95, nl.n_pi)
    oracle.set_cells(LIB)
    exact = brute_exact(nl, p)
    np.testing.assert_allclose(o.sp(p), exact, atol=1e-12)


def brute_exact(nl, p):
    """Exact P(net = 1) by enumeration, cells evaluated by Python."""
    M = 1 << nl.n_pi
    vals = np.zeros((nl.n_nets, M), dtype=bool)
    for m in range(M):
        v = [(m >> i) & 1 for i in range(nl.n_pi)] + [0] * nl.n_gates
        done = [True] * nl.n_pi + [False] * nl.n_gates
        while not all(done):
            for g in range(nl.n_gates):
                if done[nl.n_pi + g]:
                    continue
                ins = nl.fanin[nl.fanin_ptr[g]:nl.fanin_ptr[g + 1]]
                if all(done[n] for n in ins):
                    op = int(nl.op[g])
                    xs = [v[n] for n in ins]
                    if op >= synth.CELL_BASE:
                        out = _py_eval(nl.cells[op - synth.CELL_BASE], xs)
                    else:
                        out = bool(brute.TRUTH[op](*[bool(x) for x in xs]))
                    v[nl.n_pi + g] = int(out)
                    done[nl.n_pi + g] = True
        vals[:, m] = v
    idx = np.arange(M)
    w = np.ones(M)
    for i in range(nl.n_pi):
        bit = (idx >> i) & 1
        w *= np.where(bit == 1, p[i], 1.0 - p[i])
    return vals.astype(np.float64) @ w


def test_adjoint_with_cells_equals_complex_step():
    nl = synth.random_dag(_cell_spec(600, 24, 10), 5)
    cap = synth.net_caps(nl.n_nets, 5)
    o = oracle.Netlist.of(nl)
    p = np.random.default_rng(5).uniform(0.1, 0.9, nl.n_pi)
    beta = np.random.default_rng(6).uniform(0.5, 2.0, nl.n_nets)
    P = o.sp(p)
    adj = o.adjoint(P, beta, cap)
    for i in range(nl.n_pi):
        cs = o.power_complex_step(p, beta, cap.astype(np.float64), i)
        assert adj["dpi"][i] == pytest.approx(cs, rel=1e-10, abs=1e-12)


def test_sim_with_cells_counts_exhaustive_stimulus():
    """Exhaustive stimulus: every net's ones count equals T times its
    number of satisfying PI assignments (cells evaluated by Python)."""
    nl = synth.random_dag(_cell_spec(60, 6, 5), 7)
    o = oracle.Netlist.of(nl)
    words = np.zeros((nl.n_pi, 2), dtype=np.uint64)
    words[:, 0] = brute.pack_minterm_words(nl.n_pi)
    words[:, 1] = words[:, 0]
    ones, _ = o.sim(2, pi_words=words)
    exact = brute_exact(nl, np.full(nl.n_pi, 0.5)) * 64
    np.testing.assert_array_equal(ones, (2 * exact).round().astype(np.uint64))


def test_pin_lists_reorder_fanin_into_expression_order():
    """The oracle's own Alg. 1 perm: a gate wired by pin list equals the
    same gate with its fan-in written in the expression's order of first
    appearance; identifiers are numbered as the parser first meets them."""
    assert oracle.expression_inputs("(I0&!S)|(I1&S)") == ["I0", "S", "I1"]
    assert oracle.expression_inputs("!(b1 ^ a_2) | 1 & b1") == ["b1", "a_2"]
    expr = "(I0&!S)|(I1&S)"
    rng = np.random.default_rng(5)
    n_pi = 9
    wires = [list(rng.choice(n_pi, 3, replace=False)) for _ in range(20)]
    op = np.full(20, oracle.CELL_BASE, np.uint8)
    ptr = np.arange(21, dtype=np.int32) * 3
    by_pins = oracle.Netlist(n_pi, op, ptr, np.array(sum(wires, []), np.int32), [expr],
                             ["I0, I1, S"])
    by_hand = oracle.Netlist(n_pi, op, ptr,
                             np.array(sum([[w[0], w[2], w[1]] for w in wires], []), np.int32),
                             [expr])
    p = rng.uniform(0.1, 0.9, n_pi)
    np.testing.assert_array_equal(by_pins.sp(p), by_hand.sp(p))
    with pytest.raises(ValueError):
        oracle.Netlist(n_pi, op, ptr, np.array(sum(wires, []), np.int32), [expr], ["I0,I1"])
