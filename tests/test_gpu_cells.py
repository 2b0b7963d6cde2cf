"""Library cells given as Boolean expressions (Sec. III-A, Alg. 1-3) on the
GPU, through the C ABI, against the FP64 oracle's interpreter of the same
expressions: probabilities and partials operation by operation, bits by
evaluating the code on packed words (counts bit-exact)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import (SP_ABS, assert_beta_close, assert_grad_close, assert_power_close,
                               oracle_column, say)

pytestmark = pytest.mark.gpu

FWD_ALL = ("sp", "tr", "sp_acc", "tr_acc", "beta", "tr_hyb", "ones", "toggles", "power")
# the fixed cells INV .. AOI21 written as expressions, in opcode order
FIXED_AS_EXPR = ("!A", "A", "A&B", "A|B", "!(A&B)", "!(A|B)", "A^B", "!(A&B|C)")


@pytest.fixture(scope="module")
def ctx():
    return api.Context(0)


def _mixed_spec(n_gates, n_pi, depth):
    ops = tuple(range(9)) + tuple(synth.CELL_BASE + c for c in range(len(synth.LIBRARY)))
    return synth.DagSpec(n_gates=n_gates, n_pi=n_pi, depth=depth, ops=ops, cells=synth.LIBRARY)


def _check_forward(res, f, col, hybrid):
    np.testing.assert_allclose(res["sp"][col], f["sp"], atol=SP_ABS, rtol=0)
    np.testing.assert_allclose(res["tr"][col], f["tr_model"], atol=SP_ABS, rtol=0)
    if hybrid:
        np.testing.assert_array_equal(res["ones"][col].astype(np.uint64), f["ones"])
        np.testing.assert_array_equal(res["toggles"][col].astype(np.uint64), f["toggles"])
        np.testing.assert_allclose(res["sp_acc"][col], f["sp_acc"], atol=SP_ABS, rtol=0)
        np.testing.assert_allclose(res["tr_acc"][col], f["tr_acc"], atol=SP_ABS, rtol=0)
        np.testing.assert_allclose(res["tr_hyb"][col], f["tr_hyb"], atol=SP_ABS, rtol=0)
        assert_beta_close(res["beta"][col], res["tr"][col], f, "beta")


@pytest.mark.parametrize("c", range(len(synth.LIBRARY)))
def test_each_library_cell_alone(ctx, c):
    """One level of 600 instances of library cell c on random distinct PIs
    (a ragged last wave), every forward output and both gradients."""
    expr = synth.LIBRARY[c]
    say(f"library cell {c}: {expr}")
    rng = np.random.default_rng(100 + c)
    n_pi, G = 40, 600
    k = synth.cell_arity(expr)
    gates = [(synth.CELL_BASE + c, list(rng.choice(n_pi, size=k, replace=False)))
             for _ in range(G)]
    nl = synth.from_gates(n_pi, gates, synth.LIBRARY)
    p = synth.pi_probs(n_pi, 30 + c)
    cap = synth.net_caps(nl.n_nets, 31 + c)
    d = api.Design(ctx, nl)
    assert d.depth == 1
    ev = api.Eval(d, mode=L.DP_HYBRID, n_sim=64 * 9, seed=5)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(FWD_ALL)
    o = oracle.Netlist.of(nl)
    f, adj = oracle_column(o, p[0], cap, mode="hybrid", n_words=9, seed=5)
    _check_forward(res, f, 0, True)
    assert_power_close(res["power"], f["power"])
    g = ev.backward(want=("dpi", "dcap"))
    assert_grad_close(g["dpi"][0], adj["dpi"], "dP/dp")
    assert_grad_close(g["dcap"], adj["dcap"], "dP/dC")


# A cell at every limit at once: 6 inputs, 32 operations, 8 stack entries.
LIMIT_CELL = "(A|(B|(C|(D|(E|(F|(A&B)))))))^(!C&!D)^(E|!F)^!(A^!B)"


def test_cell_at_every_limit(ctx):
    """Two levels of the limit cell (the second reading the first) next to
    fixed cells: every output, counts bit-exact, gradients and adjoints."""
    code, n_in = oracle.cell_code(LIMIT_CELL)
    depth, top = 0, 0
    for op, _ in code:
        top += 1 if op in ("IN", "CONST0", "CONST1") else (0 if op == "NOT" else -1)
        depth = max(depth, top)
    assert (len(code), n_in, depth) == (32, 6, 8)
    say("library cell at every limit")
    rng = np.random.default_rng(11)
    n_pi = 30
    gates = [(synth.CELL_BASE, list(rng.choice(n_pi, size=6, replace=False))) for _ in range(300)]
    lvl1 = n_pi + np.arange(300)
    gates += [(synth.CELL_BASE, list(rng.choice(lvl1, size=6, replace=False))) for _ in range(200)]
    gates += [(synth.AND2, list(rng.choice(lvl1, size=2, replace=False))) for _ in range(100)]
    nl = synth.from_gates(n_pi, gates, (LIMIT_CELL,))
    p = synth.pi_probs(n_pi, 12, batch=2)
    cap = synth.net_caps(nl.n_nets, 13)
    d = api.Design(ctx, nl)
    assert d.depth == 2
    ev = api.Eval(d, 2, mode=L.DP_HYBRID, n_sim=64 * 13, seed=4)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(FWD_ALL)
    g = ev.backward(want=("dpi", "dcap"))
    lam, _ = ev.power_gradients()
    o = oracle.Netlist.of(nl)
    dcap = np.zeros(nl.n_nets)
    for b in range(2):
        f, adj = oracle_column(o, p[b], cap, mode="hybrid", n_words=13, seed=4)
        _check_forward(res, f, b, True)
        assert_power_close(res["power"][b], f["power"], f"power[{b}]")
        assert_grad_close(g["dpi"][b], adj["dpi"], f"dP/dp[{b}]")
        assert_grad_close(lam[b], adj["lam"], f"lambda[{b}]")
        dcap += adj["dcap"]
    assert_grad_close(g["dcap"], dcap, "dP/dC")


def test_waves_holding_several_library_cells(ctx):
    """One level of the nine library cells and the fixed cells in random
    order: after sorting, most waves hold several library cells, each taking
    its turn with its own code (SP, bits, partials)."""
    say("several library cells per wave")
    ops = list(range(9)) + [synth.CELL_BASE + c for c in range(len(synth.LIBRARY))]
    rng = np.random.default_rng(7)
    n_pi, G = 40, 900
    arity = synth.arity_table(synth.LIBRARY)
    gates = []
    for _ in range(G):
        o = int(rng.choice(ops))
        gates.append((o, list(rng.choice(n_pi, size=int(arity[o]), replace=False))))
    nl = synth.from_gates(n_pi, gates, synth.LIBRARY)
    p = synth.pi_probs(n_pi, 8, batch=2)
    cap = synth.net_caps(nl.n_nets, 9)
    d = api.Design(ctx, nl)
    assert d.depth == 1
    ev = api.Eval(d, 2, mode=L.DP_HYBRID, n_sim=64 * 11, seed=6)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(FWD_ALL)
    g = ev.backward(want=("dpi", "dcap"))
    lam, _ = ev.power_gradients()
    o = oracle.Netlist.of(nl)
    dcap = np.zeros(nl.n_nets)
    for b in range(2):
        f, adj = oracle_column(o, p[b], cap, mode="hybrid", n_words=11, seed=6)
        _check_forward(res, f, b, True)
        assert_grad_close(g["dpi"][b], adj["dpi"], f"dP/dp[{b}]")
        assert_grad_close(lam[b], adj["lam"], f"lambda[{b}]")
        dcap += adj["dcap"]
    assert_grad_close(g["dcap"], dcap, "dP/dC")


@pytest.mark.parametrize("mode,sched,B", [("modeled", L.DP_SCHED_LEVEL, 3),
                                          ("modeled", L.DP_SCHED_GRAPH, 2),
                                          ("hybrid", L.DP_SCHED_LEVEL, 2),
                                          ("hybrid", L.DP_SCHED_GRAPH, 1)])
def test_mixed_dag_all_outputs(ctx, mode, sched, B):
    """3,000 gates over the nine fixed cells and the library, depth 20: every
    output per column, the PI and capacitance gradients, and every net's
    adjoint (power gradients)."""
    say(f"library dag {mode} sched={sched} B={B}")
    nl = synth.random_dag(_mixed_spec(3000, 64, 20), 11)
    assert (nl.op >= synth.CELL_BASE).any() and (nl.op < synth.CELL_BASE).any()
    p = synth.pi_probs(nl.n_pi, 12, batch=B)
    cap = synth.net_caps(nl.n_nets, 13)
    d = api.Design(ctx, nl)
    hyb = mode == "hybrid"
    ev = api.Eval(d, B, mode=L.DP_HYBRID if hyb else L.DP_MODELED, n_sim=64 * 37, seed=9)
    ev.set_schedule(sched)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(FWD_ALL if hyb else ("sp", "tr", "beta", "power"))
    g = ev.backward(want=("dpi", "dcap"))
    lam, _ = ev.power_gradients()
    o = oracle.Netlist.of(nl)
    np.testing.assert_array_equal(d.levels(), o.levels())
    dcap = np.zeros(nl.n_nets)
    for b in range(B):
        f, adj = oracle_column(o, p[b], cap, mode=mode, n_words=37, seed=9)
        _check_forward(res, f, b, hyb)
        assert_power_close(res["power"][b], f["power"], f"power[{b}]")
        assert_grad_close(g["dpi"][b], adj["dpi"], f"dP/dp[{b}]")
        assert_grad_close(lam[b], adj["lam"], f"lambda[{b}]")
        dcap += adj["dcap"]
    assert_grad_close(g["dcap"], dcap, "dP/dC")


def test_fixed_cells_written_as_expressions_run_as_fixed_cells(ctx):
    """A netlist whose gates use library expressions equal to the fixed
    cells gives bit-identical results to the fixed-cell netlist."""
    say("fixed cells as expressions")
    nl = synth.random_dag(synth.DagSpec(n_gates=2500, n_pi=64, depth=18, ops=tuple(range(8))), 17)
    as_expr = dataclasses.replace(nl, op=(nl.op.astype(np.int32) + synth.CELL_BASE).astype(np.uint8),
                                  cells=FIXED_AS_EXPR)
    p = synth.pi_probs(nl.n_pi, 18, batch=2)
    cap = synth.net_caps(nl.n_nets, 19)
    out = []
    for net in (nl, as_expr):
        d = api.Design(ctx, net)
        ev = api.Eval(d, 2, mode=L.DP_HYBRID, n_sim=64 * 20, seed=3)
        ev.set_pi_prob(p)
        ev.set_caps(cap)
        ev.set_schedule(L.DP_SCHED_PERSISTENT if net is as_expr else L.DP_SCHED_LEVEL)
        r = ev.forward(FWD_ALL)
        r.update(ev.backward(want=("dpi", "dcap")))
        out.append(r)
    for k in FWD_ALL + ("dpi", "dcap"):
        np.testing.assert_array_equal(out[0][k], out[1][k], err_msg=k)


def test_library_design_in_group_and_serving(ctx):
    """A library-cell design merged with a fixed-cell design (group launches
    and serving steps) gives what it gives alone."""
    say("library design: group and serving")
    nls = [synth.random_dag(_mixed_spec(2000, 64, 16), 21), synth.random_dag(synth.SPECS["dag2k"], 22)]
    caps = [synth.net_caps(nl.n_nets, 23 + i) for i, nl in enumerate(nls)]
    designs = [api.Design(ctx, nl) for nl in nls]
    alone, evs = [], []
    for i, (nl, d) in enumerate(zip(nls, designs)):
        ev = api.Eval(d, 2, mode=L.DP_MODELED, n_sim=128)
        ev.set_pi_prob(synth.pi_probs(nl.n_pi, 24 + i, batch=2))
        ev.set_caps(caps[i])
        r = ev.forward(("sp", "power"))
        r.update(ev.backward(want=("dpi",)))
        alone.append(r)
        evs.append(ev)
    grp = api.Group(ctx, evs)
    res = grp.run(("sp", "power"), backward=True)
    for r, a in zip(res, alone):
        for k in ("sp", "power", "dpi"):
            np.testing.assert_array_equal(r[k], a[k], err_msg=k)
    grp.close()
    srv = api.Server(ctx, hbm_budget_bytes=128 << 20, max_batch=8, max_inflight=3)
    ids = [srv.add_design(d, c, mode=L.DP_MODELED, n_sim=128, seed=5) for d, c in zip(designs, caps)]
    rng = np.random.default_rng(25)
    qs = [(k % 2, rng.uniform(0.1, 0.9, nls[k % 2].n_pi).astype(np.float32)) for k in range(16)]
    one = [srv.wait(srv.submit(ids[i], p, None, True)) for i, p in qs[:4]]
    mixed = [srv.wait(t) for t in [srv.submit(ids[i], p, None, True) for i, p in qs]]
    for k in range(4):
        assert one[k][0] == mixed[k][0]
        np.testing.assert_array_equal(one[k][1], mixed[k][1])
    o = oracle.Netlist.of(nls[0])
    for k in (0, 2, 10):
        f, adj = oracle_column(o, qs[k][1], caps[0])
        assert_power_close(mixed[k][0], f["power"])
        assert_grad_close(mixed[k][1], adj["dpi"], "served dP/dp")
    srv.close()


def test_library_errors(ctx):
    say("library errors")
    nl = synth.from_gates(3, [(synth.CELL_BASE, [0, 1])], ("A&B",))

    def compile_with(cells, net=nl):
        return api.Design(ctx, dataclasses.replace(net, cells=tuple(cells)))

    for bad, what in (("A&", "operand"), ("(A|B", "')'"), ("A $ B", "character"),
                      ("A B", "after"), ("a&b&c&d&e&f&g", "6 inputs"),
                      ("&".join(["A"] * 20), "32 operations"),
                      ("A|(B|(C|(D|(E|(F|(A|(B|C)))))))", "8 stack"), ("1", "no inputs")):
        with pytest.raises(L.DiffPowerError, match="INVALID") as ei:
            compile_with([bad])
        assert what in str(ei.value), (bad, str(ei.value))
    with pytest.raises(L.DiffPowerError, match="INVALID"):  # arity: 3 inputs, 2 pins
        compile_with(["A&B&C"])
    with pytest.raises(L.DiffPowerError, match="INVALID"):  # opcode past the library
        compile_with([])
    d = compile_with(["A&!B"])  # not a fixed cell's code
    ev = api.Eval(d, mode=L.DP_MODELED)
    with pytest.raises(L.DiffPowerError, match="UNSUPPORTED"):
        ev.set_schedule(L.DP_SCHED_PERSISTENT)
    ev.set_pi_prob(np.array([[0.3, 0.6, 0.5]], np.float32))
    ev.set_caps(np.ones(4, np.float32))
    sp = ev.forward(("sp",))["sp"][0]
    assert abs(sp[3] - 0.3 * 0.4) < 1e-6


def test_mixed_dag_many_columns_equal_single_columns(ctx):
    """40 columns (lane-serial reverse pulls for both cell kinds): each
    column's SP, power and gradients equal a one-column eval's bit for bit,
    and column 0 matches the oracle."""
    say("library dag, 40 columns")
    nl = synth.random_dag(_mixed_spec(3000, 64, 20), 21)
    B = 40
    p = synth.pi_probs(nl.n_pi, 22, batch=B)
    cap = synth.net_caps(nl.n_nets, 23)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, B, mode=L.DP_MODELED)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(("sp", "power"))
    g = ev.backward(want=("dpi",))
    one = api.Eval(d, 1, mode=L.DP_MODELED)
    one.set_caps(cap)
    for b in (0, 17, B - 1):
        one.set_pi_prob(p[b:b + 1])
        r1 = one.forward(("sp", "power"))
        g1 = one.backward(want=("dpi",))
        np.testing.assert_array_equal(r1["sp"][0], res["sp"][b], err_msg=f"sp[{b}]")
        np.testing.assert_array_equal(r1["power"][0], res["power"][b], err_msg=f"power[{b}]")
        np.testing.assert_array_equal(g1["dpi"][0], g["dpi"][b], err_msg=f"dP/dp[{b}]")
    o = oracle.Netlist.of(nl)
    f, adj = oracle_column(o, p[0], cap, mode="modeled")
    assert_power_close(res["power"][0], f["power"], "power[0]")
    assert_grad_close(g["dpi"][0], adj["dpi"], "dP/dp[0]")


MUX_OUT = "(I0&!S)|(I1&S)"  # a multiplexer written out: inputs [I0, S, I1] by first appearance


def test_pin_list_wires_the_written_out_multiplexer(ctx):
    """Alg. 1's perm: the written-out multiplexer with pin list "I0,I1,S"
    and its gates' fan-in given in that pin order.  Every output equals the
    oracle's (given the same pin list), the output SP equals the op-by-op
    value (1 - s) i0 + s i1 - i0 i1 s (1 - s) of the expression read once
    per operation, and the design is bit for bit the one compiled without a
    pin list from the fan-in put into first-appearance order by hand."""
    say("pin list: written-out multiplexer")
    rng = np.random.default_rng(77)
    n_pi, G = 24, 300
    gates = [(synth.CELL_BASE, list(rng.choice(n_pi, size=3, replace=False))) for _ in range(G)]
    by_pins = dataclasses.replace(synth.from_gates(n_pi, gates, (MUX_OUT,)), pins=("I0,I1,S",))
    # the same gates with each fan-in reordered [I0, I1, S] -> [I0, S, I1]
    by_hand = synth.from_gates(n_pi, [(op, [f[0], f[2], f[1]]) for op, f in gates], (MUX_OUT,))
    p = synth.pi_probs(n_pi, 78)
    cap = synth.net_caps(n_pi + G, 79)
    res = {}
    for name, nl in (("pins", by_pins), ("hand", by_hand)):
        d = api.Design(ctx, nl)
        ev = api.Eval(d, mode=L.DP_HYBRID, n_sim=64 * 7, seed=3)
        ev.set_pi_prob(p)
        ev.set_caps(cap)
        res[name] = ev.forward(FWD_ALL)
        res[name].update(ev.backward(want=("dpi", "dcap")))
    for k in res["pins"]:
        np.testing.assert_array_equal(res["pins"][k], res["hand"][k], err_msg=k)
    o = oracle.Netlist.of(by_pins)
    f, adj = oracle_column(o, p[0], cap, mode="hybrid", n_words=7, seed=3)
    _check_forward(res["pins"], f, 0, True)
    assert_power_close(res["pins"]["power"], f["power"])
    assert_grad_close(res["pins"]["dpi"][0], adj["dpi"], "dP/dp")
    pp = p[0].astype(np.float64)
    for g, (_, (i0, i1, s)) in enumerate(gates):
        a, b, c = pp[i0], pp[i1], pp[s]
        want = (1 - c) * a + c * b - a * b * c * (1 - c)
        assert abs(res["pins"]["sp"][0][n_pi + g] - want) <= SP_ABS


def test_identical_codes_share_one_logic_id(ctx):
    """Alg. 1's dedup: expressions that compile to the same code (up to the
    names of their identifiers, with pin lists mapping each onto its gates'
    fan-in) share one logic id; one that is a fixed cell runs as it.  The
    deduplicated design matches the oracle."""
    say("dedup of library cells")
    cells = ("A&!B", "X&!Y", MUX_OUT, "(a&!c)|(b&c)", "B&A", "Q&!P")
    pins = (None, None, "I0,I1,S", "a b c", "A,B", "P,Q")
    rng = np.random.default_rng(80)
    n_pi = 30
    gates = []
    for _ in range(900):
        c = int(rng.integers(0, len(cells)))
        gates.append((synth.CELL_BASE + c, list(rng.choice(n_pi, size=2 if c in (0, 1, 4, 5) else 3,
                                                           replace=False))))
    nl = dataclasses.replace(synth.from_gates(n_pi, gates, cells), pins=pins)
    d = api.Design(ctx, nl)
    logic, n_logic = d.cell_logic()
    # A&!B, X&!Y and Q&!P (pins P,Q: input Q is pin 1) share one code; the two
    # multiplexers another; B&A is the fixed AND2
    assert n_logic == 2
    assert logic[0] == logic[1] == logic[5] and logic[2] == logic[3] and logic[0] != logic[2]
    assert logic[4] == -1 - 2
    p = synth.pi_probs(n_pi, 81)
    cap = synth.net_caps(nl.n_nets, 82)
    ev = api.Eval(d, mode=L.DP_HYBRID, n_sim=64 * 5, seed=4)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(FWD_ALL)
    g = ev.backward(want=("dpi",))
    o = oracle.Netlist.of(nl)
    f, adj = oracle_column(o, p[0], cap, mode="hybrid", n_words=5, seed=4)
    _check_forward(res, f, 0, True)
    assert_power_close(res["power"], f["power"])
    assert_grad_close(g["dpi"][0], adj["dpi"], "dP/dp")


def test_pin_list_errors(ctx):
    say("pin list errors")
    nl = synth.from_gates(4, [(synth.CELL_BASE, [0, 1, 2])], (MUX_OUT,))
    for bad in ("I0,I1", "I0,I1,S,T", "I0,I0,S", "I0,I1,X", "I0;I1;S"):
        with pytest.raises(L.DiffPowerError, match="INVALID"):
            api.Design(ctx, dataclasses.replace(nl, pins=(bad,)))
