"""The flop cut of synthetic sequential netlists (Sec. III-A: startpoints
are primary inputs and flop outputs, endpoints primary outputs and flop
inputs), checked by simulating the sequential netlist cycle by cycle with
its flop state and the cut netlist with the same state on its pseudo-PIs."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2608_03778_amd import synth


def _comb_order(n_pi, op, fanin_ptr, fanin, source):
    """Kahn order of the gates that are not sources (a source's output is
    known before the sweep)."""
    G = len(op)
    n_nets = n_pi + G
    known = np.zeros(n_nets, bool)
    known[:n_pi] = True
    known[n_pi + np.nonzero(source)[0]] = True
    order, left = [], [g for g in range(G) if not source[g]]
    while left:
        nxt = []
        for g in left:
            if all(known[n] for n in fanin[fanin_ptr[g]:fanin_ptr[g + 1]]):
                order.append(g)
                known[n_pi + g] = True
            else:
                nxt.append(g)
        assert len(nxt) < len(left), "combinational cycle"
        left = nxt
    return order


def _eval(n_pi, op, fanin_ptr, fanin, order, values):
    for g in order:
        ins = [values[n] for n in fanin[fanin_ptr[g]:fanin_ptr[g + 1]]]
        values[n_pi + g] = oracle.gate_bits(int(op[g]), ins)


def test_cut_simulates_like_the_sequential_netlist():
    seq = synth.random_seq_dag(synth.DagSpec(n_gates=400, n_pi=12, depth=9), 16, 5)
    cut = synth.cut_flops(seq)
    nl = cut.netlist
    is_ff = seq.op == synth.DFF
    s_order = _comb_order(seq.n_pi, seq.op, seq.fanin_ptr, seq.fanin, is_ff)
    c_order = _comb_order(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin, np.zeros(nl.n_gates, bool))
    ff = np.nonzero(is_ff)[0]
    rng = np.random.default_rng(0)
    mask = (1 << 64) - 1
    state = [int(x) for x in rng.integers(0, 1 << 63, len(ff))]
    for t in range(12):
        pis = [int(x) for x in rng.integers(0, 1 << 63, seq.n_pi)]
        sv = [0] * (seq.n_pi + len(seq.op))
        sv[: seq.n_pi] = pis
        for k, g in enumerate(ff):
            sv[seq.n_pi + g] = state[k]
        _eval(seq.n_pi, seq.op, seq.fanin_ptr, seq.fanin, s_order, sv)
        cv = [0] * nl.n_nets
        cv[: seq.n_pi] = pis
        for k in range(len(ff)):
            cv[cut.ppi[k]] = state[k]
        _eval(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin, c_order, cv)
        for n in range(len(sv)):
            assert cv[cut.net_map[n]] & mask == sv[n] & mask, (t, n)
        d_vals = [sv[seq.fanin[seq.fanin_ptr[g]]] for g in ff]
        assert [cv[x] for x in cut.ppo] == d_vals
        state = d_vals  # the flops load their D inputs


def test_cut_breaks_sequential_loops_and_shares_streams():
    seq = synth.random_seq_dag(synth.DagSpec(n_gates=600, n_pi=16, depth=10), 24, 9, shared=0.3)
    cut = synth.cut_flops(seq)
    nl = cut.netlist
    oracle.Netlist.of(nl)  # acyclic, or the constructor raises
    # some flop's D depends on a flop output: the cut broke a sequential loop
    reach = np.zeros(nl.n_nets, bool)
    reach[cut.ppi] = True
    for g in _comb_order(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin, np.zeros(nl.n_gates, bool)):
        reach[nl.n_pi + g] = reach[nl.fanin[nl.fanin_ptr[g]:nl.fanin_ptr[g + 1]]].any()
    assert reach[cut.ppo].any()
    # streams: PIs their own; pseudo-PIs of flops with one D net share the first's
    ff = np.nonzero(seq.op == synth.DFF)[0]
    d = [int(seq.fanin[seq.fanin_ptr[g]]) for g in ff]
    np.testing.assert_array_equal(cut.stream[: seq.n_pi], np.arange(seq.n_pi))
    for k in range(len(ff)):
        first = d.index(d[k])
        assert cut.stream[seq.n_pi + k] == seq.n_pi + first
    assert len(set(d)) < len(d)  # the generator made some drivers shared


def test_netlist_without_flops_cuts_to_itself():
    nl = synth.random_dag(synth.DagSpec(n_gates=200, n_pi=8, depth=6), 2)
    seq = synth.SeqNetlist(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin)
    cut = synth.cut_flops(seq)
    np.testing.assert_array_equal(cut.netlist.op, nl.op)
    np.testing.assert_array_equal(cut.netlist.fanin, nl.fanin)
    np.testing.assert_array_equal(cut.net_map, np.arange(nl.n_nets))
    assert cut.ppi.size == 0 and cut.ppo.size == 0
