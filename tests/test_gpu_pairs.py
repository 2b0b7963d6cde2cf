"""Modeled sweeps that run two SP levels per launch (the second level's lanes
recompute the pins the first level drives) against the FP64 oracle, and bit
for bit against other pairings of the same levels: a design alone pairs
every two levels that hold fixed cells only, a merged group only the level
indices every design in it can pair, so the two pair different levels."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import SP_ABS, assert_grad_close, assert_power_close, oracle_column, say

pytestmark = pytest.mark.gpu

# library cells of arity 1, 2 and 3 swapped in for fixed cells of the same arity
SWAP_CELLS = ("1^A", "!(A^B)", "!((A1|A2)&B)")


@pytest.fixture(scope="module")
def ctx():
    return api.Context(0)


def _with_cells_at(nl, levels, seed):
    """nl with every gate on the given levels made a library cell of the same
    arity (so those levels cannot pair)."""
    lv = oracle.Netlist.of(nl).levels()
    ar = np.diff(nl.fanin_ptr)
    op = nl.op.astype(np.int32).copy()
    rng = np.random.default_rng(seed)
    for g in range(nl.n_gates):
        if lv[nl.n_pi + g] in levels and rng.random() < 0.5:
            op[g] = synth.CELL_BASE + int(ar[g]) - 1
    return dataclasses.replace(nl, op=op.astype(np.uint8), cells=SWAP_CELLS)


@pytest.mark.parametrize("B", [1, 5])
def test_pairs_around_library_levels_match_oracle(ctx, B):
    say(f"paired SP levels around library-cell levels, B={B}")
    nl = _with_cells_at(synth.random_dag(synth.DagSpec(n_gates=3000, n_pi=64, depth=16), 31),
                        {5, 6, 11}, 32)
    assert (nl.op >= synth.CELL_BASE).any()
    p = synth.pi_probs(nl.n_pi, 33, batch=B)
    cap = synth.net_caps(nl.n_nets, 34)
    d = api.Design(ctx, nl)
    res = {}
    for sched in (L.DP_SCHED_LEVEL, L.DP_SCHED_GRAPH):
        ev = api.Eval(d, B)
        ev.set_pi_prob(p)
        ev.set_caps(cap)
        ev.set_schedule(sched)
        r = ev.forward(("sp", "power"))
        r.update(ev.backward(want=("dpi", "dcap")))
        res[sched] = r
    for k in res[L.DP_SCHED_LEVEL]:
        np.testing.assert_array_equal(res[L.DP_SCHED_LEVEL][k], res[L.DP_SCHED_GRAPH][k], err_msg=k)
    r = res[L.DP_SCHED_LEVEL]
    o = oracle.Netlist.of(nl)
    dcap = np.zeros(nl.n_nets)
    for b in range(B):
        f, adj = oracle_column(o, p[b], cap)
        np.testing.assert_allclose(r["sp"][b], f["sp"], atol=SP_ABS, rtol=0)
        assert_power_close(r["power"][b], f["power"], f"power[{b}]")
        assert_grad_close(r["dpi"][b], adj["dpi"], f"dP/dp[{b}]")
        dcap += adj["dcap"]
    assert_grad_close(r["dcap"], dcap, "dP/dC")


def test_group_pairs_other_levels_bit_for_bit(ctx):
    """Three designs (library cells on some levels, fixed cells only, and a
    shallower one) alone and as one merged group: the same bits, although
    the group pairs a level index only where all three can."""
    say("paired SP levels: group against alone")
    nls = [_with_cells_at(synth.random_dag(synth.DagSpec(n_gates=3000, n_pi=64, depth=16), 41),
                          {3, 8, 9}, 42),
           synth.random_dag(synth.DagSpec(n_gates=2500, n_pi=48, depth=17), 43),
           synth.random_dag(synth.DagSpec(n_gates=900, n_pi=32, depth=7), 44)]
    evs, alone = [], []
    for i, nl in enumerate(nls):
        d = api.Design(ctx, nl)
        ev = api.Eval(d, 3)
        ev.set_pi_prob(synth.pi_probs(nl.n_pi, 45 + i, batch=3))
        ev.set_caps(synth.net_caps(nl.n_nets, 48 + i))
        r = ev.forward(("sp", "power"))
        r.update(ev.backward(want=("dpi",)))
        alone.append(r)
        evs.append(ev)
    grp = api.Group(ctx, evs)
    for _ in range(2):  # the group's captured graph replays: more than one launch
        res = grp.run(("sp", "power"), backward=True)
        for i, (r, a) in enumerate(zip(res, alone)):
            for k in ("sp", "power", "dpi"):
                np.testing.assert_array_equal(r[k], a[k], err_msg=f"design {i}: {k}")
    grp.close()
