"""Design groups: several designs of uneven size in one unit (one captured
graph, or one branch per eval when the unit is large) give every eval's
results bit for bit as that eval alone."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

OUT = ("sp", "tr", "power")


def _make(ctx, specs):
    evs, designs = [], []
    for k, (spec, seed, B, mode) in enumerate(specs):
        nl = synth.random_dag(synth.SPECS[spec], seed)
        d = api.Design(ctx, nl)
        ev = api.Eval(d, B, mode=mode, n_sim=64 * 24, seed=seed)
        ev.set_pi_prob(synth.pi_probs(nl.n_pi, 100 + k, batch=B))
        ev.set_caps(synth.net_caps(nl.n_nets, 200 + k))
        designs.append(d)
        evs.append(ev)
    return designs, evs


def _alone(ev):
    ev.set_schedule(L.DP_SCHED_LEVEL)
    r = ev.forward(OUT)
    r.update(ev.backward(want=("dpi",)))
    return r


def _check(got, want):
    for k in want:
        np.testing.assert_array_equal(got[k], want[k], err_msg=k)


def test_group_of_uneven_designs_matches_alone():
    say("group: 3 designs, graph")
    ctx = api.Context(0)
    specs = [("dag2k", 1, 2, L.DP_MODELED), ("dag10k", 2, 1, L.DP_HYBRID),
             ("dag2k", 3, 3, L.DP_HYBRID)]
    designs, evs = _make(ctx, specs)
    want = [_alone(ev) for ev in evs]
    grp = api.Group(ctx, evs)
    for rep in range(3):  # first run captures, later runs replay
        got = grp.run(OUT, backward=True)
        for g, w in zip(got, want):
            _check(g, w)
    # new inputs reach the replayed graph
    evs[0].set_pi_prob(synth.pi_probs(designs[0].n_pi, 999, batch=2))
    want0 = _alone(evs[0])
    got = grp.run(OUT, backward=True)
    _check(got[0], want0)
    _check(got[1], want[1])
    # direct enqueue, and other branch counts: same results
    for use_graph, branches in ((False, 0), (False, 1), (True, 2), (True, 1)):
        grp.configure(use_graph=use_graph, max_branches=branches)
        got = grp.run(OUT, backward=True)
        _check(got[0], want0)
        _check(got[1], want[1])
        _check(got[2], want[2])
    grp.configure()
    # forward only, device outputs
    import torch
    got = grp.run(("power",), backward=False, device=True)
    ctx.synchronize()  # the context's own stream is not torch's
    np.testing.assert_array_equal(got[2]["power"].cpu().numpy(), want[2]["power"])
    grp.close()


def test_large_group_runs_on_branches():
    """More launches than a graph holds: the unit is enqueued branch by
    branch, results unchanged."""
    say("group: 12 evals, direct")
    ctx = api.Context(0)
    specs = [("dag2k", 10 + k, 4, L.DP_HYBRID) for k in range(12)]
    _, evs = _make(ctx, specs)
    want = [_alone(ev) for ev in evs]
    grp = api.Group(ctx, evs)
    got = grp.run(OUT, backward=True)
    for g, w in zip(got, want):
        _check(g, w)
    grp.close()


def test_group_errors():
    ctx = api.Context(0)
    other = api.Context(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 1)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 1)
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        api.Group(other, [ev])
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        api.Group(ctx, [ev, ev])
    grp = api.Group(ctx, [ev])
    with pytest.raises(L.DiffPowerError, match="STATE"):
        grp.run()


def test_merged_level_launches_match_alone():
    """Modeled evals of four designs share one launch per level index (and
    one per reverse level): each eval's SP, power and dP/dp equal its own
    sweep bit for bit, with and without graph capture, for one and many
    columns and both beta-gradient rules."""
    say("group: merged modeled levels")
    ctx = api.Context(0)
    specs = [("dag2k", 21, 2, L.DP_MODELED), ("dag10k", 22, 1, L.DP_MODELED),
             ("dag2k", 23, 40, L.DP_MODELED), ("dag50k", 24, 1, L.DP_MODELED),
             ("dag2k", 25, 1, L.DP_HYBRID)]
    designs, evs = _make(ctx, specs)
    evs[1].set_params(mode=L.DP_MODELED, beta_grad=L.DP_BETA_STE)
    want = [_alone(ev) for ev in evs]
    grp = api.Group(ctx, evs)
    for use_graph in (True, False):
        grp.configure(use_graph=use_graph)
        for _ in range(2):
            got = grp.run(OUT, backward=True)
            for g, w in zip(got, want):
                _check(g, w)
    grp.close()
