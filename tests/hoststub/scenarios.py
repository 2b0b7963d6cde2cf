"""Host-logic scenarios run against the CPU stand-in runtime.

    python -m tests.hoststub.scenarios <libdp_stub.so> <scenario>

Prints one JSON line of results.  The library's host code runs for real
(compile and levelization, validation, schedules and graph capture
bookkeeping, merged level tables, the serving scheduler); the stand-in
launchers check each launch's extents and compute nothing, so numerical
outputs are placeholders and only flows, status codes and host-computed
structure are checked."""
from __future__ import annotations

import dataclasses
import json
import sys

import numpy as np

from paper_2608_03778_amd import _lib

_lib._settle_hip_runtime = lambda: None  # the stand-in runtime only, never a real one
_lib.load(sys.argv[1])

import oracle  # noqa: E402
from paper_2608_03778_amd import _lib as L, api, synth  # noqa: E402


def status_of(fn, *a, **kw):
    """Status name and message of a call ("OK" when it succeeds)."""
    try:
        fn(*a, **kw)
        return "OK", ""
    except L.DiffPowerError as e:
        return L.STATUS_NAMES.get(e.status, str(e.status)), str(e)


def mixed_spec(n_gates, n_pi, depth):
    ops = tuple(range(9)) + tuple(synth.CELL_BASE + c for c in range(len(synth.LIBRARY)))
    return synth.DagSpec(n_gates=n_gates, n_pi=n_pi, depth=depth, ops=ops, cells=synth.LIBRARY)


def scenario_compile(ctx):
    out = {}
    nets = {
        "fixed": synth.random_dag(synth.SPECS["dag2k"], 3),
        "library": synth.random_dag(mixed_spec(3000, 64, 18), 4),
        "flop_cut": synth.cut_flops(synth.random_seq_dag(synth.DagSpec(n_gates=1500, n_pi=20,
                                                                       depth=12), 30, 5)).netlist,
        "tree": synth.random_tree(40, 6, cells=synth.LIBRARY,
                                  ops=tuple(range(9)) + (synth.CELL_BASE, synth.CELL_BASE + 4)),
    }
    for name, nl in nets.items():
        d = api.Design(ctx, nl)
        lv = d.levels()
        ref = oracle.Netlist.of(nl).levels()
        out[f"{name}_levels_match"] = bool(np.array_equal(lv, ref))
        out[f"{name}_depth_match"] = int(d.depth) == int(ref.max())
        d.close()
    # fixed cells written as expressions compile to the same levels
    nl = synth.random_dag(synth.DagSpec(n_gates=800, n_pi=32, depth=10, ops=tuple(range(8))), 7)
    expr = dataclasses.replace(nl, op=(nl.op.astype(np.int32) + synth.CELL_BASE).astype(np.uint8),
                               cells=("!A", "A", "A&B", "A|B", "!(A&B)", "!(A|B)", "A^B",
                                      "!(A&B|C)"))
    out["expressions_levels_match"] = bool(np.array_equal(api.Design(ctx, nl).levels(),
                                                          api.Design(ctx, expr).levels()))
    # errors
    cyc = synth.from_gates(2, [(synth.AND2, [0, 3]), (synth.INV, [2])])
    out["cycle"] = status_of(api.Design, ctx, cyc)[0]
    bad_arity = synth.from_gates(2, [(synth.AND2, [0])])
    out["bad_arity"] = status_of(api.Design, ctx, bad_arity)[0]
    bad_op = synth.from_gates(2, [(12, [0, 1])])
    out["bad_op"] = status_of(api.Design, ctx, bad_op)[0]
    bad_net = synth.from_gates(2, [(synth.AND2, [0, 7])])
    out["bad_net"] = status_of(api.Design, ctx, bad_net)[0]
    one = synth.from_gates(3, [(synth.CELL_BASE, [0, 1])], ("A&B",))
    msgs = {}
    for text in ("A&", "(A|B", "A $ B", "A B", "a&b&c&d&e&f&g", "&".join(["A"] * 20),
                 "A|(B|(C|(D|(E|(F|(A|(B|C)))))))", "1"):
        st, msg = status_of(api.Design, ctx, dataclasses.replace(one, cells=(text,)))
        msgs[text] = [st, msg]
    out["parse"] = msgs
    out["cell_arity"] = status_of(api.Design, ctx, dataclasses.replace(one, cells=("A&B&C",)))[0]
    out["cell_missing"] = status_of(api.Design, ctx, dataclasses.replace(one, cells=()))[0]
    return out


def scenario_flows(ctx):
    out = {}
    for name, nl in (("fixed", synth.random_dag(synth.SPECS["dag2k"], 8)),
                     ("library", synth.random_dag(mixed_spec(2500, 48, 14), 9))):
        d = api.Design(ctx, nl)
        cap = synth.net_caps(nl.n_nets, 1)
        runs = 0
        for mode in (L.DP_MODELED, L.DP_HYBRID, L.DP_FROZEN_BETA):
            for B, S in ((1, 0), (3, 2)):
                ev = api.Eval(d, B, S, mode=mode, n_sim=64 * 40, seed=2)
                ev.set_pi_prob(synth.pi_probs(nl.n_pi, 3, batch=B))
                ev.set_caps(cap)
                if S:
                    ev.set_cell_sizes(synth.cell_sizes(nl.n_gates, 4, n_size=S))
                if mode == L.DP_FROZEN_BETA:
                    ev.set_beta(np.ones((B, nl.n_nets), np.float32))
                scheds = [(L.DP_SCHED_LEVEL, 0, 0, 1), (L.DP_SCHED_GRAPH, 0, 0, 1)]
                if mode == L.DP_HYBRID:
                    scheds += [(L.DP_SCHED_LEVEL, 8, 2, 2), (L.DP_SCHED_LEVEL, 6, 1, 3)]
                    if B > 1:  # ragged column groups, alone and with chunks on streams
                        ev.set_sim_columns(2)
                        for chunk, lanes in ((0, 1), (8, 2)):
                            ev.set_schedule(L.DP_SCHED_LEVEL, chunk, 0)
                            ev.set_sim_streams(lanes)
                            ev.forward(("sp", "tr", "power"))
                            runs += 1
                        ev.set_sim_columns(0)
                if name == "fixed":
                    scheds += [(L.DP_SCHED_PERSISTENT, 0, 0, 1)]
                for sched, chunk, ppl, lanes in scheds:
                    ev.set_schedule(sched, chunk, ppl)
                    ev.set_sim_streams(lanes)
                    ev.forward(("sp", "tr", "power"))
                    ev.backward(want=("dpi", "dcap") + (("dsize",) if S else ()))
                    runs += 1
                # a sizing sweep's two sweeps in one call: one captured graph
                # (twice: the second replays it), then the plain calls
                for sched in (L.DP_SCHED_GRAPH, L.DP_SCHED_GRAPH, L.DP_SCHED_LEVEL):
                    ev.set_schedule(sched)
                    ev.set_sim_streams(1)
                    ev.forward_backward_columns()
                    runs += 1
                ev.set_schedule(L.DP_SCHED_LEVEL)
                ev.set_sim_streams(1)
                ev.power_gradients()
                if mode == L.DP_HYBRID and S == 0:
                    tau = np.full((B, nl.n_pi), 0.3, np.float32)
                    ev.set_pi_rates(tau)
                    ev.set_pi_streams((np.arange(nl.n_pi) // 2 * 2).astype(np.int32))
                    ev.set_pi_fixed(np.arange(nl.n_pi) % 5 == 0)
                    for sched, chunk in ((L.DP_SCHED_LEVEL, 0), (L.DP_SCHED_GRAPH, 0),
                                         (L.DP_SCHED_LEVEL, 8)):
                        ev.set_schedule(sched, chunk)
                        ev.forward(("power",))
                        ev.backward(want=("dpi",))
                        runs += 1
                    ev.set_pi_rates(None)
                    ev.set_pi_streams(None)
                    ev.set_pi_fixed(None)
                if mode == L.DP_MODELED and S == 0:
                    ev.power_virus(3, 1e-3)
                    runs += 1
                ev.close()
        out[f"{name}_runs"] = runs
        # validation and state errors
        ev = api.Eval(d, 2, mode=L.DP_HYBRID, n_sim=256)
        out[f"{name}_backward_first"] = status_of(ev.backward, want=("dpi",))[0]
        out[f"{name}_forward_no_inputs"] = status_of(ev.forward, ("power",))[0]
        bad_p = np.full((2, nl.n_pi), 0.5, np.float32)
        bad_p[1, 3] = 1.5
        out[f"{name}_p_range"] = status_of(ev.set_pi_prob, bad_p)[0]
        bad_c = cap.copy()
        bad_c[5] = -1.0
        out[f"{name}_cap_range"] = status_of(ev.set_caps, bad_c)[0]
        out[f"{name}_rates_range"] = status_of(ev.set_pi_rates,
                                               np.full((2, nl.n_pi), 1.5, np.float32))[0]
        out[f"{name}_streams_range"] = status_of(ev.set_pi_streams,
                                                 np.full(nl.n_pi, nl.n_pi, np.int32))[0]
        out[f"{name}_schedule_bad"] = status_of(ev.set_schedule, 9)[0]
        out[f"{name}_persistent"] = status_of(ev.set_schedule, L.DP_SCHED_PERSISTENT)[0]
        ev.set_pi_prob(np.full((2, nl.n_pi), 0.5, np.float32))
        ev.set_caps(cap)
        out[f"{name}_virus_hybrid"] = status_of(ev.power_virus, 2, 0.1)[0]
        ev.close()
        d.close()
    return out


def scenario_group_serving(ctx):
    out = {}
    nls = [synth.random_dag(mixed_spec(2000, 40, 12), 11),
           synth.random_dag(synth.SPECS["dag2k"], 12),
           synth.random_dag(synth.DagSpec(n_gates=5000, n_pi=80, depth=25), 13)]
    designs = [api.Design(ctx, nl) for nl in nls]
    caps = [synth.net_caps(nl.n_nets, 20 + i) for i, nl in enumerate(nls)]
    evs = []
    for i, (nl, d) in enumerate(zip(nls, designs)):
        mode = L.DP_HYBRID if i == 2 else L.DP_MODELED
        ev = api.Eval(d, 2, mode=mode, n_sim=64 * 20, seed=i)
        ev.set_pi_prob(synth.pi_probs(nl.n_pi, 30 + i, batch=2))
        ev.set_caps(caps[i])
        evs.append(ev)
    grp = api.Group(ctx, evs)
    for use_graph, branches in ((True, 0), (False, 1), (False, 0), (True, 2)):
        grp.configure(use_graph=use_graph, max_branches=branches)
        for backward in (False, True):
            res = grp.run(("sp", "power"), backward=backward)
    out["group_results"] = len(res)
    grp.close()
    srv = api.Server(ctx, hbm_budget_bytes=64 << 20, max_batch=8, max_inflight=3)
    ids = [srv.add_design(d, c, mode=L.DP_MODELED, n_sim=128, seed=5)
           for d, c in zip(designs, caps)]
    rng = np.random.default_rng(1)
    tickets = []
    for k in range(60):
        i = int(rng.integers(0, 3))
        size = None if k % 3 else np.ones(nls[i].n_gates, np.float32)
        tickets.append(srv.submit(ids[i], rng.uniform(0.1, 0.9, nls[i].n_pi).astype(np.float32),
                                  size, bool(k % 2)))
    done = sum(1 for t in tickets if srv.wait(t) is not None)
    st = srv.stats()
    out["served"] = done
    out["completed"] = st["completed"]
    out["batched"] = st["device_steps"] < 60
    bad = np.ones(nls[0].n_gates, np.float32)
    bad[3] = np.nan
    t_bad = srv.submit(ids[0], np.full(nls[0].n_pi, 0.5, np.float32), bad)
    out["nan_size"] = status_of(srv.wait, t_bad)[0]
    out["bad_p"] = status_of(srv.submit, ids[0], np.full(nls[0].n_pi, 2.0, np.float32))[0]
    out["unknown_ticket"] = status_of(srv.wait, 123456)[0]
    srv.close()
    tiny = api.Server(ctx, hbm_budget_bytes=4096)
    tid = tiny.add_design(designs[2], caps[2])
    out["budget"] = status_of(tiny.submit, tid, np.full(nls[2].n_pi, 0.5, np.float32))[0]
    tiny.close()
    return out


def scenario_capture_order(ctx):
    """The order in which a host crash was once seen on the GPU: design
    groups and serving, then the autotuner (graph candidates, several
    simulation streams) on a hybrid eval, in one process; then graph
    captures of multi-column hybrid sweeps and of a hybrid design group.
    The stand-in runtime checks every capture's forks and joins, the calls
    a capturing thread may not make, event reuse across captures, and that
    each graph launch touches only live allocations."""
    out = scenario_group_serving(ctx)
    nl = synth.random_dag(synth.SPECS["dag2k"], 13)
    d = api.Design(ctx, nl)
    cap = synth.net_caps(nl.n_nets, 14)
    for B in (1, 2, 3):
        ev = api.Eval(d, B, mode=L.DP_HYBRID, n_sim=64 * 512, seed=8)
        ev.set_pi_prob(synth.pi_probs(nl.n_pi, 13, batch=B))
        ev.set_caps(cap)
        ev.forward(("sp", "ones", "toggles", "power"))
        ev.autotune(2, with_backward=True)
        ev.forward(("sp", "ones", "toggles", "power"))
        ev.backward(want=("dpi",))
        for chunk, lanes in ((128, 2), (0, 1), (128, 3)):
            ev.set_schedule(L.DP_SCHED_GRAPH, chunk, 0)
            ev.set_sim_streams(lanes)
            ev.forward(("power",))
            ev.backward(want=("dpi",))
        ev.close()
    evs = []
    for i in range(3):
        e = api.Eval(d, 2, mode=L.DP_HYBRID if i else L.DP_MODELED, n_sim=64 * 16, seed=i)
        e.set_pi_prob(synth.pi_probs(nl.n_pi, 40 + i, batch=2))
        e.set_caps(cap)
        evs.append(e)
    grp = api.Group(ctx, evs)
    for use_graph in (True, False, True):
        grp.configure(use_graph=use_graph)
        grp.run(("power",), backward=True)
    grp.close()
    out["capture_order_done"] = True
    import ctypes
    counts = (ctypes.c_long * 3)()
    ctypes.CDLL(sys.argv[1]).stub_capture_counts(counts)
    out["captures"], out["forks"], out["graph_launches"] = counts[0], counts[1], counts[2]
    return out


if __name__ == "__main__":
    context = api.Context(0)
    result = {"compile": scenario_compile, "flows": scenario_flows,
              "group_serving": scenario_group_serving,
              "capture_order": scenario_capture_order}[sys.argv[2]](context)
    print(json.dumps(result), flush=True)
