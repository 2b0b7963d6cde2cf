"""Serving: queries against device-resident designs, batched as they arrive.
Each result must equal the oracle and be identical alone and in the mix."""
from __future__ import annotations

import threading

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import assert_grad_close, assert_power_close, oracle_column, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    ctx = api.Context(0)
    specs = [synth.DagSpec(n_gates=3000, n_pi=64, depth=20),
             synth.DagSpec(n_gates=9000, n_pi=128, depth=30),
             synth.DagSpec(n_gates=20000, n_pi=256, depth=25),
             synth.DagSpec(n_gates=50000, n_pi=1024, depth=45)]
    nls = [synth.random_dag(s, 40 + i) for i, s in enumerate(specs)]
    designs = [api.Design(ctx, nl) for nl in nls]
    caps = [synth.net_caps(nl.n_nets, 50 + i) for i, nl in enumerate(nls)]
    return ctx, nls, designs, caps


def _queries(nls, n, seed):
    """The benchmark's mix: design uniform, half forward and half
    forward+backward, each query with its own p ~ U(0.1, 0.9) and per-gate
    size factors from {0.5, 1, 2, 4}, Poisson arrival gaps."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        i = int(rng.integers(0, len(nls)))
        nl = nls[i]
        p = rng.uniform(0.1, 0.9, nl.n_pi).astype(np.float32)
        s = np.array([0.5, 1, 2, 4], np.float32)[rng.integers(0, 4, nl.n_gates)]
        out.append((i, p, s, bool(rng.integers(0, 2)), float(rng.exponential(1.0 / 2000.0))))
    return out


N_QUERIES = 200


@pytest.mark.parametrize("mode", [L.DP_MODELED, L.DP_FROZEN_BETA])
def test_served_results_match_oracle_and_alone(setup, mode):
    """200 queries, each alone (one at a time) and in a mix submitted by two
    clients at Poisson times: bit for bit the same; every one against the
    oracle (power 1e-5 relative, dP/dp 1e-4 relative with the floor), in
    DP_FROZEN_BETA with the oracle's own calibration (its own 64-word
    simulation at p = 1/2 on the same seed), not the server's."""
    import time

    ctx, nls, designs, caps = setup
    say(f"serving mode {mode}")
    srv = api.Server(ctx, hbm_budget_bytes=256 << 20, max_batch=16, max_inflight=4)
    ids = [srv.add_design(d, c, mode=mode, n_sim=64 * 64, seed=5) for d, c in zip(designs, caps)]
    qs = _queries(nls, N_QUERIES, seed=mode)
    alone = [srv.wait(srv.submit(ids[i], p, s, bwd)) for (i, p, s, bwd, _) in qs]
    tickets = [None] * len(qs)

    def client(ks):
        t0 = time.perf_counter()
        due = 0.0
        for k in ks:
            i, p, s, bwd, gap = qs[k]
            due += 2 * gap  # each client carries half of the arrivals
            while time.perf_counter() - t0 < due:
                pass
            tickets[k] = srv.submit(ids[i], p, s, bwd)
    th = [threading.Thread(target=client, args=(range(0, N_QUERIES, 2),)),
          threading.Thread(target=client, args=(range(1, N_QUERIES, 2),))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    mixed = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["completed"] == 2 * N_QUERIES and st["max_inflight"] >= 1
    say(f"serving mode {mode}: {st['device_steps']} device steps for {2 * N_QUERIES} queries")
    assert st["device_steps"] < 2 * N_QUERIES  # queries were batched
    for k in range(N_QUERIES):
        assert alone[k][0] == mixed[k][0], f"query {k}: power alone {alone[k][0]} mixed {mixed[k][0]}"
        if qs[k][3]:
            np.testing.assert_array_equal(alone[k][1], mixed[k][1])
    orc = [oracle.Netlist.of(nl) for nl in nls]
    betas = [None] * len(nls)
    if mode == L.DP_FROZEN_BETA:
        for i, nl in enumerate(nls):
            f0 = orc[i].forward(np.full(nl.n_pi, 0.5, np.float32), caps[i], hybrid=True,
                                n_words=64, seed=5)
            betas[i] = f0["beta"]
    for k in range(N_QUERIES):
        i, p, s, bwd, _ = qs[k]
        if mode == L.DP_FROZEN_BETA:
            f, adj = oracle_column(orc[i], p, caps[i], s, mode="frozen", beta=betas[i])
        else:
            f, adj = oracle_column(orc[i], p, caps[i], s)
        assert_power_close(mixed[k][0], f["power"], f"served power of query {k}")
        if bwd:
            assert_grad_close(mixed[k][1], adj["dpi"], f"served dP/dp of query {k}")
    srv.close()


def test_budget_rejection_and_errors(setup):
    ctx, nls, designs, caps = setup
    say("serving budget")
    srv = api.Server(ctx, hbm_budget_bytes=4096)
    did = srv.add_design(designs[2], caps[2])
    with pytest.raises(L.DiffPowerError, match="BUDGET"):
        srv.submit(did, np.full(nls[2].n_pi, 0.5, np.float32))
    with pytest.raises(L.DiffPowerError, match="NOTFOUND"):
        srv.wait(12345)
    srv.close()
    srv = api.Server(ctx, hbm_budget_bytes=64 << 20)
    did = srv.add_design(designs[0], caps[0])
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        srv.submit(did, np.full(nls[0].n_pi, 2.0, np.float32))
    bad = np.ones(nls[0].n_gates, np.float32)
    bad[7] = np.nan
    t_bad = srv.submit(did, np.full(nls[0].n_pi, 0.5, np.float32), bad)
    t_ok = srv.submit(did, np.full(nls[0].n_pi, 0.5, np.float32))
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        srv.wait(t_bad)
    assert srv.wait(t_ok)[0] > 0
    srv.close()
