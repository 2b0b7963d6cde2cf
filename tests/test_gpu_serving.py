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
             synth.DagSpec(n_gates=20000, n_pi=256, depth=25)]
    nls = [synth.random_dag(s, 40 + i) for i, s in enumerate(specs)]
    designs = [api.Design(ctx, nl) for nl in nls]
    caps = [synth.net_caps(nl.n_nets, 50 + i) for i, nl in enumerate(nls)]
    return ctx, nls, designs, caps


def _queries(nls, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        i = int(rng.integers(0, len(nls)))
        nl = nls[i]
        p = rng.uniform(0.1, 0.9, nl.n_pi).astype(np.float32)
        s = np.array([0.5, 1, 2, 4], np.float32)[rng.integers(0, 4, nl.n_gates)]
        out.append((i, p, s, bool(rng.integers(0, 2))))
    return out


@pytest.mark.parametrize("mode", [L.DP_MODELED, L.DP_FROZEN_BETA])
def test_served_results_match_oracle_and_alone(setup, mode):
    ctx, nls, designs, caps = setup
    say(f"serving mode {mode}")
    srv = api.Server(ctx, hbm_budget_bytes=256 << 20, max_batch=16, max_inflight=4)
    ids = [srv.add_design(d, c, mode=mode, n_sim=64 * 64, seed=5) for d, c in zip(designs, caps)]
    qs = _queries(nls, 60, seed=mode)
    # alone: one at a time
    alone = []
    for (i, p, s, bwd) in qs[:12]:
        alone.append(srv.wait(srv.submit(ids[i], p, s, bwd)))
    # mixed: a burst from two client threads, so queries queue behind the
    # sweeps already on the device and get batched
    tickets = [None] * len(qs)

    def client(lo, hi):
        for k in range(lo, hi):
            i, p, s, bwd = qs[k]
            tickets[k] = srv.submit(ids[i], p, s, bwd)
    th = [threading.Thread(target=client, args=(0, 30)), threading.Thread(target=client, args=(30, 60))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    mixed = [srv.wait(t) for t in tickets]
    st = srv.stats()
    assert st["completed"] == 72 and st["max_inflight"] >= 1
    assert st["device_steps"] < 72  # queries were batched
    for k in range(12):
        assert alone[k][0] == mixed[k][0]
        if qs[k][3]:
            np.testing.assert_array_equal(alone[k][1], mixed[k][1])
    # against the oracle, with the design's frozen beta for DP_FROZEN_BETA
    for k in range(0, 60, 7):
        i, p, s, bwd = qs[k]
        o = oracle.Netlist.of(nls[i])
        if mode == L.DP_FROZEN_BETA:
            f0 = o.forward(np.full(nls[i].n_pi, 0.5, np.float32), caps[i], hybrid=True,
                           n_words=64, seed=5)
            beta = f0["beta"].astype(np.float32).astype(np.float64)
            f, adj = oracle_column(o, p, caps[i], s, mode="frozen", beta=beta)
            rel = 2e-4  # beta enters as its float32 calibration
        else:
            f, adj = oracle_column(o, p, caps[i], s)
            rel = None
        if rel:
            np.testing.assert_allclose(mixed[k][0], f["power"], rtol=rel)
        else:
            assert_power_close(mixed[k][0], f["power"])
            if bwd:
                assert_grad_close(mixed[k][1], adj["dpi"], "served dP/dp")
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
