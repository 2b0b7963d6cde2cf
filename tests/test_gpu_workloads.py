"""Parity at the full workload sizes, in the launch configuration bench.py
times: the 117K-gate design with 65,536 vectors and finite differences, the
1M-gate bench design with 65,536 vectors (every net, counts bit-exact)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, rank, synth
from tests.gpu_helpers import (SP_ABS, assert_beta_close, assert_grad_close, assert_power_close,
                               say)
from oracle.parallel import sim_counts

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def ctx():
    return api.Context(0)


def _full_check(ctx, name, n_sim, seed, fd_samples=0, tilings=(), schedules=()):
    spec = synth.SPECS[name]
    nl = synth.random_dag(spec, seed=1)
    p = synth.pi_probs(nl.n_pi, seed=2)
    cap = synth.net_caps(nl.n_nets, seed=3)
    T = n_sim // 64
    say(f"{name}: GPU hybrid fwd+bwd, {T} words")
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 1, mode=L.DP_HYBRID, n_sim=n_sim, seed=seed)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    res = ev.forward(("sp", "tr", "tr_acc", "tr_hyb", "beta", "ones", "toggles", "power"))
    g = ev.backward(want=("dpi", "dcap"))
    say(f"{name}: oracle")
    o = oracle.Netlist.of(nl)
    ones, tog = sim_counts(nl, p[0], T, seed)
    P = o.sp(p[0].astype(np.float64))
    f = {**o.power(P, cap, hybrid=True, ones=ones, toggles=tog, n_words=T), "sp": P}
    adj = o.adjoint(P, f["beta"], cap)
    np.testing.assert_array_equal(res["ones"][0].astype(np.uint64), ones)
    np.testing.assert_array_equal(res["toggles"][0].astype(np.uint64), tog)
    np.testing.assert_allclose(res["sp"][0], P, atol=SP_ABS, rtol=0)
    np.testing.assert_allclose(res["tr"][0], f["tr_model"], atol=SP_ABS, rtol=0)
    np.testing.assert_allclose(res["tr_acc"][0], f["tr_acc"], atol=SP_ABS, rtol=0)
    np.testing.assert_allclose(res["tr_hyb"][0], f["tr_hyb"], atol=SP_ABS, rtol=0)
    assert_beta_close(res["beta"][0], res["tr"][0], f, f"{name} beta")
    assert_power_close(res["power"], f["power"], f"{name} power")
    assert_grad_close(g["dpi"][0], adj["dpi"], f"{name} dP/dp")
    assert_grad_close(g["dcap"], adj["dcap"], f"{name} dP/dC")
    for ppl in tilings:  # other launch tilings: the same results bit for bit
        say(f"{name}: per-level launches, {ppl} word pairs per lane")
        ev.set_schedule(L.DP_SCHED_LEVEL, 0, ppl)
        r2 = ev.forward(("ones", "toggles", "sp", "power"))
        g2 = ev.backward(want=("dpi", "dcap"))
        for k in r2:
            np.testing.assert_array_equal(r2[k], res[k], err_msg=f"{k} at {ppl} pairs per lane")
        for k in g2:
            np.testing.assert_array_equal(g2[k], g[k], err_msg=f"{k} at {ppl} pairs per lane")
    for sched in schedules:  # the other schedules the benchmark times: bit for bit
        say(f"{name}: schedule {sched}")
        ev.set_schedule(sched)
        for rep in range(2):  # a captured graph replays: check more than one launch
            r2 = ev.forward(("ones", "toggles", "sp", "power"))
            g2 = ev.backward(want=("dpi", "dcap"))
            for k in r2:
                np.testing.assert_array_equal(r2[k], res[k], err_msg=f"{k}, schedule {sched}")
            for k in g2:
                np.testing.assert_array_equal(g2[k], g[k], err_msg=f"{k}, schedule {sched}")
    if fd_samples:
        # FP64 central differences of the oracle's frozen-beta power, h = 1e-6
        rng = np.random.default_rng(7)
        idx = rng.choice(nl.n_pi, fd_samples, replace=False)
        h = 1e-6
        p64 = p[0].astype(np.float64)
        fd = np.zeros(fd_samples)
        for k, i in enumerate(idx):
            e = np.zeros_like(p64)
            e[i] = h
            fd[k] = (o.frozen_power(p64 + e, f["beta"], cap)
                     - o.frozen_power(p64 - e, f["beta"], cap)) / (2 * h)
        rounding = 4 * np.finfo(np.float64).eps * abs(f["power"]) / h
        err = np.abs(g["dpi"][0][idx] - fd)
        tol = 1e-4 * np.abs(fd) + 1e-6 * np.abs(adj["dpi"]).max() + rounding
        assert (err <= tol).all(), f"FD mismatch at {idx[err > tol][:5]}"
        # rank agreement of the GPU gradient with the differences (Sec. V-C)
        m = rank.agreement(g["dpi"][0][idx], fd, 20)
        say(f"{name}: rank agreement with FD on {fd_samples} PIs: {m}")
        assert m["pearson"] > 0.9999 and m["top_k_overlap"] >= 0.95


def test_dag117k_hybrid_fwd_bwd_with_fd():
    """117,000 gates, 2,048 PIs, depth 60, 65,536 vectors; FD on 200 PIs."""
    _full_check(api.Context(0), "dag117k", 65536, seed=11, fd_samples=200)


def test_dag1m_bench_configuration():
    """The bench workload: 1M gates, 8,192 PIs, depth 100, 65,536 vectors,
    default schedule; every net's counts bit-exact; then the tilings the
    benchmark chooses among (per-level launches of whole rows on one
    stream, 2, 4 or 8 word pairs per lane) give the same results."""
    _full_check(api.Context(0), "dag1m", 65536, seed=1, tilings=(2, 4, 8))


def test_dag117k_sizing_sweep_spot_parity():
    """32 PI vectors x 256 size vectors on the 117K-gate design, hybrid with
    65,536 vectors: power[b][s] and the per-(b, s) gradients of 64 random
    (b, s) pairs against the oracle."""
    ctx = api.Context(0)
    nl = synth.random_dag(synth.SPECS["dag117k"], seed=1)
    B, S, T = 32, 256, 1024
    p = synth.pi_probs(nl.n_pi, seed=5, batch=B, lo=0.05, hi=0.95)
    cap = synth.net_caps(nl.n_nets, seed=6)
    size = synth.cell_sizes(nl.n_gates, seed=7, n_size=S)
    say("sizing sweep: GPU")
    d = api.Design(ctx, nl)
    ev = api.Eval(d, B, S, mode=L.DP_HYBRID, n_sim=64 * T, seed=1)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    ev.set_cell_sizes(size)
    power = ev.forward(("power",))["power"]
    cols = ev.backward_columns()
    # the whole sweep captured as two graph launches, and as one, as the
    # benchmark also times it, gives the same results bit for bit (the autotuner's own pick
    # is checked in a process of its own: test_gpu_autotune.py)
    say("sizing sweep: graph schedule")
    ev.set_schedule(L.DP_SCHED_GRAPH)
    for _ in range(2):
        np.testing.assert_array_equal(ev.forward(("power",))["power"], power)
        np.testing.assert_array_equal(ev.backward_columns(), cols)
    say("sizing sweep: forward and reverse as one graph launch")
    for _ in range(2):
        pw, g = ev.forward_backward_columns()
        np.testing.assert_array_equal(pw, power)
        np.testing.assert_array_equal(g, cols)
    o = oracle.Netlist.of(nl)
    rng = np.random.default_rng(3)
    for b in rng.choice(B, 4, replace=False):
        say(f"sizing sweep: oracle column {b}")
        ones, tog = sim_counts(nl, p[b], T, 1)
        P = o.sp(p[b].astype(np.float64))
        for s_ in rng.choice(S, 16, replace=False):
            f = o.power(P, cap, size[s_], hybrid=True, ones=ones, toggles=tog, n_words=T)
            adj = o.adjoint(P, f["beta"], cap, size[s_])
            assert_power_close(power[b, s_], f["power"], f"power[{b},{s_}]")
            assert_grad_close(cols[b, s_], adj["dpi"], f"dP/dp[{b},{s_}]")


def test_dag2m_scale_chunked():
    """2M gates, 16,384 PIs, depth 120, 262,144 vectors in word chunks: every
    net's counts bit-exact, SP/TR, power and gradients; the captured graph
    and the persistent reverse sweep give the same results bit for bit."""
    _full_check(api.Context(0), "dag2m", 262144, seed=1,
                schedules=(L.DP_SCHED_GRAPH, L.DP_SCHED_PERSISTENT))
