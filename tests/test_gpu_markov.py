"""Startpoint stimulus model and sequential boundaries on the GPU, through the
C ABI, against the FP64 oracle: Markov chains with target transition rates
and shared streams (Sec. III-C) give the oracle's counts bit for bit;
startpoints excluded from the gradients get zero; a flop-cut sequential
netlist runs end to end."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import (SP_ABS, assert_beta_close, assert_grad_close, assert_power_close,
                               oracle_column, say)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return api.Context(0)


def _rates(p, frac, seed):
    """Rates in [0, 2 min(p, 1 - p)], a random fraction of the bound."""
    r = np.random.default_rng(seed).uniform(0, frac, p.shape)
    return (r * 2 * np.minimum(p, 1 - p)).astype(np.float32)


@pytest.mark.parametrize("sched,chunk,lanes,T", [(L.DP_SCHED_LEVEL, 0, 1, 300),
                                                 (L.DP_SCHED_GRAPH, 0, 1, 131),
                                                 (L.DP_SCHED_LEVEL, 64, 2, 300),
                                                 (L.DP_SCHED_LEVEL, 6, 3, 257)])
def test_markov_counts_match_oracle(ctx, sched, chunk, lanes, T):
    """B = 3 columns with their own rates, shared streams, ragged tiles of
    the word scan and chunk halos: every count bit-exact, every float output
    within its tolerance, gradients against the oracle."""
    say(f"markov sched={sched} chunk={chunk} lanes={lanes} T={T}")
    nl = synth.random_dag(synth.DagSpec(n_gates=2500, n_pi=64, depth=16), 31)
    B = 3
    p = synth.pi_probs(nl.n_pi, 32, batch=B)
    p[:, :4] = [0.0, 1.0, 0.5, 0.5]  # constants and a clock-like lane (tau = 1)
    tau = _rates(p, 1.0, 33)
    tau[:, 2] = 1.0
    stream = np.arange(nl.n_pi, dtype=np.int32)
    stream[10:20] = 10  # one shared stream
    cap = synth.net_caps(nl.n_nets, 34)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, B, mode=L.DP_HYBRID, n_sim=64 * T, seed=35)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    ev.set_pi_rates(tau)
    ev.set_pi_streams(stream)
    ev.set_schedule(sched, chunk)
    ev.set_sim_streams(lanes)
    res = ev.forward(("sp", "tr", "sp_acc", "tr_acc", "beta", "tr_hyb", "ones", "toggles",
                      "power"))
    g = ev.backward(want=("dpi",))
    o = oracle.Netlist.of(nl)
    for b in range(B):
        words = oracle.stimulus_model(p[b], 35, T, tau=tau[b], stream=stream)
        f, adj = oracle_column(o, p[b], cap, mode="hybrid", n_words=T, pi_words=words)
        np.testing.assert_array_equal(res["ones"][b].astype(np.uint64), f["ones"])
        np.testing.assert_array_equal(res["toggles"][b].astype(np.uint64), f["toggles"])
        np.testing.assert_allclose(res["sp"][b], f["sp"], atol=SP_ABS, rtol=0)
        np.testing.assert_allclose(res["tr_acc"][b], f["tr_acc"], atol=SP_ABS, rtol=0)
        np.testing.assert_allclose(res["tr_hyb"][b], f["tr_hyb"], atol=SP_ABS, rtol=0)
        assert_beta_close(res["beta"][b], res["tr"][b], f, f"beta[{b}]")
        assert_power_close(res["power"][b], f["power"], f"power[{b}]")
        assert_grad_close(g["dpi"][b], adj["dpi"], f"dP/dp[{b}]")
    # the shared stream with one (p, tau): identical PI words, so equal counts
    same = p.copy()
    same[:, 10:20] = p[:, 10:11]
    t_same = tau.copy()
    t_same[:, 10:20] = tau[:, 10:11]
    ev.set_pi_prob(same)
    ev.set_pi_rates(t_same)
    r2 = ev.forward(("ones", "toggles"))
    for b in range(B):
        assert (r2["ones"][b][10:20] == r2["ones"][b][10]).all()
        assert (r2["toggles"][b][10:20] == r2["toggles"][b][10]).all()
    # tau = 0 and tau = 1 at p = 1/2: no toggles, and every transition a toggle
    assert (res["toggles"][:, 0] == 0).all() and (res["toggles"][:, 1] == 0).all()
    assert (res["toggles"][:, 2] == 64 * (T - 1)).all()


def test_independence_rate_equals_independent_stimulus(ctx):
    """Rates 2p(1-p) at dyadic p: the Markov words are the independent
    generator's bit for bit (GPU against GPU), and the shared-stream map of
    the independent generator matches the oracle."""
    say("markov at the independence rate")
    nl = synth.random_dag(synth.DagSpec(n_gates=1500, n_pi=48, depth=12), 36)
    rng = np.random.default_rng(37)
    p = rng.choice(np.array([0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875], np.float32),
                   (2, nl.n_pi)).astype(np.float32)
    tau = (2 * p * (1 - p)).astype(np.float32)
    cap = synth.net_caps(nl.n_nets, 38)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 2, mode=L.DP_HYBRID, n_sim=64 * 100, seed=39)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    ind = ev.forward(("ones", "toggles", "power"))
    ev.set_pi_rates(tau)
    mk = ev.forward(("ones", "toggles", "power"))
    for k in ("ones", "toggles", "power"):
        np.testing.assert_array_equal(ind[k], mk[k], err_msg=k)
    ev.set_pi_rates(None)
    stream = (np.arange(nl.n_pi) // 3 * 3).astype(np.int32)
    ev.set_pi_streams(stream)
    sh = ev.forward(("ones", "toggles"))
    o = oracle.Netlist.of(nl)
    for b in range(2):
        ones, tog = o.sim(100, pi_words=oracle.stimulus_model(p[b], 39, 100, stream=stream))
        np.testing.assert_array_equal(sh["ones"][b].astype(np.uint64), ones)
        np.testing.assert_array_equal(sh["toggles"][b].astype(np.uint64), tog)


@pytest.mark.parametrize("mode", [L.DP_MODELED, L.DP_HYBRID])
def test_fixed_startpoints_are_excluded_from_gradients(ctx, mode):
    say(f"fixed startpoints mode={mode}")
    nl = synth.random_dag(synth.DagSpec(n_gates=2000, n_pi=40, depth=14), 40)
    p = synth.pi_probs(nl.n_pi, 41, batch=2)
    cap = synth.net_caps(nl.n_nets, 42)
    fixed = np.zeros(nl.n_pi, np.uint8)
    fixed[[0, 7, 8, 30]] = 1
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 2, mode=mode, n_sim=64 * 40, seed=43)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    fw = ev.forward(("power",))
    free = ev.backward(want=("dpi", "dcap"))
    lam_free, _ = ev.power_gradients()
    ev.set_pi_fixed(fixed)  # the forward stays valid
    fx = ev.backward(want=("dpi", "dcap"))
    lam_fx, _ = ev.power_gradients()
    assert (fx["dpi"][:, fixed != 0] == 0).all() and (lam_fx[:, :nl.n_pi][:, fixed != 0] == 0).all()
    np.testing.assert_array_equal(fx["dpi"][:, fixed == 0], free["dpi"][:, fixed == 0])
    np.testing.assert_array_equal(fx["dcap"], free["dcap"])
    np.testing.assert_array_equal(lam_fx[:, nl.n_pi:], lam_free[:, nl.n_pi:])
    assert (fw["power"] == ev.forward(("power",))["power"]).all()
    if mode == L.DP_MODELED:  # the ascent leaves fixed startpoints in place
        _, pf, _ = ev.power_virus(5, 1e-4)
        np.testing.assert_array_equal(pf[:, fixed != 0], p[:, fixed != 0])
        assert (pf[:, fixed == 0] != p[:, fixed == 0]).any()


def test_flop_cut_netlist_end_to_end(ctx):
    """A sequential netlist cut at its flops: data PIs, a clock and a reset
    excluded from the gradients, pseudo-PIs with shared streams and Markov
    rates; counts bit-exact, power and gradients against the oracle."""
    say("flop cut end to end")
    seq = synth.random_seq_dag(synth.DagSpec(n_gates=4000, n_pi=30, depth=18), 40, 44)
    cut = synth.cut_flops(seq)
    nl = cut.netlist
    T = 200
    p = synth.pi_probs(nl.n_pi, 45)
    p[0, 0], p[0, 1] = 0.5, 0.0            # clock, reset
    # pseudo-PIs that share a driver carry the same signal: the same p and tau
    p[0] = p[0][cut.stream]
    tau = _rates(p, 0.8, 46)
    tau[0] = tau[0][cut.stream]
    tau[0, 0], tau[0, 1] = 1.0, 0.0
    fixed = np.zeros(nl.n_pi, np.uint8)
    fixed[:2] = 1
    cap = synth.net_caps(nl.n_nets, 47)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 1, mode=L.DP_HYBRID, n_sim=64 * T, seed=48)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    ev.set_pi_rates(tau)
    ev.set_pi_streams(cut.stream)
    ev.set_pi_fixed(fixed)
    res = ev.forward(("sp", "ones", "toggles", "power"))
    g = ev.backward(want=("dpi",))
    o = oracle.Netlist.of(nl)
    words = oracle.stimulus_model(p[0], 48, T, tau=tau[0], stream=cut.stream)
    f = o.forward(p[0], cap, hybrid=True, n_words=T, pi_words=words)
    adj = o.adjoint(f["sp"], f["beta"], cap, fixed=fixed)
    np.testing.assert_array_equal(res["ones"][0].astype(np.uint64), f["ones"])
    np.testing.assert_array_equal(res["toggles"][0].astype(np.uint64), f["toggles"])
    assert_power_close(res["power"], f["power"])
    assert_grad_close(g["dpi"][0], adj["dpi"], "dP/dp")
    assert (g["dpi"][0][:2] == 0).all()
    # pseudo-PIs on one stream: one signal
    for k in range(len(cut.ppi)):
        s = cut.stream[cut.ppi[k]]
        assert res["ones"][0][cut.ppi[k]] == res["ones"][0][s]


def test_stimulus_model_errors(ctx):
    say("stimulus model errors")
    nl = synth.random_dag(synth.DagSpec(n_gates=100, n_pi=8, depth=4), 49)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 2, mode=L.DP_HYBRID, n_sim=256)
    bad = np.full((2, 8), 0.2, np.float32)
    bad[1, 3] = 1.5
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        ev.set_pi_rates(bad)
    bad[1, 3] = np.nan
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        ev.set_pi_rates(bad)
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        ev.set_pi_streams(np.array([0, 1, 2, 3, 4, 5, 6, 8], np.int32))
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        ev.set_pi_streams(np.array([0, 1, 2, 3, 4, 5, 6, -1], np.int32))
