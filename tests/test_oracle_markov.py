"""Pins of the oracle's startpoint stimulus model (Sec. III-C: Markov chains
calibrated to a target SP and TR, shared streams for startpoints with a
common sequential driver) and of the fixed-startpoint gradient rule, each
against something other than the oracle: an independent Python route,
exact rationals, the independent stimulus at the independence rate, the
chain's stationary and transition laws, closed-form extremes."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import synth
from tests import brute


def _counts(words):
    """(ones, toggles) of each row of uint64 words [n][T]."""
    ones = np.array([sum(brute.popcount(int(w)) for w in row) for row in words])
    tog = np.array([sum(brute.popcount(int(a) ^ int(b)) for a, b in zip(row[1:], row[:-1]))
                    for row in words])
    return ones, tog


def test_probabilities_against_exact_rationals():
    for p, tau in ((0.3, 0.2), (0.9, 0.15), (0.01, 0.02), (0.5, 1.0), (0.7, 0.05)):
        pf, tf = Fraction(float(np.float32(p))), Fraction(float(np.float32(tau)))
        rise, stay = oracle.markov_probs(p, tau)
        ex_rise = min(tf / (2 * (1 - pf)), Fraction(1))
        ex_stay = max(1 - tf / (2 * pf), Fraction(0))
        assert abs(Fraction(rise) - ex_rise) <= Fraction(2, 1 << 52)
        assert abs(Fraction(stay) - ex_stay) <= Fraction(2, 1 << 52)
    # stationarity: p = p stay + (1 - p) rise, i.e. p b = (1 - p) a
    for p in (0.1, 0.37, 0.5, 0.8):
        tau = 0.7 * 2 * min(p, 1 - p)
        rise, stay = oracle.markov_probs(p, tau)
        pf = float(np.float32(p))
        assert abs(pf * stay + (1 - pf) * rise - pf) < 1e-7
    assert oracle.markov_probs(0.0, 0.0) == (0.0, 0.0)
    assert oracle.markov_probs(1.0, 0.0) == (1.0, 1.0)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    # tau past 2p: never stays at 1
    assert oracle.markov_probs(0.2, 0.9) == (f32(0.9) / (2 * (1 - f32(0.2))), 0.0)
    assert oracle.threshold_d(0.5) == 1 << 31 and oracle.threshold_d(1.0) == 1 << 32
    assert oracle.threshold_d(-0.1) == 0 and oracle.threshold_d(0.0) == 0
    assert oracle.threshold_d(2.0 ** -32) == 1 and oracle.threshold_d(2.0 ** -33) == 0


def test_independence_rate_reproduces_independent_words():
    """tau = 2p(1-p) makes every cycle an independent Bernoulli(p) draw;
    at dyadic p both chain probabilities equal p exactly, so the words are
    the independent stimulus bit for bit."""
    p = np.array([0.5, 0.25, 0.125, 0.75, 0.375, 0.0, 1.0, 0.5], np.float32)
    tau = (2 * p * (1 - p)).astype(np.float32)
    for pi, ti in zip(p, tau):
        assert oracle.markov_probs(pi, ti) == (float(pi), float(pi))
    T = 40
    w_ind = oracle.stimulus(p, 77, 0, T)
    np.testing.assert_array_equal(oracle.stimulus_model(p, 77, T, tau=tau), w_ind)
    np.testing.assert_array_equal(oracle.stimulus_model(p, 77, T), w_ind)
    np.testing.assert_array_equal(oracle.stimulus_model(p, 77, T, stream=np.arange(8)), w_ind)


def test_small_case_against_independent_python_route():
    p = np.array([0.3, 0.8, 0.5, 0.05, 0.6], np.float32)
    tau = np.array([0.1, 0.3, 1.0, 0.09, 0.0], np.float32)
    stream = np.array([0, 1, 2, 0, 4], np.int32)
    for t_, s_ in ((tau, stream), (tau, None), (None, stream)):
        np.testing.assert_array_equal(oracle.stimulus_model(p, 2 ** 40 + 9, 6, tau=t_, stream=s_),
                                      brute.markov_words(p, t_, s_, 2 ** 40 + 9, 6))


@pytest.mark.parametrize("p", [0.1, 0.3, 0.5, 0.8])
@pytest.mark.parametrize("frac", [0.05, 0.5, 1.0])
def test_chain_laws(p, frac):
    """SP_acc near p, TR_acc near tau, and the per-state transition
    frequencies near a and b, within 6 sigma of each statistic's law (the
    chain's autocorrelation lambda = 1 - a - b widens the first two)."""
    tau = frac * 2 * min(p, 1 - p)
    T = 600
    w = oracle.stimulus_model(np.full(4, p, np.float32), 5, T, tau=np.full(4, tau, np.float32),
                              stream=np.arange(4))
    ones, tog = _counts(w)
    rise, stay = oracle.markov_probs(p, tau)
    fall = 1 - stay
    lam = 1 - rise - fall
    infl = (1 + abs(lam)) / max(1 - abs(lam), 1e-3)
    n = 4 * 64 * T
    sp = ones.sum() / n
    assert abs(sp - p) < 6 * np.sqrt(p * (1 - p) / n * infl) + 1e-9
    tr = tog.sum() / (4 * 64 * (T - 1))
    assert abs(tr - tau) < 6 * np.sqrt(max(tau * (1 - tau), 1e-12) / n * 2 * infl) + 1e-9
    # conditional frequencies from the lane series
    bits = ((w[:, :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.int8)
    prev, nxt = bits[:, :-1, :].ravel(), bits[:, 1:, :].ravel()
    n0, n1 = (prev == 0).sum(), (prev == 1).sum()
    if n0:
        r = ((prev == 0) & (nxt == 1)).sum() / n0
        assert abs(r - rise) < 6 * np.sqrt(rise * (1 - rise) / n0) + 1e-9
    if n1:
        f = ((prev == 1) & (nxt == 0)).sum() / n1
        assert abs(f - fall) < 6 * np.sqrt(fall * (1 - fall) / n1) + 1e-9


def test_extremes():
    T = 30
    p = np.array([0.3, 0.5, 0.5, 0.0, 1.0], np.float32)
    # tau = 0: every lane keeps its first bit
    w = oracle.stimulus_model(p, 3, T, tau=np.zeros(5, np.float32))
    for row in w:
        assert (row == row[0]).all()
    _, tog = _counts(w)
    assert (tog == 0).all()
    # p = 1/2, tau = 1: every lane changes every cycle
    w = oracle.stimulus_model(p[1:2], 3, T, tau=np.ones(1, np.float32))
    assert all(int(w[0, t]) == (~int(w[0, t - 1])) & ((1 << 64) - 1) for t in range(1, T))
    # constant startpoints
    w = oracle.stimulus_model(p[3:], 3, T, tau=np.zeros(2, np.float32))
    assert (w[0] == 0).all() and (w[1] == np.uint64((1 << 64) - 1)).all()


def test_shared_streams():
    """Startpoints on one stream with one (p, tau) carry the same words; on
    one independent stream a lower p gives a subset of a higher p's ones
    (the same uniforms against a lower threshold)."""
    T = 20
    p = np.array([0.4, 0.4, 0.7, 0.7, 0.2, 0.9], np.float32)
    tau = np.array([0.3, 0.3, 0.2, 0.2, 0.1, 0.1], np.float32)
    stream = np.array([0, 0, 2, 2, 0, 0], np.int32)
    w = oracle.stimulus_model(p, 11, T, tau=tau, stream=stream)
    np.testing.assert_array_equal(w[0], w[1])
    np.testing.assert_array_equal(w[2], w[3])
    assert not np.array_equal(w[0], w[2])
    wi = oracle.stimulus_model(p, 11, T, stream=stream)
    np.testing.assert_array_equal(wi[4] & ~wi[0], np.zeros(T, np.uint64))
    np.testing.assert_array_equal(wi[0] & ~wi[5], np.zeros(T, np.uint64))


def test_simulated_pi_counts_are_the_words_counts():
    nl = synth.random_dag(synth.DagSpec(n_gates=200, n_pi=12, depth=8), 3)
    p = synth.pi_probs(nl.n_pi, 4)[0]
    tau = (0.5 * 2 * np.minimum(p, 1 - p)).astype(np.float32)
    w = oracle.stimulus_model(p, 8, 25, tau=tau)
    ones, tog = oracle.Netlist.of(nl).sim(25, pi_words=w)
    o2, t2 = _counts(w)
    np.testing.assert_array_equal(ones[: nl.n_pi], o2)
    np.testing.assert_array_equal(tog[: nl.n_pi], t2)


def test_fixed_startpoints_have_zero_gradient():
    nl = synth.random_dag(synth.DagSpec(n_gates=300, n_pi=16, depth=9), 6)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 7)[0].astype(np.float64)
    cap = synth.net_caps(nl.n_nets, 8)
    P = o.sp(p)
    beta = np.ones(nl.n_nets)
    fixed = np.zeros(nl.n_pi, np.uint8)
    fixed[[0, 5, 9]] = 1
    free = o.adjoint(P, beta, cap)
    fx = o.adjoint(P, beta, cap, fixed=fixed)
    assert (fx["dpi"][fixed != 0] == 0).all()
    np.testing.assert_array_equal(fx["dpi"][fixed == 0], free["dpi"][fixed == 0])
    np.testing.assert_array_equal(fx["lam"][nl.n_pi:], free["lam"][nl.n_pi:])
    np.testing.assert_array_equal(fx["dcap"], free["dcap"])
