"""Power-virus gradient ascent (Alg. 4) on the GPU against the oracle's.

Tolerance of the ascended probabilities: each step adds eta * grad, and the
FP32 gradient is within 1e-4 relative of the FP64 one (the gradient bar), so
after `steps` steps |p_gpu - p_oracle| <= steps * eta * 1e-4 * max|grad| plus
the clip; with 40 steps, eta = 1e-3 and |grad| < 100 that is 4e-4.  Where the
oracle's p is that close to 1/2 the threshold may go either way; everywhere
else v0 must agree.  P_virus of the GPU's own vectors is checked against the
oracle's evaluation of the same vectors (exact up to summation order)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

STEPS, ETA = 40, 1e-3
P_ABS = STEPS * ETA * 1e-4 * 100.0


def _run(mode, beta=None):
    ctx = api.Context(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 7)
    cap = synth.net_caps(nl.n_nets, 7)
    B = 2
    p0 = np.stack([np.full(nl.n_pi, 0.5, np.float32),
                   np.random.default_rng(7).uniform(0.2, 0.8, nl.n_pi).astype(np.float32)])
    d = api.Design(ctx, nl)
    ev = api.Eval(d, B, mode=mode)
    ev.set_pi_prob(p0)
    ev.set_caps(cap)
    if beta is not None:
        ev.set_beta(np.tile(beta.astype(np.float32), (B, 1)))
    v0, pf, pv = ev.power_virus(STEPS, ETA)
    o = oracle.Netlist.of(nl)
    for b in range(B):
        p_o, v0_o, pv_o = o.power_virus(p0[b].astype(np.float64), cap, steps=STEPS, eta=ETA,
                                        beta=None if beta is None else beta.astype(np.float64))
        np.testing.assert_allclose(pf[b], p_o, atol=P_ABS, rtol=0)
        decided = np.abs(p_o - 0.5) > P_ABS
        np.testing.assert_array_equal(v0[b][decided], v0_o[decided])
        assert pv[b] == pytest.approx(o.virus_power(v0[b], cap), rel=1e-12)
        if (v0[b] == v0_o).all():
            assert pv[b] == pytest.approx(pv_o, rel=1e-12)
    return nl, ev, o, cap


def test_power_virus_modeled_matches_oracle():
    say("power virus, modeled")
    nl, ev, o, cap = _run(L.DP_MODELED)
    # steps = 0 thresholds the start: the pair's P_virus is the oracle's
    p = np.random.default_rng(1).uniform(0, 1, (2, nl.n_pi)).astype(np.float32)
    ev.set_pi_prob(p)
    v0, pf, pv = ev.power_virus(0, ETA)
    np.testing.assert_array_equal(v0, (p >= 0.5).astype(np.uint8))
    np.testing.assert_array_equal(pf, p)
    for b in range(2):
        assert pv[b] == pytest.approx(o.virus_power(v0[b], cap), rel=1e-12)


def test_power_virus_beta_scaled_matches_oracle():
    say("power virus, beta scaling")
    nl = synth.random_dag(synth.SPECS["dag2k"], 7)
    beta = np.random.default_rng(8).uniform(0.5, 2.0, nl.n_nets)
    _run(L.DP_FROZEN_BETA, beta)


def test_power_virus_errors():
    ctx = api.Context(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 1)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 1, mode=L.DP_HYBRID, n_sim=128)
    ev.set_pi_prob(np.full(nl.n_pi, 0.5, np.float32))
    ev.set_caps(synth.net_caps(nl.n_nets, 1))
    with pytest.raises(L.DiffPowerError, match="UNSUPPORTED"):
        ev.power_virus(1, ETA)
    ev = api.Eval(d, 1, 2)
    ev.set_pi_prob(np.full(nl.n_pi, 0.5, np.float32))
    ev.set_caps(synth.net_caps(nl.n_nets, 1))
    with pytest.raises(L.DiffPowerError, match="UNSUPPORTED"):
        ev.power_virus(1, ETA)
    ev = api.Eval(d, 1)
    with pytest.raises(L.DiffPowerError, match="STATE"):
        ev.power_virus(1, ETA)
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        ev.power_virus(-1, ETA)
