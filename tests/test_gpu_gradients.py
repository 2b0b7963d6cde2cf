"""Every net's adjoint and the Eq. 8 sizing score from the GPU, against the
oracle's adjoint and score, and the rank agreement of the GPU adjoints with
finite differences of the oracle (Sec. V-C).

Score tolerance: S = |lambda| P (1 - P) / |1 - 2P|, so its relative error is
that of lambda (the 1e-4 gradient bar) plus the SP error (1e-5 absolute)
divided by min(P, 1 - P) and by |1 - 2P|; on nets with |1 - 2P| > 0.02 and
min(P, 1 - P) > 0.02 that is below 2e-3."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, rank, synth
from tests.gpu_helpers import assert_grad_close, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode,ste", [(L.DP_MODELED, False), (L.DP_HYBRID, False),
                                      (L.DP_HYBRID, True)])
def test_every_net_adjoint_and_score(mode, ste):
    say(f"power gradients mode={mode} ste={ste}")
    ctx = api.Context(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 15)
    cap = synth.net_caps(nl.n_nets, 15)
    B = 2
    p = synth.pi_probs(nl.n_pi, 15, batch=B)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, B, mode=mode, n_sim=64 * 30, seed=4,
                  beta_grad=L.DP_BETA_STE if ste else L.DP_BETA_LOCAL)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    ev.forward(("power",))
    dpi = ev.backward(want=("dpi",))["dpi"]
    lam, score = ev.power_gradients()
    o = oracle.Netlist.of(nl)
    for b in range(B):
        # the oracle's own calibration on the same seeded stimulus (every
        # column draws the same counters, so column b is a one-column run)
        f = o.forward(p[b], cap, hybrid=mode == L.DP_HYBRID, n_words=30, seed=4)
        P, beta = f["sp"], f["beta"]
        adj = o.adjoint(P, beta, cap, beta_ste=ste)
        assert_grad_close(lam[b], adj["lam"], f"lambda[{b}]")
        np.testing.assert_array_equal(lam[b][: nl.n_pi], dpi[b])
        S = o.sizing_score(P, adj["lam"])
        Pg = P[nl.n_pi:]
        ok = (np.abs(1 - 2 * Pg) > 0.02) & (np.minimum(Pg, 1 - Pg) > 0.02)
        np.testing.assert_allclose(score[b][ok], S[ok], rtol=2e-3, atol=1e-6 * S.max())
        assert np.isfinite(score[b]).all() and (score[b] >= 0).all()


def test_adjoint_rank_agreement_with_finite_differences():
    """GPU adjoints of 80 sampled nets against oracle central differences of
    the frozen-beta power (SP-override hook): Pearson, top-10 overlap and
    Jaccard."""
    say("rank agreement")
    ctx = api.Context(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 16)
    cap = synth.net_caps(nl.n_nets, 16)
    p = synth.pi_probs(nl.n_pi, 16)
    d = api.Design(ctx, nl)
    ev = api.Eval(d, 1)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    ev.forward(("power",))
    lam, _ = ev.power_gradients()
    o = oracle.Netlist.of(nl)
    p64 = p[0].astype(np.float64)
    P = o.sp(p64)
    beta = np.ones(nl.n_nets)
    rng = np.random.default_rng(16)
    nets = [n for n in rng.choice(nl.n_nets, 120, replace=False) if 1e-3 < P[n] < 1 - 1e-3][:80]
    h = 1e-6
    fd = np.array([(o.power(o.sp_override(p64, n, h), cap, beta=beta)["power"]
                    - o.power(o.sp_override(p64, n, -h), cap, beta=beta)["power"]) / (2 * h)
                   for n in nets])
    m = rank.agreement(lam[0][nets], fd, 10)
    say(f"rank agreement {m}")
    assert m["pearson"] > 0.99999
    assert m["top_k_overlap"] == 1.0 and m["jaccard_top_k"] == 1.0
