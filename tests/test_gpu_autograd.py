"""The torch.autograd binding: gradients equal the oracle's adjoint, and a
finite-difference check of the same function through torch."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import assert_grad_close, assert_power_close, oracle_column, say

pytestmark = pytest.mark.gpu


def test_autograd_matches_oracle():
    import torch

    from paper_2608_03778_amd.autograd import power
    say("autograd")
    torch.cuda.set_device(0)
    ctx = api.Context.for_torch(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 12)
    d = api.Design(ctx, nl)
    B, S = 2, 3
    p = synth.pi_probs(nl.n_pi, 12, batch=B)
    cap = synth.net_caps(nl.n_nets, 13)
    size = synth.cell_sizes(nl.n_gates, 14, n_size=S)
    ev = api.Eval(d, B, S, mode=L.DP_MODELED)
    tp = torch.tensor(p, device="cuda", requires_grad=True)
    tc = torch.tensor(cap, device="cuda", requires_grad=True)
    ts = torch.tensor(size, device="cuda", requires_grad=True)
    P = power(ev, tp, tc, ts)
    w = torch.tensor(np.random.default_rng(3).uniform(0.5, 2.0, (B, S)), dtype=torch.float32,
                     device="cuda")
    (P * w).sum().backward()
    o = oracle.Netlist.of(nl)
    gp = np.zeros((B, nl.n_pi))
    gc = np.zeros(nl.n_nets)
    gs = np.zeros((S, nl.n_gates))
    wn = w.cpu().numpy()
    for b in range(B):
        for s in range(S):
            f, adj = oracle_column(o, p[b], cap, size[s])
            assert_power_close(P[b, s].item(), f["power"])
            gp[b] += wn[b, s] * adj["dpi"]
            gc += wn[b, s] * adj["dcap"]
            gs[s] += wn[b, s] * adj["dsize"]
    assert_grad_close(tp.grad.cpu().numpy().ravel(), gp.ravel(), "grad p")
    assert_grad_close(tc.grad.cpu().numpy(), gc, "grad C")
    assert_grad_close(ts.grad.cpu().numpy().ravel(), gs.ravel(), "grad s")


def test_torch_stream_ordering_and_graph_on_null_stream():
    """A context on torch's (null) stream: inputs torch computes just before
    a call, and outputs torch reads just after, need no extra
    synchronisation; the captured-graph schedule works on that stream and
    gives the per-level results bitwise."""
    import torch
    say("torch stream ordering")
    torch.cuda.set_device(0)
    ctx = api.Context.for_torch(0)
    nl = synth.random_dag(synth.SPECS["dag2k"], 21)
    d = api.Design(ctx, nl)
    p = synth.pi_probs(nl.n_pi, 21)
    cap = synth.net_caps(nl.n_nets, 22)
    ref = api.Eval(d, 1, mode=L.DP_HYBRID, n_sim=4096, seed=3)
    ref.set_pi_prob(p)
    ref.set_caps(cap)
    want = ref.forward(("sp", "ones", "power"))
    for sched in (L.DP_SCHED_LEVEL, L.DP_SCHED_GRAPH, L.DP_SCHED_PERSISTENT):
        ev = api.Eval(d, 1, mode=L.DP_HYBRID, n_sim=4096, seed=3)
        ev.set_schedule(sched)
        for _ in range(3):
            # inputs produced by torch kernels right before the calls
            tp = torch.zeros(1, nl.n_pi, device="cuda").add_(torch.from_numpy(p).cuda())
            tc = torch.full((nl.n_nets,), 2.0, device="cuda").mul_(0.0).add_(
                torch.from_numpy(cap).cuda())
            ev.set_pi_prob(tp)
            ev.set_caps(tc)
            out = ev.forward(("sp", "ones", "power"), device=True)
            # read by torch kernels right after
            sp = (out["sp"] * 1.0).cpu().numpy()
            ones = out["ones"].clone().cpu().numpy().view(np.uint32)
            pw = (out["power"] + 0.0).cpu().numpy()
            np.testing.assert_array_equal(ones, want["ones"])
            np.testing.assert_array_equal(sp, want["sp"])
            np.testing.assert_array_equal(pw, want["power"])
