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
