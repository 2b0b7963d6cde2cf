"""dp_forward_static (no allocation, static device scratch) against
dp_forward on a one-column eval, through the C ABI: bit for bit on every
output, on two calls in a row, the second with a smaller design, in
DP_MODELED and DP_FROZEN_BETA."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2608_03778_amd import _lib as L
from paper_2608_03778_amd import api, synth
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _eval_forward(d, p, cap, mode, beta):
    ev = api.Eval(d, 1, mode=mode)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    if beta is not None:
        ev.set_beta(beta[None, :])
    r = ev.forward(("sp", "tr", "power"))
    ev.close()
    return r


@pytest.mark.parametrize("mode", [L.DP_MODELED, L.DP_FROZEN_BETA])
def test_static_forward_matches_eval_forward(mode):
    import torch
    torch.cuda.set_device(0)
    ctx = api.Context.for_torch(0)
    cases = [synth.DagSpec(n_gates=30000, n_pi=512, depth=40),   # several tiles, ragged tail
             synth.DagSpec(n_gates=2500, n_pi=64, depth=18)]     # then a smaller design
    for k, spec in enumerate(cases):
        nl = synth.random_dag(spec, 70 + k)
        say(f"static forward mode={mode} case={k} gates={nl.n_gates}")
        d = api.Design(ctx, nl)
        p = synth.pi_probs(nl.n_pi, 71 + k)[0]
        cap = synth.net_caps(nl.n_nets, 72 + k)
        beta = None
        if mode == L.DP_FROZEN_BETA:
            beta = np.random.default_rng(73 + k).uniform(0.1, 10.0, nl.n_nets).astype(np.float32)
        ref = _eval_forward(d, p, cap, mode, beta)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        out_power = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
        out_sp = torch.full((nl.n_nets,), -1.0, dtype=torch.float32, device="cuda")
        out_tr = torch.full((nl.n_nets,), -1.0, dtype=torch.float32, device="cuda")
        d.forward_static(dev(p), dev(cap), mode=mode, beta=dev(beta) if beta is not None else None,
                         out_power=out_power, out_sp=out_sp, out_tr=out_tr)
        torch.cuda.synchronize()
        assert out_power.item() == float(ref["power"][0, 0])
        np.testing.assert_array_equal(out_sp.cpu().numpy(), ref["sp"][0])
        np.testing.assert_array_equal(out_tr.cpu().numpy(), ref["tr"][0])
        d.close()


def test_static_forward_rejects_what_it_cannot_run():
    import torch
    torch.cuda.set_device(0)
    ctx = api.Context.for_torch(0)
    say("static forward errors")
    nl = synth.random_dag(synth.DagSpec(n_gates=500, n_pi=16, depth=6), 3)
    d = api.Design(ctx, nl)
    t = lambda n: torch.zeros(n, dtype=torch.float32, device="cuda")
    with pytest.raises(L.DiffPowerError, match="UNSUPPORTED"):
        d.forward_static(t(nl.n_pi), t(nl.n_nets), mode=L.DP_HYBRID, out_power=t(1))
    with pytest.raises(L.DiffPowerError, match="INVALID"):
        d.forward_static(t(nl.n_pi), t(nl.n_nets), mode=L.DP_FROZEN_BETA, out_power=t(1))
    # more nets than the static scratch holds: rejected before any launch
    wide = synth.Netlist(n_pi=(1 << 21), op=np.array([1], np.uint8),
                         fanin_ptr=np.array([0, 1], np.int32), fanin=np.array([0], np.int32))
    dw = api.Design(ctx, wide)
    with pytest.raises(L.DiffPowerError, match="at most"):
        dw.forward_static(t(dw.n_pi), t(dw.n_nets), out_power=t(1))
