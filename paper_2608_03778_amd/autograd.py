"""torch.autograd binding of the forward/reverse sweeps.

``power(ev, pi_prob, cap, sizes=None)`` returns switching power [B][S'] as
a differentiable tensor; its backward runs the library's reverse sweep
(Sec. III-E) with the upstream gradient as the seed weights, giving
gradients for the PI probabilities [B][n_pi], the capacitances [n_nets] and
the size factors [S][n_gates].  beta and the stimulus are held fixed, as in
the library.  Torch only provides device memory and the stream.
"""
from __future__ import annotations

import torch

from .api import Eval


class PowerFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pi_prob, cap, sizes, ev: Eval):
        ev.set_pi_prob(pi_prob.detach().contiguous())
        ev.set_caps(cap.detach().contiguous())
        if sizes is not None:
            ev.set_cell_sizes(sizes.detach().contiguous())
        out = ev.forward(("power",), device=True)
        ctx.ev = ev
        ctx.has_sizes = sizes is not None
        return out["power"]

    @staticmethod
    def backward(ctx, grad_power):
        ev = ctx.ev
        want = ("dpi", "dcap", "dsize") if ctx.has_sizes else ("dpi", "dcap")
        g = ev.backward(grad_power.detach().float().contiguous(), want=want, device=True)
        return g["dpi"], g["dcap"], g.get("dsize"), None


def power(ev: Eval, pi_prob, cap, sizes=None):
    """Differentiable switching power of the eval's design, [B][S']."""
    return PowerFn.apply(pi_prob, cap, sizes, ev)
