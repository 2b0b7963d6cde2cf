"""The library autotuner (launch schedules, simulation tilings, word chunks
and streams) keeps every result: the schedule it picks gives the default
schedule's SP, counts, power and gradients bit for bit, and both match the
FP64 oracle.

Each case runs in a child process of its own, on a fresh device context:
the in-process test of the autotuner after the design-group and serving
tests stays skipped (test_gpu_parity.py) until the host crash it once
showed there has a known cause."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import numpy as np
import pytest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def child(mode: str) -> dict:
    """Body run in the child process; prints one JSON line."""
    import oracle
    from paper_2608_03778_amd import _lib as L
    from paper_2608_03778_amd import api, synth
    from tests.gpu_helpers import (SP_ABS, assert_grad_close, assert_power_close,
                                   oracle_column)

    nl = synth.random_dag(synth.SPECS["dag2k"], 13)
    B = 2 if mode == "hybrid" else 5
    p = synth.pi_probs(nl.n_pi, 13, batch=B)
    cap = synth.net_caps(nl.n_nets, 14)
    ctx = api.Context(0)
    d = api.Design(ctx, nl)
    hyb = mode == "hybrid"
    kw = dict(mode=L.DP_HYBRID, n_sim=64 * 512, seed=8) if hyb else dict(mode=L.DP_MODELED)
    outs = ("sp", "ones", "toggles", "power") if hyb else ("sp", "power")
    ev = api.Eval(d, B, **kw)
    ev.set_pi_prob(p)
    ev.set_caps(cap)
    a = ev.forward(outs)
    a.update(ev.backward(want=("dpi", "dcap")))
    ms = ev.autotune(2, with_backward=True)
    sch = ev.get_schedule()
    assert ms > 0, ms
    assert sch["schedule"] in (L.DP_SCHED_LEVEL, L.DP_SCHED_GRAPH), sch
    if hyb:
        assert sch["pairs_per_lane"] in (1, 2, 4, 8), sch
    for rep in range(2):  # a captured schedule replays: check more than one launch
        b = ev.forward(outs)
        b.update(ev.backward(want=("dpi", "dcap")))
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"{k} after autotune, pass {rep}")
    o = oracle.Netlist.of(nl)
    for col in range(B):
        f, adj = oracle_column(o, p[col], cap, mode=mode, n_words=512, seed=8)
        np.testing.assert_allclose(b["sp"][col], f["sp"], atol=SP_ABS, rtol=0)
        if hyb:
            np.testing.assert_array_equal(b["ones"][col].astype(np.uint64), f["ones"])
            np.testing.assert_array_equal(b["toggles"][col].astype(np.uint64), f["toggles"])
        assert_power_close(b["power"][col], f["power"], f"power column {col}")
        assert_grad_close(b["dpi"][col], adj["dpi"], f"dP/dp column {col}")
    return dict(ok=True, ms=ms, schedule=sch)


@pytest.mark.parametrize("mode", ["hybrid", "modeled"])
def test_autotune_keeps_results_fresh_process(mode):
    say(f"autotune ({mode}) in a child process")
    r = subprocess.run([sys.executable, "-u", "-m", "tests.test_gpu_autotune", mode], cwd=ROOT,
                       capture_output=True, text=True, timeout=180)
    tail = (r.stdout[-2000:] + r.stderr[-2000:]).strip()
    assert r.returncode == 0, f"child exited with {r.returncode}:\n{tail}"
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    res = json.loads(line)
    assert res["ok"], tail
    say(f"autotune ({mode}): {res['schedule']} at {res['ms']:.3f} ms")


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    print(json.dumps(child(sys.argv[1])), flush=True)
