"""Run the oracle's cycle-range simulation over word ranges in worker
processes (spawned fresh: they import only the oracle, never the GPU
library) and add the exact integer counts."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_NL = None


def _init(n_pi, op, fanin_ptr, fanin, cells):
    global _NL
    import oracle
    _NL = oracle.Netlist(n_pi, op, fanin_ptr, fanin, cells)


def _run(args):
    a, b, p, seed = args
    return _NL.sim_range(a, b, p, seed=seed)


def sim_counts(nl, p, n_words, seed, workers=None):
    """(ones, toggles) of the full run of n_words words, as uint64."""
    workers = workers or min(16, os.cpu_count() or 1, n_words)
    bounds = np.linspace(0, n_words, workers + 1).astype(int)
    jobs = [(int(bounds[i]), int(bounds[i + 1]), np.asarray(p, np.float32), int(seed))
            for i in range(workers) if bounds[i + 1] > bounds[i]]
    ctx = mp.get_context("spawn")
    with ctx.Pool(len(jobs), initializer=_init,
                  initargs=(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin,
                            tuple(getattr(nl, "cells", ())))) as pool:
        parts = pool.map(_run, jobs)
    ones = sum(x[0] for x in parts)
    tog = sum(x[1] for x in parts)
    return ones, tog
