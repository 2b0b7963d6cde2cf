"""The oracle on several host cores -- test and baseline infrastructure.

Worker processes are spawned fresh and import only the oracle (never the
GPU library).  Two kinds of work split without changing any result:

* the simulation over word ranges: the counts of disjoint cycle ranges
  (``Netlist.sim_range``) add up exactly, so the full run's ones and
  toggles are integer sums of the parts;
* central finite differences over startpoints: each startpoint's pair of
  forward evaluations is independent of the others.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_NL = None


def _init(n_pi, op, fanin_ptr, fanin, cells):
    global _NL
    from . import Netlist
    _NL = Netlist(n_pi, op, fanin_ptr, fanin, cells)


def _sim_part(args):
    a, b, p, seed = args
    return _NL.sim_range(a, b, p, seed=seed)


def _fd_part(args):
    pis, p, beta, cap, h, kappa = args
    out = []
    for i in pis:
        up = p.copy()
        dn = p.copy()
        up[i] += h
        dn[i] -= h
        fu = _NL.power(_NL.sp(up), cap, kappa=kappa, beta=beta)["power"]
        fd = _NL.power(_NL.sp(dn), cap, kappa=kappa, beta=beta)["power"]
        out.append((fu - fd) / (2.0 * h))
    return out


def workers_for(n_tasks, workers=None):
    return max(1, min(workers or (os.cpu_count() or 1), n_tasks))


def _pool(nl, n):
    ctx = mp.get_context("spawn")
    return ctx.Pool(n, initializer=_init,
                    initargs=(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin,
                              tuple(getattr(nl, "cells", ()))))


def sim_counts(nl, p, n_words, seed, workers=None):
    """(ones, toggles) of the full run of n_words words, as uint64, over
    `workers` processes (default: every host core)."""
    workers = workers_for(n_words, workers)
    bounds = np.linspace(0, n_words, workers + 1).astype(int)
    jobs = [(int(bounds[i]), int(bounds[i + 1]), np.asarray(p, np.float32), int(seed))
            for i in range(workers) if bounds[i + 1] > bounds[i]]
    with _pool(nl, len(jobs)) as pool:
        parts = pool.map(_sim_part, jobs)
    ones = sum(x[0] for x in parts)
    tog = sum(x[1] for x in parts)
    return ones, tog


def fd_gradients(nl, p, pis, cap, beta, h=1e-6, kappa=0.5, workers=None):
    """Central differences (P(p + h e_i) - P(p - h e_i)) / 2h of the power
    with beta held fixed, for the startpoints `pis`, over `workers`
    processes."""
    pis = [int(i) for i in pis]
    workers = workers_for(len(pis), workers)
    chunks = [pis[k::workers] for k in range(workers)]
    p64 = np.asarray(p, np.float64)
    b64 = np.asarray(beta, np.float64)
    jobs = [(c, p64, b64, np.asarray(cap, np.float32), float(h), float(kappa)) for c in chunks if c]
    with _pool(nl, len(jobs)) as pool:
        parts = pool.map(_fd_part, jobs)
    out = np.zeros(len(pis))
    pos = {i: k for k, i in enumerate(pis)}
    for c, vals in zip([c for c in chunks if c], parts):
        for i, v in zip(c, vals):
            out[pos[i]] = v
    return out
