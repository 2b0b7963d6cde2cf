"""The oracle split over worker processes (the CPU baseline's all-core
runs) gives the single-process results: simulation counts exactly, finite
differences to the last bit."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import parallel
from paper_2608_03778_amd import synth


def test_word_ranges_add_up_to_the_full_run():
    nl = synth.random_dag(synth.SPECS["dag2k"], 3)
    p = synth.pi_probs(nl.n_pi, 3)[0]
    o = oracle.Netlist.of(nl)
    ones, tog = o.sim(37, p_pi=p, seed=5)
    pones, ptog = parallel.sim_counts(nl, p, 37, seed=5, workers=3)
    np.testing.assert_array_equal(pones, ones)
    np.testing.assert_array_equal(ptog, tog)


def test_finite_differences_split_over_workers():
    nl = synth.random_dag(synth.DagSpec(n_gates=400, n_pi=32, depth=8), 4)
    p = synth.pi_probs(nl.n_pi, 4)[0].astype(np.float64)
    cap = synth.net_caps(nl.n_nets, 4)
    o = oracle.Netlist.of(nl)
    beta = np.ones(nl.n_nets)
    pis = [0, 5, 9, 31, 17]
    h = 1e-6
    serial = []
    for i in pis:
        up, dn = p.copy(), p.copy()
        up[i] += h
        dn[i] -= h
        serial.append((o.power(o.sp(up), cap, beta=beta)["power"]
                       - o.power(o.sp(dn), cap, beta=beta)["power"]) / (2 * h))
    got = parallel.fd_gradients(nl, p, pis, cap, beta, h=h, workers=2)
    np.testing.assert_array_equal(got, np.array(serial))
