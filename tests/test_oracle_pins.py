"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (no GPU).  Each test names what it pins; a plausible slip in the
oracle (a dropped term, a wrong sign, a swapped pin) fails at least one."""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2608_03778_amd import synth
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- gate rules
@pytest.mark.parametrize("op", range(9))
def test_gate_sp_equals_minterm_sum(op):
    """Sec. II-B: P(out=1) under independent inputs is the minterm sum."""
    rng = np.random.default_rng(op)
    k = brute.ARITY[op]
    for _ in range(50):
        p = rng.random(k)
        assert oracle.gate_sp(op, p) == pytest.approx(brute.gate_probability(op, p), abs=1e-15)
    for corner in itertools.product((0.0, 1.0), repeat=k):
        assert oracle.gate_sp(op, corner) == brute.gate_probability(op, corner)


@pytest.mark.parametrize("op", range(9))
def test_gate_partials_equal_minterm_derivative(op):
    """Sec. III-E partial derivatives, against the derivative of the minterm
    sum (computed term by term, not from the closed forms)."""
    rng = np.random.default_rng(100 + op)
    k = brute.ARITY[op]
    for _ in range(50):
        p = rng.random(k)
        np.testing.assert_allclose(oracle.gate_partials(op, p),
                                   brute.gate_probability_grad(op, p), atol=1e-14)


def test_paper_partial_examples():
    """The examples printed in Sec. III-E: dAND/dA = P_B, dOR/da = 1-b,
    dXOR/da = 1-2b, dNOT/dx = -1."""
    a, b = 0.3, 0.8
    assert oracle.gate_partials(synth.AND2, [a, b])[0] == pytest.approx(b)
    assert oracle.gate_partials(synth.OR2, [a, b])[0] == pytest.approx(1 - b)
    assert oracle.gate_partials(synth.XOR2, [a, b])[0] == pytest.approx(1 - 2 * b)
    assert oracle.gate_partials(synth.INV, [a])[0] == -1.0
    # Alg. 2's AND and NAND examples
    assert oracle.gate_sp(synth.AND2, [a, b]) == pytest.approx(a * b)
    assert oracle.gate_sp(synth.NAND2, [a, b]) == pytest.approx(1 - a * b)


@pytest.mark.parametrize("op", range(9))
def test_gate_bits_truth_table(op):
    """Sec. III-C: each lane of a simulated word follows the cell's Boolean
    function; lanes enumerate every input assignment."""
    k = brute.ARITY[op]
    words = brute.pack_minterm_words(k)
    out = oracle.gate_bits(op, words)
    for lane in range(64):
        ins = [bool((lane >> i) & 1) for i in range(k)]
        assert bool((out >> lane) & 1) == bool(brute.TRUTH[op](*ins)), (op, lane)


# ------------------------------------------------------------ propagation
@pytest.mark.parametrize("seed", range(12))
def test_tree_sp_is_exact(seed):
    """On fan-out-free trees the independence assumption holds, so the
    propagated SP of every net equals exhaustive enumeration."""
    nl = synth.random_tree(n_leaves=4 + seed, seed=seed)
    o = oracle.Netlist.of(nl)
    p = np.random.default_rng(seed).uniform(0.05, 0.95, nl.n_pi)
    exact = brute.exact_probabilities(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin, p)
    np.testing.assert_allclose(o.sp(p), exact, atol=1e-12)


def test_closed_forms():
    """AND chain = prod p_i; XOR tree = (1 - prod(1-2p_i))/2 (piling-up);
    INV chain of even length = identity, odd = complement."""
    rng = np.random.default_rng(7)
    n = 12
    p = rng.uniform(0.05, 0.95, n)
    gates = [(synth.AND2, [0, 1])]
    for i in range(2, n):
        gates.append((synth.AND2, [n + len(gates) - 1, i]))
    o = oracle.Netlist.of(synth.from_gates(n, gates))
    assert o.sp(p)[-1] == pytest.approx(np.prod(p), rel=1e-13)
    gates = [(synth.XOR2, [0, 1])]
    for i in range(2, n):
        gates.append((synth.XOR2, [i, n + len(gates) - 1]))
    o = oracle.Netlist.of(synth.from_gates(n, gates))
    assert o.sp(p)[-1] == pytest.approx(0.5 * (1 - np.prod(1 - 2 * p)), abs=1e-14)
    gates = [(synth.INV, [0])] + [(synth.INV, [1 + i]) for i in range(8)]
    o = oracle.Netlist.of(synth.from_gates(1, gates))
    P = o.sp([0.3])
    assert P[-1] == pytest.approx(1 - 0.3) and P[-2] == pytest.approx(0.3)


def test_reconvergence_is_not_exact_but_bounded():
    """With reconvergence the model ignores spatial correlation (Sec. II-B):
    XOR(a, a) is modeled as 2a(1-a) while it is constantly 0.  SP stays in
    [0, 1] and TR_model in [0, 1/2] on random reconvergent DAGs."""
    o = oracle.Netlist.of(synth.from_gates(1, [(synth.XOR2, [0, 0])]))
    assert o.sp([0.3])[-1] == pytest.approx(2 * 0.3 * 0.7)
    nl = synth.random_dag(synth.SPECS["dag2k"], 3)
    o = oracle.Netlist.of(nl)
    P = o.sp(synth.pi_probs(nl.n_pi, 3)[0])
    assert (P >= 0).all() and (P <= 1).all()
    tr = o.power(P, np.ones(nl.n_nets, np.float32))["tr_model"]
    assert (tr <= 0.5).all() and (tr >= 0).all()


def test_topological_order_and_cycle():
    nl = synth.random_dag(synth.SPECS["dag2k"], 1)
    o = oracle.Netlist.of(nl)
    lv = o.levels()
    assert lv.max() == 20
    for g in range(nl.n_gates):
        ins = nl.fanin[nl.fanin_ptr[g]:nl.fanin_ptr[g + 1]]
        assert lv[nl.n_pi + g] == 1 + lv[ins].max()
    with pytest.raises(ValueError, match="cycle"):
        oracle.Netlist(1, [synth.AND2, synth.BUF], [0, 2, 3], [0, 2, 1])
    with pytest.raises(ValueError, match="malformed"):
        oracle.Netlist(1, [synth.AND2], [0, 1], [0])


# -------------------------------------------------------------- simulation
def _reconvergent_small(seed):
    spec = synth.DagSpec(n_gates=40, n_pi=6, depth=6, reconv=0.5)
    return synth.random_dag(spec, seed)


@pytest.mark.parametrize("seed", range(4))
def test_sim_exhaustive_stimulus_counts(seed):
    """Pass 2 with every PI assignment in the 64 lanes of each word: ones[n]
    = T * (#assignments with net n = 1) exactly, reconvergence included;
    a stimulus constant in time gives no toggles."""
    nl = _reconvergent_small(seed)
    o = oracle.Netlist.of(nl)
    T = 5
    w = np.repeat(brute.pack_minterm_words(nl.n_pi)[:, None], T, axis=1)
    ones, tog = o.sim(T, pi_words=w)
    vals = brute.eval_all_minterms(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin)
    np.testing.assert_array_equal(ones, T * vals.sum(axis=1))
    assert (tog == 0).all()


@pytest.mark.parametrize("seed", range(3))
def test_sim_alternating_stimulus_toggles(seed):
    """Alternating every PI lane each cycle: a net toggles in a lane iff its
    value differs between the assignment and its complement."""
    nl = _reconvergent_small(10 + seed)
    o = oracle.Netlist.of(nl)
    T = 7
    base = brute.pack_minterm_words(nl.n_pi)
    w = np.stack([base if t % 2 == 0 else ~base for t in range(T)], axis=1).astype(np.uint64)
    ones, tog = o.sim(T, pi_words=w)
    vals = brute.eval_all_minterms(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin)
    comp = (1 << nl.n_pi) - 1 - np.arange(1 << nl.n_pi)
    flips = (vals != vals[:, comp]).sum(axis=1)  # per 64 lanes
    np.testing.assert_array_equal(tog, (T - 1) * flips)
    assert (tog[: nl.n_pi] == 64 * (T - 1)).all()


def test_sim_chain_and_self_xor():
    """BUF/INV chains preserve toggles and complement ones; XOR(a, a) never
    toggles and is never 1."""
    gates = [(synth.INV, [0]), (synth.BUF, [1]), (synth.INV, [2]), (synth.XOR2, [0, 0])]
    o = oracle.Netlist.of(synth.from_gates(1, gates))
    T = 50
    w = oracle.stimulus([0.37], seed=9, t0=0, n_words=T)
    ones, tog = o.sim(T, pi_words=w)
    assert tog[1] == tog[2] == tog[3] == tog[0]
    assert ones[1] == 64 * T - ones[0] and ones[3] == ones[0]
    assert ones[4] == 0 and tog[4] == 0


def test_sim_statistics_iid():
    """i.i.d. Bernoulli(p) stimulus: on PIs SP_acc is within 5 sigma of p and
    TR_acc within 5 sigma of 2p(1-p)."""
    p = np.array([0.1, 0.25, 0.5, 0.77, 0.9], dtype=np.float32)
    T = 400
    nl = synth.from_gates(5, [(synth.BUF, [i]) for i in range(5)])
    o = oracle.Netlist.of(nl)
    ones, tog = o.sim(T, p_pi=p, seed=1234)
    n = 64.0 * T
    for i, pi in enumerate(p.astype(np.float64)):
        sd = math.sqrt(pi * (1 - pi) / n)
        assert abs(ones[i] / n - pi) < 5 * sd
        tr = 2 * pi * (1 - pi)
        assert abs(tog[i] / (64.0 * (T - 1)) - tr) < 5 * math.sqrt(tr * (1 - tr) / (64 * (T - 1))) * 2


# ------------------------------------------------------------------ Philox
def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                v = [int(x, 16) for x in line.split()]
                rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, want in _kat():
        assert list(oracle.philox4x32_10(ctr, key)) == want
        assert brute.philox4x32_10(ctr, key) == want


def test_philox_matches_independent_python():
    rng = np.random.default_rng(5)
    for _ in range(200):
        ctr = rng.integers(0, 2**32, 4, dtype=np.uint64)
        key = rng.integers(0, 2**32, 2, dtype=np.uint64)
        assert list(oracle.philox4x32_10(ctr, key)) == brute.philox4x32_10(ctr, key)


def test_threshold_exact():
    """floor(p * 2^32) of the float32 value, exactly."""
    assert oracle.threshold(0.0) == 0
    assert oracle.threshold(1.0) == 2**32
    assert oracle.threshold(0.5) == 2**31
    rng = np.random.default_rng(1)
    for p in rng.random(500).astype(np.float32):
        assert oracle.threshold(p) == math.floor(Fraction(float(p)) * 2**32)


def test_stimulus_word_definition():
    """Bit j of word t of PI i is lane j%4 of Philox(t, i, j//4, 0; seed)
    compared with the threshold."""
    seed = 0x1234_5678_9ABC_DEF0
    key = [seed & 0xFFFFFFFF, seed >> 32]
    p = np.array([0.3, 0.61], dtype=np.float32)
    w = oracle.stimulus(p, seed, t0=3, n_words=2)
    for i in range(2):
        thr = math.floor(Fraction(float(p[i])) * 2**32)
        for tt in range(2):
            t = 3 + tt
            want = 0
            for j in range(64):
                u = brute.philox4x32_10([t, i, j // 4, 0], key)[j % 4]
                if u < thr:
                    want |= 1 << j
            assert int(w[i, tt]) == want


# ------------------------------------------------------------------- power
def test_power_buffer_chain_half():
    """All-BUF/INV circuit at p = 1/2: TR = 1/2 on every net, so modeled
    P = kappa * 1/2 * sum C (Eq. 1 and 2)."""
    gates = [(synth.BUF, [0]), (synth.INV, [1]), (synth.INV, [0]), (synth.BUF, [3])]
    nl = synth.from_gates(1, gates)
    o = oracle.Netlist.of(nl)
    cap = np.array([1.0, 2.0, 3.5, 0.25, 4.0], dtype=np.float32)
    out = o.forward([0.5], cap, kappa=0.5)
    assert out["power"] == pytest.approx(0.5 * 0.5 * cap.astype(np.float64).sum(), rel=1e-15)


def test_power_euler_and_linearity():
    """Power is homogeneous of degree 1 in C: sum_n C_n dP/dC_n = P, and
    P(2C) = 2 P(C)."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 2)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 2)[0]
    cap = synth.net_caps(nl.n_nets, 2)
    size = synth.cell_sizes(nl.n_gates, 2)[0]
    for hyb in (False, True):
        f = o.forward(p, cap, size, hybrid=hyb, n_words=16, seed=4)
        adj = o.adjoint(f["sp"], f["beta"], cap, size)
        euler = float((cap.astype(np.float64) * adj["dcap"]).sum())
        assert euler == pytest.approx(f["power"], rel=1e-12)
        f2 = o.forward(p, 2 * cap, size, hybrid=hyb, n_words=16, seed=4)
        assert f2["power"] == pytest.approx(2 * f["power"], rel=1e-13)
        # sizes scale the driven net's load: s_g dP/ds_g summed = gate-net power
        gsum = float((size.astype(np.float64) * adj["dsize"]).sum())
        pi_part = float((f["beta"] * f["ceff"] * f["tr_model"])[: nl.n_pi].sum()) * 0.5
        assert gsum + pi_part == pytest.approx(f["power"], rel=1e-12)


def test_beta_rules():
    """Eq. 5 clip bounds and the zero-denominator reading (0/0 -> 1,
    x/0 -> beta_max)."""
    nl = synth.from_gates(3, [(synth.BUF, [0]), (synth.BUF, [1]), (synth.BUF, [2])])
    o = oracle.Netlist.of(nl)
    T = 4
    rng = np.random.default_rng(0)
    w = np.zeros((3, T), dtype=np.uint64)
    w[1] = rng.integers(0, 2**63, T, dtype=np.uint64)  # toggling although p = 0
    w[2] = np.uint64(2**64 - 1)                           # constant 1 at p = 1/2
    P = o.sp([0.0, 0.0, 0.5])
    ones, tog = o.sim(T, pi_words=w)
    out = o.power(P, np.ones(6, np.float32), hybrid=True, ones=ones, toggles=tog, n_words=T)
    assert out["beta"][0] == 1.0            # 0 / 0
    assert out["beta"][1] == 10.0           # x / 0
    assert out["beta"][2] == 0.1            # 0 / 0.5, clipped at beta_min
    assert out["tr_acc"][1] == pytest.approx(tog[1] / (64 * (T - 1)))


def test_sp_acc_reconvergent_exact():
    """Exhaustive stimulus at p = 1/2 gives SP_acc = exact P(net = 1),
    capturing reconvergence that the modeled SP misses."""
    nl = _reconvergent_small(3)
    o = oracle.Netlist.of(nl)
    T = 3
    w = np.repeat(brute.pack_minterm_words(nl.n_pi)[:, None], T, axis=1)
    p = np.full(nl.n_pi, 0.5)
    out = o.forward(p.astype(np.float32), np.ones(nl.n_nets, np.float32), hybrid=True, n_words=T,
                    pi_words=w)
    exact = brute.exact_probabilities(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin, p)
    np.testing.assert_allclose(out["sp_acc"], exact, atol=1e-15)


# ----------------------------------------------------------------- adjoint
def _fd_tol(g_fd, power, h):
    return 1e-4 * abs(g_fd) + 4 * np.finfo(np.float64).eps * abs(power) / h


@pytest.mark.parametrize("hybrid", [False, True])
def test_adjoint_complex_step_all_pis(hybrid):
    """Eq. 7 against the complex-step derivative (no cancellation) for every
    PI of the 2,000-gate DAG, beta frozen."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 1)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 1)[0]
    cap = synth.net_caps(nl.n_nets, 1)
    size = synth.cell_sizes(nl.n_gates, 1)[0]
    f = o.forward(p, cap, size, hybrid=hybrid, n_words=8, seed=3)
    adj = o.adjoint(f["sp"], f["beta"], cap, size)
    p64 = p.astype(np.float64)
    cs = np.array([o.power_complex_step(p64, f["beta"], f["ceff"], i) for i in range(nl.n_pi)])
    np.testing.assert_allclose(adj["dpi"], cs, rtol=1e-11, atol=1e-12 * np.abs(cs).max())


def test_adjoint_central_fd_all_pis():
    """FP64 central differences, h = 1e-6, on all 64 PIs (beta frozen)."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 5)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 5)[0]
    cap = synth.net_caps(nl.n_nets, 5)
    f = o.forward(p, cap, hybrid=True, n_words=8, seed=11)
    adj = o.adjoint(f["sp"], f["beta"], cap)
    h = 1e-6
    p64 = p.astype(np.float64)
    for i in range(nl.n_pi):
        e = np.zeros_like(p64)
        e[i] = h
        g = (o.frozen_power(p64 + e, f["beta"], cap) - o.frozen_power(p64 - e, f["beta"], cap)) / (2 * h)
        assert abs(adj["dpi"][i] - g) <= _fd_tol(g, f["power"], h), i


def test_adjoint_and_chain_closed_form():
    """AND chain y = prod p_i, power only on y: dP/dp_i = kappa C 2(1-2y)
    prod_{j != i} p_j."""
    n = 6
    p = np.array([0.9, 0.8, 0.85, 0.7, 0.95, 0.6])
    gates = [(synth.AND2, [0, 1])] + [(synth.AND2, [n + k, k + 2]) for k in range(n - 2)]
    nl = synth.from_gates(n, gates)
    o = oracle.Netlist.of(nl)
    cap = np.zeros(nl.n_nets, np.float32)
    cap[-1] = 3.0
    P = o.sp(p)
    adj = o.adjoint(P, np.ones(nl.n_nets), cap, kappa=0.5)
    y = np.prod(p)
    for i in range(n):
        want = 0.5 * 3.0 * 2 * (1 - 2 * y) * np.prod(np.delete(p, i))
        assert adj["dpi"][i] == pytest.approx(want, rel=1e-13)


def test_adjoint_beta_modes():
    """Eq. 6 taken literally (beta_ste) equals the local-beta gradient when
    beta = 1, and on a BUF chain compounds the betas along the path."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 4)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 4)[0]
    cap = synth.net_caps(nl.n_nets, 4)
    P = o.sp(p)
    one = np.ones(nl.n_nets)
    a = o.adjoint(P, one, cap)
    b = o.adjoint(P, one, cap, beta_ste=True)
    np.testing.assert_allclose(a["lam"], b["lam"], rtol=1e-15, atol=0)
    chain = synth.from_gates(1, [(synth.BUF, [0]), (synth.BUF, [1])])
    oc = oracle.Netlist.of(chain)
    Pc = oc.sp([0.25])
    beta = np.array([2.0, 3.0, 0.5])
    capc = np.array([0.0, 0.0, 1.0], np.float32)
    lam = oc.adjoint(Pc, beta, capc, kappa=1.0, beta_ste=True)["lam"]
    local = 1.0 * 2 * (1 - 2 * 0.25)
    assert lam[2] == pytest.approx(0.5 * local)
    assert lam[0] == pytest.approx(2.0 * 3.0 * 0.5 * local)
    lam_l = oc.adjoint(Pc, beta, capc, kappa=1.0)["lam"]
    assert lam_l[0] == pytest.approx(0.5 * local)


def test_adjoint_ste_is_the_derivative_of_its_surrogate():
    """Eq. 6 read literally (beta_ste) is reverse mode through a surrogate
    forward in which every net passes on y_n = beta_n x_n + (1 - beta_n) x*_n
    (x*_n its value at the base point: the same value, slope beta_n) and the
    power is sum_n kappa C_n 2 y_n (1 - y_n).  The surrogate's complex-step
    derivative, from a minterm-sum forward written here, equals the STE
    adjoint at every PI of a random DAG whose betas are far from 1."""
    nl = synth.random_dag(synth.DagSpec(n_gates=300, n_pi=12, depth=10), 7)
    o = oracle.Netlist.of(nl)
    rng = np.random.default_rng(7)
    p = rng.uniform(0.1, 0.9, nl.n_pi)
    cap = synth.net_caps(nl.n_nets, 7)
    beta = rng.uniform(0.3, 2.5, nl.n_nets)
    kappa = 0.5
    gate_order = np.argsort(o.levels()[nl.n_pi:], kind="stable")

    def surrogate(dp, slope, base):
        y = np.zeros(nl.n_nets, dtype=complex)
        y[: nl.n_pi] = p + slope[: nl.n_pi] * dp  # x* = p at a PI
        for g in gate_order:
            fan = nl.fanin[nl.fanin_ptr[g]:nl.fanin_ptr[g + 1]]
            x = brute.gate_probability(int(nl.op[g]), [y[i] for i in fan])
            n = nl.n_pi + g
            y[n] = slope[n] * x + (1 - slope[n]) * base[n]
        return y, sum(kappa * float(cap[n]) * 2 * y[n] * (1 - y[n]) for n in range(nl.n_nets))

    ones = np.ones(nl.n_nets)
    base = surrogate(np.zeros(nl.n_pi), ones, np.zeros(nl.n_nets))[0].real  # plain forward
    y0 = surrogate(np.zeros(nl.n_pi), beta, base)[0]
    np.testing.assert_allclose(y0.real, base, rtol=0, atol=1e-14)  # the same values, any beta
    P = o.sp(p)
    np.testing.assert_allclose(base, P, rtol=0, atol=1e-14)
    lam = o.adjoint(P, beta, cap, kappa=kappa, beta_ste=True)["lam"]
    h = 1e-30
    cs = np.array([surrogate(np.eye(nl.n_pi)[i] * 1j * h, beta, base)[1].imag / h
                   for i in range(nl.n_pi)])
    np.testing.assert_allclose(lam[: nl.n_pi], cs, rtol=1e-12, atol=1e-14 * np.abs(cs).max())
    # and it is not the local-beta gradient, which the surrogate does not give
    lam_local = o.adjoint(P, beta, cap, kappa=kappa)["lam"]
    assert np.abs(lam_local[: nl.n_pi] - cs).max() > 1e-3 * np.abs(cs).max()


def test_stimulus_threshold_boundary():
    """A lane whose uniform equals the threshold exactly is 0 (strict u < thr):
    find a Philox output with 8 trailing zero bits, so u / 2^32 is a float32,
    and use that value as the PI probability."""
    seed = 77
    key = [seed, 0]
    for t in range(4096):
        u = brute.philox4x32_10([t, 0, 0, 0], key)
        lane = next((l for l in range(4) if u[l] % 256 == 0 and u[l] > 0), None)
        if lane is not None:
            break
    else:  # pragma: no cover
        pytest.skip("no suitable draw")
    p = np.float32(u[lane] / 2**32)
    assert float(p) * 2**32 == u[lane]
    w = oracle.stimulus(np.array([p]), seed, t0=t, n_words=1)
    assert (int(w[0, 0]) >> lane) & 1 == 0
    w2 = oracle.stimulus(np.array([np.nextafter(p, np.float32(1))]), seed, t0=t, n_words=1)
    assert (int(w2[0, 0]) >> lane) & 1 == 1


def test_sim_ranges_add_up():
    """Counts over disjoint cycle ranges sum to the counts of their union, and
    the range form agrees with explicit stimulus words."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 8)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 8)[0]
    T = 37
    ones, tog = o.sim(T, p_pi=p, seed=21)
    parts = [(0, 1), (1, 10), (10, 11), (11, 37)]
    so = np.zeros_like(ones)
    st = np.zeros_like(tog)
    for a, b in parts:
        x, y = o.sim_range(a, b, p, seed=21)
        so += x
        st += y
    np.testing.assert_array_equal(so, ones)
    np.testing.assert_array_equal(st, tog)
    w = oracle.stimulus(p, 21, 0, T)
    ones2, tog2 = o.sim(T, pi_words=w)
    np.testing.assert_array_equal(ones2, ones)
    np.testing.assert_array_equal(tog2, tog)


# ---------------------------------------------------------------- power virus (Alg. 4)
def _virus_brute(nl, v0, cap):
    """Eq. 3 at net level by brute force: evaluate every net under v0 and
    under its complement v1 = 1 - v0 (all assignments enumerated)."""
    vals = brute.eval_all_minterms(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin)
    m0 = sum(int(b) << i for i, b in enumerate(v0))
    m1 = ((1 << nl.n_pi) - 1) ^ m0
    toggled = vals[:, m0] != vals[:, m1]
    return float(np.asarray(cap, dtype=np.float64)[toggled].sum())


@pytest.mark.parametrize("seed", range(6))
def test_virus_power_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    nl = synth.random_dag(synth.DagSpec(n_gates=40, n_pi=8, depth=6), seed)
    cap = synth.net_caps(nl.n_nets, seed)
    o = oracle.Netlist.of(nl)
    for _ in range(5):
        v0 = rng.integers(0, 2, nl.n_pi).astype(np.uint8)
        assert o.virus_power(v0, cap) == pytest.approx(_virus_brute(nl, v0, cap), rel=1e-12)


def test_virus_power_closed_forms():
    # a BUF/INV chain toggles everywhere: P_virus = sum of all caps
    gates = [(synth.INV, [0])] + [(synth.BUF if k % 2 else synth.INV, [k]) for k in range(1, 6)]
    nl = synth.from_gates(1, gates)
    cap = synth.net_caps(nl.n_nets, 3)
    o = oracle.Netlist.of(nl)
    for v in (0, 1):
        assert o.virus_power(np.array([v], np.uint8), cap) == pytest.approx(float(cap.sum()))
    # XOR of two toggling inputs never toggles; AND toggles only from (1, 1)
    nl = synth.from_gates(2, [(synth.XOR2, [0, 1]), (synth.AND2, [0, 1])])
    cap = np.array([1.0, 2.0, 4.0, 8.0], np.float32)
    o = oracle.Netlist.of(nl)
    assert o.virus_power(np.array([1, 0], np.uint8), cap) == pytest.approx(3.0)
    assert o.virus_power(np.array([1, 1], np.uint8), cap) == pytest.approx(11.0)
    assert o.virus_power(np.array([0, 0], np.uint8), cap) == pytest.approx(11.0)


def test_virus_ascent_step_is_the_proxy_gradient():
    """One step moves each unclipped startpoint by eta times the derivative
    of the Eq. 9 proxy, taken independently by the complex-step method."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 4)
    cap = synth.net_caps(nl.n_nets, 4)
    o = oracle.Netlist.of(nl)
    rng = np.random.default_rng(4)
    p0 = rng.uniform(0.2, 0.8, nl.n_pi)
    beta = rng.uniform(0.5, 2.0, nl.n_nets)
    eta = 1e-3
    p1, _, _ = o.power_virus(p0, cap, steps=1, eta=eta, beta=beta)
    ceff = cap.astype(np.float64)
    for i in range(0, nl.n_pi, 7):
        g = o.power_complex_step(p0, beta, ceff, i, kappa=1.0)
        assert (p1[i] - p0[i]) / eta == pytest.approx(g, rel=1e-9, abs=1e-12)


def test_virus_ascent_raises_the_proxy_and_thresholds():
    nl = synth.random_dag(synth.SPECS["dag2k"], 5)
    cap = synth.net_caps(nl.n_nets, 5)
    o = oracle.Netlist.of(nl)
    proxy = []
    for steps in range(0, 12, 2):
        p, v0, pv = o.power_virus(np.full(nl.n_pi, 0.5), cap, steps=steps, eta=1e-3)
        P = o.sp(p)
        proxy.append(o.power(P, cap, kappa=1.0)["power"])
        np.testing.assert_array_equal(v0, (p >= 0.5).astype(np.uint8))
        assert pv == pytest.approx(o.virus_power(v0, cap))
        assert ((p >= 0.0) & (p <= 1.0)).all()
    assert all(b >= a - 1e-9 for a, b in zip(proxy, proxy[1:]))


# ---------------------------------------------------------------- internal adjoints, Eq. 8 score
def _fd_internal(o, p, beta, cap, nets, h=1e-6):
    """Central differences of the frozen-beta power with one net's SP
    shifted (the SP-override hook), for each net in `nets`."""
    out = []
    for n in nets:
        up = o.power(o.sp_override(p, n, h), cap, beta=beta)["power"]
        dn = o.power(o.sp_override(p, n, -h), cap, beta=beta)["power"]
        out.append((up - dn) / (2 * h))
    return np.array(out)


@pytest.mark.parametrize("hybrid_beta", [False, True])
def test_internal_adjoint_equals_finite_differences(hybrid_beta):
    nl = synth.random_dag(synth.SPECS["dag2k"], 9)
    cap = synth.net_caps(nl.n_nets, 9)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 9)[0].astype(np.float64)
    rng = np.random.default_rng(9)
    beta = rng.uniform(0.5, 2.0, nl.n_nets) if hybrid_beta else np.ones(nl.n_nets)
    P = o.sp(p)
    lam = o.adjoint(P, beta, cap)["lam"]
    nets = np.concatenate([rng.choice(nl.n_pi, 10, replace=False),
                           nl.n_pi + rng.choice(nl.n_gates, 60, replace=False)])
    nets = [n for n in nets if 1e-3 < P[n] < 1 - 1e-3]
    fd = _fd_internal(o, p, beta, cap, nets)
    total = o.power(P, cap, beta=beta)["power"]
    tol = 1e-4 * np.abs(fd) + 4 * np.finfo(np.float64).eps * abs(total) / 1e-6
    assert (np.abs(lam[nets] - fd) <= tol).all()


def test_sizing_score_equals_chain_rule_by_differences():
    """Eq. 8 through Eq. 2, checked with a ratio of central differences:
    dP/dalpha_n = dP_total / dalpha_n as P_n is shifted, times the local
    power kappa beta C alpha_n."""
    nl = synth.random_dag(synth.SPECS["dag2k"], 10)
    cap = synth.net_caps(nl.n_nets, 10)
    o = oracle.Netlist.of(nl)
    p = synth.pi_probs(nl.n_pi, 10)[0].astype(np.float64)
    beta = np.ones(nl.n_nets)
    P = o.sp(p)
    S = o.sizing_score(P, o.adjoint(P, beta, cap)["lam"])
    rng = np.random.default_rng(10)
    h, kappa = 1e-6, 0.5
    checked = 0
    for g in rng.choice(nl.n_gates, 80, replace=False):
        n = nl.n_pi + g
        if not (abs(1 - 2 * P[n]) > 0.05 and 1e-3 < P[n] < 1 - 1e-3):
            continue
        dP = (o.power(o.sp_override(p, n, h), cap, beta=beta)["power"]
              - o.power(o.sp_override(p, n, -h), cap, beta=beta)["power"])
        a_up, a_dn = 2 * (P[n] + h) * (1 - P[n] - h), 2 * (P[n] - h) * (1 - P[n] + h)
        local = kappa * cap[n] * 2 * P[n] * (1 - P[n])
        s_fd = abs(dP / (a_up - a_dn)) / (kappa * cap[n]) * local
        assert S[g] == pytest.approx(s_fd, rel=1e-4)
        checked += 1
    assert checked > 40
    # the flat point: P = 1/2 uses the floor, never divides by zero
    assert np.isfinite(o.sizing_score(np.full(nl.n_nets, 0.5), np.ones(nl.n_nets))).all()


def test_rank_metrics():
    from paper_2608_03778_amd import rank
    a = np.array([5.0, -4.0, 3.0, 0.5, 0.1])
    assert list(rank.top_k(a, 2)) == [0, 1]
    assert rank.top_k_overlap(a, a * 2, 3) == 1.0
    assert rank.top_k_overlap(a, [0.1, 0.2, 0.3, 9.0, 8.0], 2) == 0.0
    assert rank.jaccard_top_k(a, [5.0, 0.0, 3.0, 4.0, 0.0], 2) == pytest.approx(1 / 3)
    assert rank.pearson(a, 2 * a + 1) == pytest.approx(1.0)
    assert rank.pearson(a, -a) == pytest.approx(-1.0)
