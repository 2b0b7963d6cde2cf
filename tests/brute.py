"""Brute-force references that share nothing with the oracle or the HIP path.

Cells are defined here by their Boolean functions, written as Python boolean
expressions; signal probabilities come from summing minterm weights over all
input assignments, derivatives from differentiating those sums, simulation
counts from evaluating the circuit on every assignment.
"""
from __future__ import annotations

import itertools

import numpy as np

# Boolean definition of each cell (pin order as in the library header).
TRUTH = {
    0: lambda a: not a,                              # INV
    1: lambda a: a,                                  # BUF
    2: lambda a, b: a and b,                         # AND2
    3: lambda a, b: a or b,                          # OR2
    4: lambda a, b: not (a and b),                   # NAND2
    5: lambda a, b: not (a or b),                    # NOR2
    6: lambda a, b: a != b,                          # XOR2
    7: lambda a1, a2, b: not ((a1 and a2) or b),     # AOI21
    8: lambda i0, i1, s: i1 if s else i0,            # MUX2
}
ARITY = {0: 1, 1: 1, 2: 2, 3: 2, 4: 2, 5: 2, 6: 2, 7: 3, 8: 3}


def minterm_weight(m, p):
    w = 1.0
    for bit, pk in zip(m, p):
        w *= pk if bit else (1.0 - pk)
    return w


def gate_probability(op, p):
    """P(out = 1) with independent inputs, by enumeration of minterms."""
    return sum(minterm_weight(m, p) for m in itertools.product((0, 1), repeat=ARITY[op])
               if TRUTH[op](*map(bool, m)))


def gate_probability_grad(op, p):
    """d P(out = 1) / d p_k by differentiating the minterm sum term by term."""
    k = ARITY[op]
    g = np.zeros(k)
    for m in itertools.product((0, 1), repeat=k):
        if not TRUTH[op](*map(bool, m)):
            continue
        for j in range(k):
            rest = minterm_weight([b for i, b in enumerate(m) if i != j],
                                  [q for i, q in enumerate(p) if i != j])
            g[j] += rest if m[j] else -rest
    return g


def eval_all_minterms(n_pi, op, fanin_ptr, fanin):
    """Boolean value of every net under every PI assignment.

    Returns bool [n_nets][2**n_pi]; column m assigns PI i the bit i of m.
    Gates are evaluated by repeated sweeps until every gate is resolved, so
    the caller's gate order need not be topological.
    """
    M = 1 << n_pi
    G = len(op)
    vals = np.zeros((n_pi + G, M), dtype=bool)
    idx = np.arange(M)
    for i in range(n_pi):
        vals[i] = (idx >> i) & 1
    done = np.zeros(n_pi + G, dtype=bool)
    done[:n_pi] = True
    vec = {o: np.vectorize(TRUTH[o], otypes=[bool]) for o in TRUTH}
    while not done.all():
        progress = False
        for g in range(G):
            if done[n_pi + g]:
                continue
            ins = fanin[fanin_ptr[g]:fanin_ptr[g + 1]]
            if all(done[n] for n in ins):
                vals[n_pi + g] = vec[int(op[g])](*[vals[n] for n in ins])
                done[n_pi + g] = True
                progress = True
        if not progress:
            raise ValueError("cycle")
    return vals


def exact_probabilities(n_pi, op, fanin_ptr, fanin, p):
    """Exact P(net = 1) for independent PIs, by enumerating all assignments
    (valid with reconvergence too)."""
    vals = eval_all_minterms(n_pi, op, fanin_ptr, fanin)
    M = 1 << n_pi
    idx = np.arange(M)
    w = np.ones(M)
    for i in range(n_pi):
        bit = (idx >> i) & 1
        w *= np.where(bit == 1, p[i], 1.0 - p[i])
    return vals.astype(np.float64) @ w


def pack_minterm_words(n_pi):
    """One 64-bit word per PI whose 64 lanes enumerate all 2**n_pi (<= 64)
    assignments (lane m assigns PI i the bit i of m, lanes repeat)."""
    assert n_pi <= 6
    words = []
    for i in range(n_pi):
        w = 0
        for lane in range(64):
            if (lane >> i) & 1:
                w |= 1 << lane
        words.append(w)
    return np.array(words, dtype=np.uint64)


def popcount(x: int) -> int:
    return bin(int(x)).count("1")


# -- Philox4x32-10 written from Salmon et al., SC'11, independently of the
#    oracle's C implementation.
_M0, _M1 = 0xD2511F53, 0xCD9E8D57
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(x) & _MASK for x in ctr)
    k0, k1 = (int(x) & _MASK for x in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        prod0 = _M0 * c0
        prod1 = _M1 * c2
        c0, c1, c2, c3 = ((prod1 >> 32) ^ c1 ^ k0, prod1 & _MASK,
                          (prod0 >> 32) ^ c3 ^ k1, prod0 & _MASK)
    return [c0, c1, c2, c3]


def markov_words(p, tau, stream, seed, n_words):
    """Startpoint stimulus with transition rates and shared streams, written
    from the definition independently of the oracle: lane j of startpoint i
    starts from Bernoulli(p) and then keeps 1 with probability
    1 - tau / (2p) and rises from 0 with probability tau / (2 (1 - p)),
    each cycle's draw being lane j mod 4 of Philox(t, stream_i, j div 4)."""
    import math

    def thr(x):
        v = x * 4294967296.0
        return 0 if not v > 0 else (1 << 32 if v >= 4294967296.0 else math.floor(v))

    key = (seed & _MASK, seed >> 32)
    out = []
    for i, pi in enumerate(p):
        pf = float(np.float32(pi))
        s = i if stream is None else int(stream[i])
        t_p = thr(pf)
        if tau is None:
            t_rise = t_stay = t_p
        else:
            tf = float(np.float32(tau[i]))
            if pf <= 0:
                rise, stay = 0.0, 0.0
            elif pf >= 1:
                rise, stay = 1.0, 1.0
            else:
                rise, stay = min(tf / (2.0 * (1.0 - pf)), 1.0), max(1.0 - tf / (2.0 * pf), 0.0)
            t_rise, t_stay = thr(rise), thr(stay)
        state = [0] * 64
        row = []
        for t in range(n_words):
            w = 0
            for j in range(64):
                u = philox4x32_10((t, s, j // 4, 0), key)[j % 4]
                limit = t_p if t == 0 else (t_stay if state[j] else t_rise)
                state[j] = 1 if u < limit else 0
                w |= state[j] << j
            row.append(w)
        out.append(row)
    return np.array(out, dtype=np.uint64)
