"""Seeded synthetic netlists and query inputs.

This module only draws random structures and values; it holds none of the
power model's arithmetic (no signal probabilities, no simulation, no power).
Both the HIP path and the CPU oracle are fed from it, so they see identical
inputs.

The paper evaluates on proprietary and IWLS 2005 netlists (Sec. V-A) that
are not available here.  The stand-ins are random levelized combinational
DAGs shaped like the paper's designs (cells, pins per cell and depth of
Table III) and like the workload sizes this project measures:

* ``depth`` levels of equal width (remainder spread over the first levels);
  level 0 holds the primary inputs (PIs);
* gate types i.i.d. uniform over the nine fixed cells;
* pin 0 of a gate at level L reads a net of level L-1, so the gate's
  as-soon-as-possible level is exactly L;
* every other pin, with probability ``reconv``, reads one of the fan-in
  nets of pin 0's driver gate (a two-path reconvergence); otherwise it reads
  a net of any level < L, drawn with weight equal to that net's remaining
  fan-out budget;
* fan-out budgets are Geometric(mean ``fo_mean``) truncated at ``fo_cap``,
  with a heavy tail: with probability 1e-3 a budget is LogUniform[4 mean, cap];
* the inputs of one gate are distinct nets;
* the caller's gate numbering is a random permutation of the level order, so
  consumers of a netlist must levelize it themselves.

Values: PI probabilities U(lo, hi) as float32, net capacitances
LogNormal(ln 2 fF, 0.5) as float32, per-gate size factors uniform over
{0.5, 1, 2, 4}.
"""
from __future__ import annotations

import dataclasses
import math
import re

import numpy as np

# Opcode numbering of the nine fixed cells.  The C-ABI header and the oracle
# each declare the same numbering on their own; it is an interface, not code.
INV, BUF, AND2, OR2, NAND2, NOR2, XOR2, AOI21, MUX2 = range(9)
CELL_BASE = 16  # gate opcode of library cell c
OP_NAMES = ("INV", "BUF", "AND2", "OR2", "NAND2", "NOR2", "XOR2", "AOI21", "MUX2")
ARITY = np.array([1, 1, 2, 2, 2, 2, 2, 3, 3], dtype=np.int32)


@dataclasses.dataclass
class Netlist:
    """A gate netlist in the caller's numbering.

    Net ids: ``[0, n_pi)`` are PIs; ``n_pi + g`` is the output net of gate g.
    ``fanin[fanin_ptr[g]:fanin_ptr[g+1]]`` are gate g's input nets in pin
    order (INV/BUF: A; 2-input: A, B; AOI21: A1, A2, B; MUX2: I0, I1, S).
    """

    n_pi: int
    op: np.ndarray         # uint8 [G]
    fanin_ptr: np.ndarray  # int32 [G+1]
    fanin: np.ndarray      # int32 [sum of arities]
    stats: dict = dataclasses.field(default_factory=dict)
    # library cells (Boolean expressions); gate opcode CELL_BASE + c is cell c
    cells: tuple = ()
    # per cell, its pin names in fan-in order ("I0,I1,S"), or None for the
    # expression's identifiers in order of first appearance; () = all None
    pins: tuple = ()

    @property
    def n_gates(self) -> int:
        return int(self.op.shape[0])

    @property
    def n_nets(self) -> int:
        return self.n_pi + self.n_gates


def cell_arity(expr: str) -> int:
    """Inputs of a library cell: its distinct identifiers."""
    return len(dict.fromkeys(re.findall(r"[A-Za-z_][A-Za-z0-9_]*", expr)))


def arity_table(cells=()) -> np.ndarray:
    """Arity of every opcode: the nine fixed cells, then the library."""
    t = np.zeros(CELL_BASE + len(cells), dtype=np.int32)
    t[:9] = ARITY
    for c, e in enumerate(cells):
        t[CELL_BASE + c] = cell_arity(e)
    return t


# A small cell library for the generic-cell workloads: read-once cells with
# up to six inputs, a read-many majority, the multiplexer as an expression
# and a constant.
LIBRARY = (
    "!((A1&A2)|(B1&B2))",    # AOI22
    "!((A1|A2)&B)",          # OAI21
    "A&B|A&C|B&C",           # MAJ3 (inputs read twice)
    "!(A^B)",                # XNOR2
    "(A&B)|(C&D)|(E&F)",     # AO222
    "(I0&!S)|(I1&S)",        # MUX2 written out (S read twice)
    "A&!B",                  # AND with an inverted input
    "A|B|C|D",               # OR4
    "1^A",                   # a constant operand
)


@dataclasses.dataclass
class DagSpec:
    n_gates: int
    n_pi: int
    depth: int
    reconv: float = 0.3
    fo_mean: float = 2.5
    fo_cap: int = 64
    ops: tuple = tuple(range(9))
    cells: tuple = ()


# The workloads measured by this project (sizes, PI counts, depths, fan-out).
SPECS = {
    "dag2k": DagSpec(n_gates=2_000, n_pi=64, depth=20),
    "dag117k": DagSpec(n_gates=117_000, n_pi=2_048, depth=60),
    "dag2m": DagSpec(n_gates=2_000_000, n_pi=16_384, depth=120, fo_mean=3.0, fo_cap=256),
    # serving designs: (n_pi, depth) log-interpolated between the three above
    "dag10k": DagSpec(n_gates=10_000, n_pi=256, depth=30),
    "dag50k": DagSpec(n_gates=50_000, n_pi=1_024, depth=45),
    "dag300k": DagSpec(n_gates=300_000, n_pi=4_096, depth=75, fo_mean=3.0, fo_cap=256),
    "dag500k": DagSpec(n_gates=500_000, n_pi=6_144, depth=85, fo_mean=3.0, fo_cap=256),
    "dag1m": DagSpec(n_gates=1_000_000, n_pi=8_192, depth=100, fo_mean=3.0, fo_cap=256),
    "dag1500k": DagSpec(n_gates=1_500_000, n_pi=12_288, depth=110, fo_mean=3.0, fo_cap=256),
}


def _budgets(rng: np.random.Generator, n: int, mean: float, cap: int) -> np.ndarray:
    b = rng.geometric(1.0 / mean, size=n).astype(np.int64)
    np.minimum(b, cap, out=b)
    tail = rng.random(n) < 1e-3
    if tail.any():
        lo, hi = math.log(4.0 * mean), math.log(float(cap))
        if hi > lo:
            b[tail] = np.rint(np.exp(rng.uniform(lo, hi, size=int(tail.sum())))).astype(np.int64)
    return b


def _weighted_pick(rng, cdf: np.ndarray, k: int) -> np.ndarray:
    """Indices drawn with probability proportional to the increments of cdf."""
    u = rng.random(k) * cdf[-1]
    idx = np.searchsorted(cdf, u, side="right")
    return np.minimum(idx, cdf.shape[0] - 1)


def random_dag(spec: DagSpec, seed: int) -> Netlist:
    """A random levelized DAG following the recipe in the module docstring."""
    rng = np.random.default_rng(seed)
    G, n_pi, D = spec.n_gates, spec.n_pi, spec.depth
    if D < 1 or G < D:
        raise ValueError("need at least one gate per level")
    ops_choice = np.asarray(spec.ops, dtype=np.int32)
    arity = arity_table(spec.cells)
    kmax = max(3, int(arity[ops_choice].max()))
    widths = np.full(D, G // D, dtype=np.int64)
    widths[: G % D] += 1
    n_nets = n_pi + G
    # generator-internal net ids are level ordered: PIs, then level 1, ...
    lvl_start = np.zeros(D + 2, dtype=np.int64)
    lvl_start[1] = n_pi
    lvl_start[2:] = n_pi + np.cumsum(widths)
    budget = _budgets(rng, n_nets, spec.fo_mean, spec.fo_cap)
    op = np.empty(G, dtype=np.uint8)
    pins = np.full((G, kmax), -1, dtype=np.int64)
    n_reconv = 0
    n_other = 0
    for L in range(1, D + 1):
        a, b = lvl_start[L] - n_pi, lvl_start[L + 1] - n_pi  # gate range
        w = int(b - a)
        gop = ops_choice[rng.integers(0, ops_choice.shape[0], size=w)]
        op[a:b] = gop
        k = arity[gop]
        # weights: remaining budget, with a floor so exhausted nets stay reachable
        wts = np.maximum(budget[: lvl_start[L]], 0).astype(np.float64) + 1e-3
        prev_lo, prev_hi = lvl_start[L - 1], lvl_start[L]
        cdf_prev = np.cumsum(wts[prev_lo:prev_hi])
        cdf_all = np.cumsum(wts)
        p0 = prev_lo + _weighted_pick(rng, cdf_prev, w)
        pins[a:b, 0] = p0
        for j in range(1, kmax):
            need = np.nonzero(k > j)[0]
            if need.size == 0:
                continue
            n_other += need.size
            choice = _weighted_pick(rng, cdf_all, need.size)
            drv = p0[need] - n_pi  # driver gate of pin 0 (negative => PI)
            want = (rng.random(need.size) < spec.reconv) & (drv >= 0)
            if want.any():
                dg = drv[want]
                dk = arity[op[dg]]
                slot = (rng.random(dg.size) * dk).astype(np.int64)
                choice[want] = pins[dg, slot]
                n_reconv += int(want.sum())
            pins[a + need, j] = choice
        # enforce distinct inputs within a gate by redrawing colliding pins
        for _ in range(100):
            blk = pins[a:b]
            dups = []
            for j in range(1, kmax):
                dj = np.zeros(w, dtype=bool)
                for i in range(j):
                    dj |= blk[:, j] == blk[:, i]
                dups.append((j, (k > j) & dj))
            if not any(d.any() for _, d in dups):
                break
            for j, dup in dups:
                idx = np.nonzero(dup)[0]
                if idx.size:
                    pins[a + idx, j] = _weighted_pick(rng, cdf_all, idx.size)
        else:  # pragma: no cover - vanishingly unlikely
            raise RuntimeError("could not draw distinct fan-ins")
        used = pins[a:b][pins[a:b] >= 0]
        np.subtract.at(budget, used, 1)
    # shuffle the caller's gate numbering
    perm = rng.permutation(G)  # generator gate g -> caller gate perm[g]
    net_map = np.empty(n_nets, dtype=np.int64)
    net_map[:n_pi] = np.arange(n_pi)
    net_map[n_pi:] = n_pi + perm
    c_op = np.empty(G, dtype=np.uint8)
    c_op[perm] = op
    c_pins = np.full((G, kmax), -1, dtype=np.int64)
    m = pins >= 0
    mapped = np.where(m, net_map[np.where(m, pins, 0)], -1)
    c_pins[perm] = mapped
    k = arity[c_op]
    fanin_ptr = np.zeros(G + 1, dtype=np.int32)
    fanin_ptr[1:] = np.cumsum(k)
    mask = np.arange(kmax)[None, :] < k[:, None]
    fanin = c_pins[mask].astype(np.int32)
    fo = np.bincount(pins[m].ravel(), minlength=n_nets)
    stats = dict(
        n_gates=G, n_pi=n_pi, n_nets=n_nets, depth=D,
        level_width_min=int(widths.min()), level_width_max=int(widths.max()),
        fanin_edges=int(fanin.shape[0]),
        pins=int(n_nets + fanin.shape[0]),
        fanout_mean=float(fo.mean()), fanout_max=int(fo.max()),
        primary_outputs=int((fo == 0).sum()),
        reconvergent_pin_fraction=(n_reconv / n_other) if n_other else 0.0,
        seed=seed,
    )
    return Netlist(n_pi=n_pi, op=c_op, fanin_ptr=fanin_ptr, fanin=fanin, stats=stats,
                   cells=tuple(spec.cells))


def from_gates(n_pi: int, gates, cells=()) -> Netlist:
    """Build a netlist from a list of ``(op, [input nets])`` in caller order."""
    op = np.array([g[0] for g in gates], dtype=np.uint8)
    k = [len(g[1]) for g in gates]
    fanin_ptr = np.zeros(len(gates) + 1, dtype=np.int32)
    fanin_ptr[1:] = np.cumsum(k)
    fanin = np.array([n for g in gates for n in g[1]], dtype=np.int32)
    return Netlist(n_pi=n_pi, op=op, fanin_ptr=fanin_ptr, fanin=fanin, cells=tuple(cells))


def random_tree(n_leaves: int, seed: int, ops=tuple(range(9)), cells=()) -> Netlist:
    """A random fan-out-free tree: every net (PI or gate output) feeds at most
    one gate pin, so the inputs of every gate are independent signals."""
    rng = np.random.default_rng(seed)
    ops = np.asarray(ops, dtype=np.int32)
    ARITY = arity_table(cells)
    free = list(range(n_leaves))  # nets not yet consumed
    gates = []
    while len(free) > 1 or not gates:
        rng.shuffle(free)
        cand = [o for o in ops if ARITY[o] <= len(free)]
        o = int(cand[rng.integers(0, len(cand))])
        k = int(ARITY[o])
        ins = [free.pop() for _ in range(k)]
        gates.append((o, ins))
        free.append(n_leaves + len(gates) - 1)
        if len(gates) > 20 * n_leaves:
            break
    return from_gates(n_leaves, gates, cells)


# -- sequential boundaries (Sec. III-A: timing startpoints are primary inputs
#    and flip-flop outputs, endpoints are primary outputs and flip-flop inputs)

DFF = 255  # opcode of a flip-flop in a sequential netlist; it never reaches the library


@dataclasses.dataclass
class SeqNetlist:
    """A netlist with flip-flops: gate g with op DFF has one input, its D net,
    and its output net n_pi + g is the flop's Q.  Combinational cycles are
    allowed only through flops."""

    n_pi: int
    op: np.ndarray
    fanin_ptr: np.ndarray
    fanin: np.ndarray
    cells: tuple = ()


@dataclasses.dataclass
class Cut:
    """A sequential netlist cut at its flops into the combinational netlist
    the library evaluates: startpoints are the PIs and then one pseudo-PI per
    flop (flop order), gates keep their relative order."""

    netlist: Netlist
    ppi: np.ndarray      # int32 [n_ff] PI id of flop k's output in the cut netlist
    ppo: np.ndarray      # int32 [n_ff] cut net id of flop k's D input (an endpoint)
    stream: np.ndarray   # int32 [n_pi + n_ff] shared stream of every startpoint
    net_map: np.ndarray  # int32 [n_nets of the sequential netlist] -> cut net id


def cut_flops(seq: SeqNetlist) -> Cut:
    """Cut at the flops.  Pseudo-PIs of flops whose D inputs are one net carry
    one signal, so they share a stream (Sec. III-C): the stream of the first
    such flop's pseudo-PI."""
    op = np.asarray(seq.op)
    G = op.shape[0]
    is_ff = op == DFF
    ff = np.nonzero(is_ff)[0]
    comb = np.nonzero(~is_ff)[0]
    n_ff = ff.shape[0]
    n_start = seq.n_pi + n_ff
    net_map = np.empty(seq.n_pi + G, dtype=np.int32)
    net_map[: seq.n_pi] = np.arange(seq.n_pi)
    net_map[seq.n_pi + ff] = seq.n_pi + np.arange(n_ff)
    net_map[seq.n_pi + comb] = n_start + np.arange(comb.shape[0])
    gates = []
    for g in comb:
        ins = seq.fanin[seq.fanin_ptr[g]:seq.fanin_ptr[g + 1]]
        gates.append((int(op[g]), [int(net_map[n]) for n in ins]))
    for g in ff:
        if seq.fanin_ptr[g + 1] - seq.fanin_ptr[g] != 1:
            raise ValueError(f"flop {g} needs exactly one input")
    d_seq = np.array([seq.fanin[seq.fanin_ptr[g]] for g in ff], dtype=np.int64)
    ppo = net_map[d_seq].astype(np.int32) if n_ff else np.zeros(0, np.int32)
    stream = np.arange(n_start, dtype=np.int32)
    first = {}
    for k, dn in enumerate(d_seq.tolist()):
        stream[seq.n_pi + k] = seq.n_pi + first.setdefault(dn, k)
    nl = from_gates(n_start, gates, seq.cells)
    return Cut(netlist=nl, ppi=(seq.n_pi + np.arange(n_ff)).astype(np.int32), ppo=ppo,
               stream=stream, net_map=net_map)


def random_seq_dag(spec: DagSpec, n_ff: int, seed: int, shared: float = 0.25) -> SeqNetlist:
    """A sequential netlist: a random DAG over n_pi + n_ff startpoints whose
    last n_ff startpoints are flop outputs, each flop's D a random net (a
    fraction `shared` of the flops reuses another flop's D, so their outputs
    share a driver), flops and gates interleaved in a random order."""
    rng = np.random.default_rng(seed)
    comb = random_dag(dataclasses.replace(spec, n_pi=spec.n_pi + n_ff), seed)
    n_pi, G = spec.n_pi, comb.n_gates
    n_nets = comb.n_nets
    d = rng.integers(0, n_nets, n_ff)
    for k in range(1, n_ff):
        if rng.random() < shared:
            d[k] = d[rng.integers(0, k)]
    # sequential gate order: a random interleaving of the gates and the flops
    order = rng.permutation(G + n_ff)  # position -> (gate g < G, or flop g - G)
    pos = np.empty(G + n_ff, dtype=np.int64)
    pos[order] = np.arange(G + n_ff)
    seq_net = np.empty(n_nets, dtype=np.int64)  # combinational net -> sequential net
    seq_net[:n_pi] = np.arange(n_pi)
    seq_net[n_pi:n_pi + n_ff] = n_pi + pos[G + np.arange(n_ff)]
    seq_net[n_pi + n_ff:] = n_pi + pos[np.arange(G)]
    ops, fins = [], []
    for x in order:
        if x < G:
            ops.append(int(comb.op[x]))
            fins.append(seq_net[comb.fanin[comb.fanin_ptr[x]:comb.fanin_ptr[x + 1]]])
        else:
            ops.append(DFF)
            fins.append(seq_net[[d[x - G]]])
    fanin_ptr = np.zeros(G + n_ff + 1, dtype=np.int32)
    fanin_ptr[1:] = np.cumsum([len(f) for f in fins])
    return SeqNetlist(n_pi=n_pi, op=np.array(ops, dtype=np.uint8), fanin_ptr=fanin_ptr,
                      fanin=np.concatenate(fins).astype(np.int32), cells=tuple(spec.cells))


def pi_probs(n_pi: int, seed: int, batch: int = 1, lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """PI probabilities, float32 [batch][n_pi], U(lo, hi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(batch, n_pi)).astype(np.float32)


def net_caps(n_nets: int, seed: int) -> np.ndarray:
    """Net load capacitances in fF, float32, LogNormal(ln 2, 0.5)."""
    rng = np.random.default_rng(seed)
    return rng.lognormal(math.log(2.0), 0.5, size=n_nets).astype(np.float32)


def cell_sizes(n_gates: int, seed: int, n_size: int = 1) -> np.ndarray:
    """Per-gate size factors, float32 [n_size][n_gates], uniform on {0.5,1,2,4}."""
    rng = np.random.default_rng(seed)
    levels = np.array([0.5, 1.0, 2.0, 4.0], dtype=np.float32)
    return levels[rng.integers(0, 4, size=(n_size, n_gates))]
