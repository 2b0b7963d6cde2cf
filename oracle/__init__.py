"""DiffPower FP64 CPU oracle -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liborc.so`` (built from
``diffpower_oracle.c`` with gcc by ``oracle/build.py``) with ctypes and
numpy; it never loads or calls the HIP library, and the HIP library never
loads it.

Every function follows the paper (arXiv 2608.03778) passage named in the C
source.  The wrappers only marshal arrays and loop over query columns.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborc.so")

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_d = ctypes.c_double
_int = ctypes.c_int


def _declare(lib):
    lib.orc_threshold_d.argtypes = [_d]
    lib.orc_threshold_d.restype = _u64
    lib.orc_markov_probs.argtypes = [ctypes.c_float, ctypes.c_float, _p, _p]
    lib.orc_markov_probs.restype = None
    lib.orc_stimulus_model.argtypes = [_i32, _p, _p, _p, _u64, _i64, _p]
    lib.orc_stimulus_model.restype = None
    lib.orc_cell_compile.argtypes = [ctypes.c_char_p, _p, _p]
    lib.orc_cell_compile.restype = _int
    lib.orc_set_cells.argtypes = [_int, _p]
    lib.orc_set_cells.restype = _int
    lib.orc_op_arity.argtypes = [_int]
    lib.orc_op_arity.restype = _int
    lib.orc_topo_order.argtypes = [_i32, _i32, _p, _p, _p, _p]
    lib.orc_topo_order.restype = _int
    lib.orc_levels.argtypes = [_i32, _i32, _p, _p, _p, _p]
    lib.orc_levels.restype = None
    lib.orc_gate_sp.argtypes = [_int, _p]
    lib.orc_gate_sp.restype = _d
    lib.orc_gate_partials.argtypes = [_int, _p, _p]
    lib.orc_gate_partials.restype = None
    lib.orc_gate_bits.argtypes = [_int, _p]
    lib.orc_gate_bits.restype = _u64
    lib.orc_sp.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _p]
    lib.orc_sp.restype = None
    lib.orc_power_complex_step.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _p, _p, _d, _i32, _d]
    lib.orc_power_complex_step.restype = _d
    lib.orc_philox4x32_10.argtypes = [_p, _p, _p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_threshold.argtypes = [ctypes.c_float]
    lib.orc_threshold.restype = _u64
    lib.orc_stimulus_word.argtypes = [_i32, _i64, ctypes.c_float, _u64]
    lib.orc_stimulus_word.restype = _u64
    lib.orc_stimulus.argtypes = [_i32, _p, _u64, _i64, _i64, _p]
    lib.orc_stimulus.restype = None
    lib.orc_sim.argtypes = [_i32, _i32, _p, _p, _p, _p, _i64, _p, _p, _u64, _p, _p]
    lib.orc_sim.restype = None
    lib.orc_sim_range.argtypes = [_i32, _i32, _p, _p, _p, _p, _i64, _i64, _p, _u64, _p, _p]
    lib.orc_sim_range.restype = None
    lib.orc_power.argtypes = [_i32, _i32, _p, _p, _p, _i64, _p, _p, _d, _int, _d, _d, _p,
                              _p, _p, _p, _p, _p, _p]
    lib.orc_power.restype = _d
    lib.orc_adjoint.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _p, _p, _p, _d, _int, _p, _p, _p]
    lib.orc_adjoint.restype = None
    lib.orc_sp_override.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _i64, _d, _p]
    lib.orc_sp_override.restype = None
    lib.orc_sizing_score.argtypes = [_i32, _i32, _p, _p, _d, _p]
    lib.orc_sizing_score.restype = None
    lib.orc_virus_power.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _p]
    lib.orc_virus_power.restype = _d
    lib.orc_power_virus.argtypes = [_i32, _i32, _p, _p, _p, _p, _p, _p, _i32, _d, _p, _p]
    lib.orc_power_virus.restype = _d


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


CELL_BASE = 16  # opcode of library cell c is CELL_BASE + c
CODE_OPS = ("IN", "NOT", "AND", "OR", "XOR", "CONST0", "CONST1")


def cell_code(expr: str):
    """The oracle's post-order code of one cell expression: ([(op, arg)],
    n_inputs).  Raises ValueError on a syntax error."""
    code = np.zeros(64, dtype=np.uint16)
    n_in = ctypes.c_int(0)
    n = _load().orc_cell_compile(expr.encode(), _ptr(code), ctypes.byref(n_in))
    if n < 0:
        raise ValueError(f"cannot compile cell expression {expr!r}")
    return [(CODE_OPS[int(c) & 0xFF], int(c) >> 8) for c in code[:n]], n_in.value


def set_cells(exprs) -> None:
    """Register the cell library every later evaluation uses."""
    exprs = [e.encode() for e in (exprs or [])]
    arr = (ctypes.c_char_p * max(len(exprs), 1))(*exprs)
    rc = _load().orc_set_cells(len(exprs), ctypes.cast(arr, ctypes.c_void_p))
    if rc != 0:
        raise ValueError(f"cell {-rc - 1} does not compile")


def expression_inputs(expr: str):
    """A cell expression's identifiers in order of first appearance: the
    inputs the oracle's compiler numbers 0, 1, ... as it reads left to
    right."""
    import re
    seen = []
    for m in re.finditer(r"[A-Za-z_][A-Za-z0-9_]*", expr):
        if m.group(0) not in seen:
            seen.append(m.group(0))
    return seen


def _inputs_in_expression_order(op, fanin_ptr, fanin, cells, pins):
    """Reorder each library-cell gate's fan-in from its pin list's order
    (pins[c], names separated by commas or blanks) into the order of its
    expression's inputs (Alg. 1's perm), so the rest of the oracle reads
    input k at position k."""
    import re
    out = fanin.copy()
    for c, pl in enumerate(pins):
        if not pl:
            continue
        names = [x for x in re.split(r"[,\s]+", pl) if x]
        ids = expression_inputs(cells[c])
        if sorted(names) != sorted(ids) or len(set(names)) != len(names):
            raise ValueError(f"pin list {pl!r} does not match the inputs {ids} of cell {c}")
        src = [names.index(ident) for ident in ids]  # fan-in position of input k
        for g in np.nonzero(op == CELL_BASE + c)[0]:
            a = int(fanin_ptr[g])
            out[a:a + len(ids)] = fanin[[a + j for j in src]]
    return out


class Netlist:
    """The oracle's own copy of a netlist (caller numbering) plus its
    topological order.  Gates with opcode CELL_BASE + c are instances of
    cells[c], a Boolean expression."""

    def __init__(self, n_pi, op, fanin_ptr, fanin, cells=None, pins=None):
        lib = _load()
        self.cells = list(cells or [])
        set_cells(self.cells)
        self.n_pi = int(n_pi)
        self.op = _c(op, np.uint8)
        self.fanin_ptr = _c(fanin_ptr, np.int32)
        self.fanin = _c(fanin, np.int32)
        if pins and any(pins):
            self.fanin = _inputs_in_expression_order(self.op, self.fanin_ptr, self.fanin,
                                                     self.cells, list(pins))
        self.n_gates = int(self.op.shape[0])
        self.n_nets = self.n_pi + self.n_gates
        self.order = np.zeros(max(self.n_gates, 1), dtype=np.int32)
        rc = lib.orc_topo_order(self.n_pi, self.n_gates, _ptr(self.op), _ptr(self.fanin_ptr),
                                _ptr(self.fanin), _ptr(self.order))
        if rc == -1:
            raise ValueError("malformed netlist")
        if rc == -2:
            raise ValueError("combinational cycle")

    @classmethod
    def of(cls, nl):
        return cls(nl.n_pi, nl.op, nl.fanin_ptr, nl.fanin, getattr(nl, "cells", None),
                   getattr(nl, "pins", None))

    def _args(self):
        set_cells(self.cells)  # the library is process state: bind ours first
        return (self.n_pi, self.n_gates, _ptr(self.op), _ptr(self.fanin_ptr), _ptr(self.fanin),
                _ptr(self.order))

    def levels(self) -> np.ndarray:
        lv = np.zeros(self.n_nets, dtype=np.int32)
        set_cells(self.cells)
        _load().orc_levels(self.n_pi, self.n_gates, _ptr(self.fanin_ptr), _ptr(self.fanin),
                           _ptr(self.order), _ptr(lv))
        return lv

    def sp(self, p_pi) -> np.ndarray:
        """Modeled static probability of every net (float64 [n_nets])."""
        p = _c(p_pi, np.float64)
        P = np.zeros(self.n_nets, dtype=np.float64)
        _load().orc_sp(*self._args(), _ptr(p), _ptr(P))
        return P

    def sim(self, n_words, pi_words=None, p_pi=None, seed=0):
        """(ones, toggles) uint64 [n_nets] over n_words simulated words."""
        w = _c(pi_words, np.uint64)
        p = _c(p_pi, np.float32)
        ones = np.zeros(self.n_nets, dtype=np.uint64)
        tog = np.zeros(self.n_nets, dtype=np.uint64)
        _load().orc_sim(*self._args(), int(n_words), _ptr(w), _ptr(p), int(seed), _ptr(ones),
                        _ptr(tog))
        return ones, tog

    def sim_range(self, t_begin, t_end, p_pi, seed=0):
        """(ones, toggles) over the cycles [t_begin, t_end) with generated
        stimulus; disjoint ranges add up."""
        p = _c(p_pi, np.float32)
        ones = np.zeros(self.n_nets, dtype=np.uint64)
        tog = np.zeros(self.n_nets, dtype=np.uint64)
        _load().orc_sim_range(*self._args(), int(t_begin), int(t_end), _ptr(p), int(seed),
                              _ptr(ones), _ptr(tog))
        return ones, tog

    def power(self, P, cap, size=None, *, kappa=0.5, hybrid=False, ones=None, toggles=None,
              n_words=0, beta_min=0.1, beta_max=10.0, beta=None):
        """Finalize: dict of tr_model, sp_acc, tr_acc, beta, tr_hyb, ceff and
        the total power."""
        n = self.n_nets
        out = {k: np.zeros(n, dtype=np.float64)
               for k in ("tr_model", "sp_acc", "tr_acc", "beta", "tr_hyb", "ceff")}
        P = _c(P, np.float64)
        cap = _c(cap, np.float32)
        size = _c(size, np.float32)
        ones = _c(ones, np.uint64)
        toggles = _c(toggles, np.uint64)
        beta = _c(beta, np.float64)
        set_cells(self.cells)
        out["power"] = _load().orc_power(
            self.n_pi, self.n_gates, _ptr(P), _ptr(ones), _ptr(toggles), int(n_words), _ptr(cap),
            _ptr(size), float(kappa), int(bool(hybrid)), float(beta_min), float(beta_max),
            _ptr(beta), _ptr(out["tr_model"]), _ptr(out["sp_acc"]), _ptr(out["tr_acc"]),
            _ptr(out["beta"]), _ptr(out["tr_hyb"]), _ptr(out["ceff"]))
        return out

    def adjoint(self, P, beta, cap, size=None, *, kappa=0.5, beta_ste=False, fixed=None):
        """dict of lambda [n_nets], dpi [n_pi], dcap [n_nets], dsize [n_gates].
        fixed [n_pi] (nonzero = a fixed infrastructure startpoint, such as a
        clock or a reset): excluded from the gradients, its lambda and dpi
        are 0 (startpoints feed nothing upstream, so nothing else changes)."""
        n = self.n_nets
        lam = np.zeros(n, dtype=np.float64)
        dcap = np.zeros(n, dtype=np.float64)
        dsize = np.zeros(max(self.n_gates, 1), dtype=np.float64)
        _load().orc_adjoint(*self._args(), _ptr(_c(P, np.float64)), _ptr(_c(beta, np.float64)),
                            _ptr(_c(cap, np.float32)), _ptr(_c(size, np.float32)), float(kappa),
                            int(bool(beta_ste)), _ptr(lam), _ptr(dcap), _ptr(dsize))
        if fixed is not None:
            lam[: self.n_pi][np.asarray(fixed) != 0] = 0.0
        return dict(lam=lam, dpi=lam[: self.n_pi].copy(), dcap=dcap, dsize=dsize[: self.n_gates])

    def power_complex_step(self, p_pi, beta, ceff, pi, *, kappa=0.5, h=1e-30):
        return _load().orc_power_complex_step(
            *self._args(), _ptr(_c(p_pi, np.float64)), _ptr(_c(beta, np.float64)),
            _ptr(_c(ceff, np.float64)), float(kappa), int(pi), float(h))

    def sp_override(self, p_pi, net: int, delta: float) -> np.ndarray:
        """SP with P[net] shifted by delta (propagated downstream)."""
        P = np.zeros(self.n_nets, dtype=np.float64)
        _load().orc_sp_override(*self._args(), _ptr(_c(p_pi, np.float64)), int(net),
                                float(delta), _ptr(P))
        return P

    def sizing_score(self, P, lam, eps=2.0 ** -20) -> np.ndarray:
        """Eq. 8 score of every gate (caller gate order)."""
        S = np.zeros(max(self.n_gates, 1), dtype=np.float64)
        set_cells(self.cells)
        _load().orc_sizing_score(self.n_pi, self.n_gates, _ptr(_c(P, np.float64)),
                                 _ptr(_c(lam, np.float64)), float(eps), _ptr(S))
        return S[: self.n_gates]

    def virus_power(self, v0, cap) -> float:
        """P_virus (Eq. 3 at net level) of the vector pair (v0, 1 - v0)."""
        v = _c(v0, np.uint8)
        return float(_load().orc_virus_power(*self._args(), _ptr(_c(cap, np.float32)), _ptr(v)))

    def power_virus(self, p0, cap, *, steps=100, eta=0.1, beta=None):
        """Alg. 4: gradient ascent of the Eq. 9 proxy from p0, then the
        thresholded pair and its P_virus.  Returns (p_final, v0, p_virus)."""
        p = np.array(p0, dtype=np.float64, copy=True)
        v0 = np.zeros(self.n_pi, dtype=np.uint8)
        pv = _load().orc_power_virus(*self._args(), _ptr(_c(cap, np.float32)),
                                     _ptr(_c(beta, np.float64)), int(steps), float(eta), _ptr(p),
                                     _ptr(v0))
        return p, v0, float(pv)

    # -- whole-query compositions -----------------------------------------
    def forward(self, p_pi, cap, size=None, *, hybrid=False, n_words=0, seed=0, pi_words=None,
                kappa=0.5, beta_min=0.1, beta_max=10.0):
        """One query column: SP, optional simulation, finalize."""
        P = self.sp(np.asarray(p_pi, dtype=np.float32).astype(np.float64))
        ones = tog = None
        if hybrid:
            ones, tog = self.sim(n_words, pi_words=pi_words, p_pi=p_pi, seed=seed)
        out = self.power(P, cap, size, kappa=kappa, hybrid=hybrid, ones=ones, toggles=tog,
                         n_words=n_words, beta_min=beta_min, beta_max=beta_max)
        out["sp"] = P
        if hybrid:
            out["ones"], out["toggles"] = ones, tog
        return out

    def frozen_power(self, p_pi64, beta, cap, size=None, *, kappa=0.5):
        """Power with beta held fixed, for finite differences."""
        P = self.sp(p_pi64)
        return self.power(P, cap, size, kappa=kappa, beta=beta)["power"]


def op_arity(op: int) -> int:
    return int(_load().orc_op_arity(int(op)))


def gate_sp(op: int, x) -> float:
    x = np.ascontiguousarray(np.resize(np.asarray(x, dtype=np.float64), 6))
    return float(_load().orc_gate_sp(int(op), _ptr(x)))


def gate_partials(op: int, x) -> np.ndarray:
    x = np.ascontiguousarray(np.resize(np.asarray(x, dtype=np.float64), 6))
    d = np.zeros(6, dtype=np.float64)
    _load().orc_gate_partials(int(op), _ptr(x), _ptr(d))
    return d[: op_arity(op)]


def gate_bits(op: int, w) -> int:
    w = np.ascontiguousarray(np.resize(np.asarray(w, dtype=np.uint64), 6))
    return int(_load().orc_gate_bits(int(op), _ptr(w)))


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def threshold(p: float) -> int:
    return int(_load().orc_threshold(float(np.float32(p))))


def markov_probs(p: float, tau: float):
    """(rise, stay): the chain's P(0 -> 1) and P(1 -> 1) for stationary
    probability p and transition rate tau (float32 inputs)."""
    a, st = _d(), _d()
    _load().orc_markov_probs(float(np.float32(p)), float(np.float32(tau)), ctypes.byref(a),
                             ctypes.byref(st))
    return a.value, st.value


def threshold_d(x: float) -> int:
    return int(_load().orc_threshold_d(float(x)))


def stimulus_model(p_pi, seed: int, n_words: int, tau=None, stream=None) -> np.ndarray:
    """uint64 [n_pi][n_words]: per-startpoint Markov chains with transition
    rates tau (None: independent cycles) on shared streams (None: own)."""
    p = _c(p_pi, np.float32)
    n = p.shape[0]
    w = np.zeros((n, n_words), dtype=np.uint64)
    _load().orc_stimulus_model(int(n), _ptr(p), _ptr(_c(tau, np.float32)),
                               _ptr(_c(stream, np.int32)), int(seed), int(n_words), _ptr(w))
    return w


def stimulus(p_pi, seed: int, t0: int, n_words: int) -> np.ndarray:
    """uint64 [n_pi][n_words] stimulus words t0 .. t0+n_words-1."""
    p = _c(p_pi, np.float32)
    w = np.zeros((p.shape[0], n_words), dtype=np.uint64)
    _load().orc_stimulus(int(p.shape[0]), _ptr(p), int(seed), int(t0), int(n_words), _ptr(w))
    return w
