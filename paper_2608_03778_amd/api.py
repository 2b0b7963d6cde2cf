"""Thin Python binding over the C ABI (argument marshalling only).

Arrays may be numpy arrays (host memory, ``on_device = 0``) or torch CUDA
tensors (device memory, ``on_device = 1``; the context should then run on
torch's current stream).  Every computation happens in libdiffpower.
"""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional

import numpy as np

from . import _lib as L
from ._lib import check


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _in_ptr(x, dtype):
    """(pointer, on_device, keepalive) for an input array."""
    if x is None:
        return None, 0, None
    if _is_torch(x):
        import torch
        tdt = {np.float32: torch.float32, np.uint64: torch.int64, np.int32: torch.int32}[dtype]
        if x.dtype != tdt and not (dtype == np.uint64 and x.dtype == torch.uint64):
            x = x.to(tdt)
        x = x.contiguous()
        return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), 0, a


HIP_STREAM_LEGACY = 1  # hipStreamLegacy: the device's null stream


class Context:
    """A GPU and the stream library calls enqueue on."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self.lib = L.load()
        h = ctypes.c_void_p()
        check(self.lib.dp_ctx_create(int(device), ctypes.c_void_p(stream) if stream else None,
                                     ctypes.byref(h)))
        self.handle = h
        self.device = device

    @classmethod
    def for_torch(cls, device: int = 0):
        """Enqueue on torch's current stream, so library calls are ordered
        with torch's work on the tensors they read and write."""
        import torch
        torch.cuda.set_device(device)
        h = torch.cuda.current_stream(device).cuda_stream
        return cls(device, h if h else HIP_STREAM_LEGACY)

    def set_stream(self, stream: Optional[int]):
        check(self.lib.dp_ctx_set_stream(self.handle, ctypes.c_void_p(stream) if stream else None))

    def synchronize(self):
        check(self.lib.dp_ctx_synchronize(self.handle))

    def close(self):
        if self.handle:
            self.lib.dp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Design:
    """A compiled, device-resident netlist (immutable)."""

    def __init__(self, ctx: Context, netlist):
        self.ctx = ctx
        self.lib = ctx.lib
        op = np.ascontiguousarray(netlist.op, dtype=np.uint8)
        ptr = np.ascontiguousarray(netlist.fanin_ptr, dtype=np.int32)
        fan = np.ascontiguousarray(netlist.fanin, dtype=np.int32)
        nl = L.Netlist(int(netlist.n_pi), int(op.shape[0]), op.ctypes.data, ptr.ctypes.data,
                       fan.ctypes.data)
        h = ctypes.c_void_p()
        cells = [c.encode() for c in getattr(netlist, "cells", ()) or ()]
        pins = list(getattr(netlist, "pins", ()) or ())
        self.n_cells = len(cells)
        if cells and pins:
            arr = (ctypes.c_char_p * len(cells))(*cells)
            parr = (ctypes.c_char_p * len(cells))(*[(x.encode() if x else None) for x in pins])
            check(self.lib.dp_compile_library(ctx.handle, ctypes.byref(nl), len(cells),
                                              ctypes.cast(arr, ctypes.c_void_p),
                                              ctypes.cast(parr, ctypes.c_void_p),
                                              ctypes.byref(h)))
        elif cells:
            arr = (ctypes.c_char_p * len(cells))(*cells)
            check(self.lib.dp_compile_cells(ctx.handle, ctypes.byref(nl), len(cells),
                                            ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(h)))
        else:
            check(self.lib.dp_compile(ctx.handle, ctypes.byref(nl), ctypes.byref(h)))
        self.handle = h
        info = L.DesignInfo()
        check(self.lib.dp_design_info(h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in L.DesignInfo._fields_ if k != "reserved"}
        self.n_pi, self.n_gates, self.n_nets = info.n_pi, info.n_gates, info.n_nets
        self.depth = info.depth

    def forward_static(self, p, cap, *, out_power, mode=L.DP_MODELED, beta=None, out_sp=None,
                       out_tr=None, **kw):
        """One modeled (or frozen-beta) forward through dp_forward_static,
        which allocates nothing: every argument is a torch CUDA tensor the
        caller owns (p [n_pi], cap and beta [n_nets], out_power [1], out_sp
        and out_tr [n_nets] or None).  Enqueued on the context's stream."""
        prm = params(mode, **kw)

        def dev(x):
            if x is None:
                return None
            if not (_is_torch(x) and x.is_cuda and x.is_contiguous()):
                raise ValueError("forward_static takes contiguous torch CUDA tensors")
            return ctypes.c_void_p(x.data_ptr())
        check(self.lib.dp_forward_static(self.handle, ctypes.byref(prm), dev(p), dev(cap),
                                         dev(beta), dev(out_power), dev(out_sp), dev(out_tr)))

    def cell_logic(self):
        """(logic id of every library cell, or -1 - op for one that runs as a
        fixed cell; number of distinct ids)."""
        logic = np.zeros(max(self.n_cells, 1), dtype=np.int32)
        n = ctypes.c_int32()
        check(self.lib.dp_design_cell_logic(self.handle, logic.ctypes.data_as(ctypes.c_void_p),
                                            ctypes.byref(n)))
        return logic[: self.n_cells], n.value

    def levels(self) -> np.ndarray:
        lv = np.zeros(self.n_nets, dtype=np.int32)
        check(self.lib.dp_design_levels(self.handle, lv.ctypes.data_as(ctypes.c_void_p)))
        return lv

    def close(self):
        if self.handle:
            self.lib.dp_design_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def params(mode=L.DP_MODELED, *, n_sim=4096, seed=1, vdd=1.0, fclk=1.0, energy_factor=0.5,
           beta_min=0.1, beta_max=10.0, beta_grad=L.DP_BETA_LOCAL) -> L.Params:
    p = L.Params()
    L.load().dp_params_default(ctypes.byref(p))
    p.mode, p.n_sim, p.seed = int(mode), int(n_sim), int(seed)
    p.vdd, p.fclk, p.energy_factor = float(vdd), float(fclk), float(energy_factor)
    p.beta_min, p.beta_max, p.beta_grad = float(beta_min), float(beta_max), int(beta_grad)
    return p


_FWD_FIELDS = ("sp", "tr", "sp_acc", "tr_acc", "beta", "tr_hyb", "ones", "toggles", "power")


class Eval:
    """Workspaces for B query columns and S size vectors of one design."""

    def __init__(self, design: Design, n_cols: int = 1, n_size: int = 0, **kw):
        self.design = design
        self.lib = design.lib
        self.B, self.S = int(n_cols), int(n_size)
        self.prm = params(**kw)
        h = ctypes.c_void_p()
        check(self.lib.dp_eval_create(design.handle, self.B, self.S, ctypes.byref(self.prm),
                                      ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    @property
    def n_words(self) -> int:
        return int(self.prm.n_sim) // 64

    def set_params(self, **kw):
        self.prm = params(**kw)
        check(self.lib.dp_eval_set_params(self.handle, ctypes.byref(self.prm)))

    def _set(self, fn, x, dtype, key):
        ptr, dev, keep = _in_ptr(x, dtype)
        self._keep[key] = keep  # device copies are enqueued, keep the source alive
        check(fn(self.handle, ptr, dev))

    def set_pi_prob(self, p):
        self._set(self.lib.dp_set_pi_prob, p, np.float32, "p")

    def set_caps(self, cap):
        self._set(self.lib.dp_set_caps, cap, np.float32, "cap")

    def set_cell_sizes(self, size):
        self._set(self.lib.dp_set_cell_sizes, size, np.float32, "size")

    def set_beta(self, beta):
        self._set(self.lib.dp_set_beta, beta, np.float32, "beta")

    def set_stimulus(self, words):
        if words is None:
            check(self.lib.dp_set_stimulus(self.handle, None, 0))
            return
        self._set(self.lib.dp_set_stimulus, words, np.uint64, "stim")

    def set_pi_rates(self, tau):
        """Target transition rate of every PI, [B][n_pi] (None: independent
        cycles)."""
        if tau is None:
            check(self.lib.dp_set_pi_rates(self.handle, None, 0))
            return
        self._set(self.lib.dp_set_pi_rates, tau, np.float32, "tau")

    def set_pi_streams(self, stream):
        """Philox stream of every PI, [n_pi] (None: its own)."""
        if stream is None:
            check(self.lib.dp_set_pi_streams(self.handle, None))
            return
        a = np.ascontiguousarray(stream, dtype=np.int32)
        check(self.lib.dp_set_pi_streams(self.handle, a.ctypes.data))

    def set_pi_fixed(self, fixed):
        """PIs excluded from the gradients, [n_pi] booleans (None: none)."""
        if fixed is None:
            check(self.lib.dp_set_pi_fixed(self.handle, None))
            return
        a = np.ascontiguousarray(fixed, dtype=np.uint8)
        check(self.lib.dp_set_pi_fixed(self.handle, a.ctypes.data))

    def set_schedule(self, schedule=L.DP_SCHED_AUTO, words_per_chunk=0, pairs_per_lane=0):
        check(self.lib.dp_eval_set_schedule(self.handle, int(schedule), int(words_per_chunk),
                                            int(pairs_per_lane)))

    def _out(self, name, device):
        nn = self.design.n_nets
        shape = {"power": (self.B, max(self.S, 1))}.get(name, (self.B, nn))
        dt = np.uint32 if name in ("ones", "toggles") else np.float32
        if device:
            import torch
            tdt = torch.int32 if dt == np.uint32 else torch.float32
            return torch.empty(shape, dtype=tdt, device=f"cuda:{self.design.ctx.device}")
        return np.empty(shape, dtype=dt)

    def forward(self, outputs: Iterable[str] = ("power",), device: bool = False) -> dict:
        """Run the forward sweep; returns the requested outputs (numpy on the
        host, or torch CUDA tensors with device=True; counts come back as
        int32 tensors holding uint32 bit patterns)."""
        res = {}
        out = L.FwdOut()
        out.on_device = int(bool(device))
        for name in outputs:
            if name not in _FWD_FIELDS:
                raise ValueError(f"unknown forward output {name!r}")
            arr = self._out(name, device)
            res[name] = arr
            setattr(out, name, arr.data_ptr() if device else arr.ctypes.data)
        check(self.lib.dp_forward(self.handle, ctypes.byref(out)))
        return res

    def backward(self, grad_power=None, want=("dpi",), device: bool = False) -> dict:
        """Reverse sweep weighted by grad_power [B][S'] (None = ones)."""
        d = self.design
        shapes = {"dpi": (self.B, d.n_pi), "dcap": (d.n_nets,), "dsize": (self.S, d.n_gates)}
        res = {}
        ptrs = {}
        for name in want:
            if device:
                import torch
                arr = torch.empty(shapes[name], dtype=torch.float32, device=f"cuda:{d.ctx.device}")
                ptrs[name] = ctypes.c_void_p(arr.data_ptr())
            else:
                arr = np.empty(shapes[name], dtype=np.float32)
                ptrs[name] = arr.ctypes.data_as(ctypes.c_void_p)
            res[name] = arr
        gptr, gdev, keep = _in_ptr(grad_power, np.float32)
        if grad_power is not None and gdev != int(bool(device)):
            raise ValueError("grad_power must live where the outputs do")
        self._keep["grad"] = keep
        check(self.lib.dp_backward(self.handle, gptr, ptrs.get("dpi"), ptrs.get("dcap"),
                                   ptrs.get("dsize"), int(bool(device))))
        return res

    def backward_columns(self, device: bool = False):
        d = self.design
        shape = (self.B, max(self.S, 1), d.n_pi)
        if device:
            import torch
            arr = torch.empty(shape, dtype=torch.float32, device=f"cuda:{d.ctx.device}")
            ptr = ctypes.c_void_p(arr.data_ptr())
        else:
            arr = np.empty(shape, dtype=np.float32)
            ptr = arr.ctypes.data_as(ctypes.c_void_p)
        check(self.lib.dp_backward_columns(self.handle, ptr, int(bool(device))))
        return arr

    def forward_backward_columns(self, device: bool = False):
        """The forward pass and backward_columns in one call (one graph
        launch under DP_SCHED_GRAPH): power [B][S'] and dP/dp [B][S'][n_pi]."""
        d = self.design
        Sp = max(self.S, 1)
        if device:
            import torch
            dev = f"cuda:{d.ctx.device}"
            power = torch.empty((self.B, Sp), dtype=torch.float32, device=dev)
            dpi = torch.empty((self.B, Sp, d.n_pi), dtype=torch.float32, device=dev)
            pp, pd = ctypes.c_void_p(power.data_ptr()), ctypes.c_void_p(dpi.data_ptr())
        else:
            power = np.empty((self.B, Sp), dtype=np.float32)
            dpi = np.empty((self.B, Sp, d.n_pi), dtype=np.float32)
            pp, pd = power.ctypes.data_as(ctypes.c_void_p), dpi.ctypes.data_as(ctypes.c_void_p)
        check(self.lib.dp_forward_backward_columns(self.handle, pp, pd, int(bool(device))))
        return power, dpi

    def power_gradients(self):
        """Every net's dPower/dP [B][n_nets] and the Eq. 8 sizing score of
        every gate [B][n_gates] (caller numbering), after a forward."""
        d = self.design
        lam = np.zeros((self.B, d.n_nets), dtype=np.float32)
        score = np.zeros((self.B, d.n_gates), dtype=np.float32)
        check(self.lib.dp_power_gradients(self.handle, lam.ctypes.data, score.ctypes.data, 0))
        return lam, score

    def power_virus(self, steps: int = 100, eta: float = 0.1):
        """Alg. 4 from the current PI probabilities: returns (v0 [B][n_pi]
        uint8, p_final [B][n_pi] float32, p_virus [B] float64)."""
        d = self.design
        v0 = np.zeros((self.B, d.n_pi), dtype=np.uint8)
        pf = np.zeros((self.B, d.n_pi), dtype=np.float32)
        pv = np.zeros(self.B, dtype=np.float64)
        check(self.lib.dp_power_virus(self.handle, int(steps), float(eta), v0.ctypes.data,
                                      pf.ctypes.data, pv.ctypes.data, 0))
        return v0, pf, pv

    def autotune(self, reps: int = 3, with_backward: bool = False) -> float:
        """Pick the fastest schedule for the forward (and, with_backward,
        the reverse) sweep; returns its ms."""
        ms = ctypes.c_double()
        check(self.lib.dp_eval_autotune(self.handle, int(reps), int(bool(with_backward)),
                                        ctypes.byref(ms)))
        return ms.value

    def set_sim_streams(self, n: int):
        check(self.lib.dp_eval_set_sim_streams(self.handle, int(n)))

    def set_sim_columns(self, n: int):
        """Query columns per simulation launch (0 = as many as fit)."""
        check(self.lib.dp_eval_set_sim_columns(self.handle, int(n)))

    def get_schedule(self) -> dict:
        sc, ch, pp, ns = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        check(self.lib.dp_eval_get_schedule(self.handle, ctypes.byref(sc), ctypes.byref(ch),
                                            ctypes.byref(pp), ctypes.byref(ns)))
        return dict(schedule=sc.value, words_per_chunk=ch.value, pairs_per_lane=pp.value,
                    sim_streams=ns.value)

    def synchronize(self):
        """Wait for the eval's stream; raises if a persistent sweep's grid
        barrier gave up since the last host synchronization."""
        check(self.lib.dp_eval_synchronize(self.handle))

    def set_barrier_timeout(self, microseconds: float):
        check(self.lib.dp_eval_set_barrier_timeout(self.handle, float(microseconds)))

    def profile(self, enable: bool = True):
        check(self.lib.dp_eval_profile(self.handle, int(bool(enable))))

    def get_profile(self) -> dict:
        p = L.Profile()
        check(self.lib.dp_eval_get_profile(self.handle, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in L.Profile._fields_}

    def close(self):
        if self.handle:
            self.lib.dp_eval_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Group:
    """Several evals (any designs of one context) run as one unit: one
    branch stream per eval, captured once into a HIP graph when the unit is
    small enough, one launch per run."""

    def __init__(self, ctx: Context, evals):
        self.lib = L.load()
        self.ctx = ctx
        self.evals = list(evals)
        arr = (ctypes.c_void_p * len(self.evals))(*[e.handle.value for e in self.evals])
        h = ctypes.c_void_p()
        check(self.lib.dp_group_create(ctx.handle, arr, len(self.evals), ctypes.byref(h)))
        self.handle = h

    def run(self, outputs: Iterable[str] = ("power",), backward: bool = False,
            device: bool = False):
        """Forward (and reverse) sweeps of every eval; returns one dict per
        eval with the requested outputs (and "dpi" when backward)."""
        n = len(self.evals)
        outs = (L.FwdOut * n)()
        res = [dict() for _ in range(n)]
        for i, ev in enumerate(self.evals):
            outs[i].on_device = int(bool(device))
            for name in outputs:
                if name not in _FWD_FIELDS:
                    raise ValueError(f"unknown forward output {name!r}")
                arr = ev._out(name, device)
                res[i][name] = arr
                setattr(outs[i], name, arr.data_ptr() if device else arr.ctypes.data)
        dpi = None
        if backward:
            dpi = (ctypes.c_void_p * n)()
            for i, ev in enumerate(self.evals):
                shape = (ev.B, ev.design.n_pi)
                if device:
                    import torch
                    arr = torch.empty(shape, dtype=torch.float32,
                                      device=f"cuda:{self.ctx.device}")
                    dpi[i] = arr.data_ptr()
                else:
                    arr = np.empty(shape, dtype=np.float32)
                    dpi[i] = arr.ctypes.data
                res[i]["dpi"] = arr
        check(self.lib.dp_group_run(self.handle, int(bool(backward)), outs, dpi,
                                    int(bool(device))))
        return res

    def configure(self, use_graph: bool = True, max_branches: int = 0):
        check(self.lib.dp_group_configure(self.handle, int(bool(use_graph)), int(max_branches)))

    def close(self):
        if self.handle:
            self.lib.dp_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query server over device-resident designs."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_batch: int = 64,
                 max_inflight: int = 8):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        check(self.lib.dp_server_create(ctx.handle, int(hbm_budget_bytes), ctypes.byref(h)))
        self.handle = h
        check(self.lib.dp_server_configure(h, int(max_batch), int(max_inflight)))
        self._live = {}
        self._designs = {}

    def configure(self, max_batch: int, max_inflight: int):
        check(self.lib.dp_server_configure(self.handle, int(max_batch), int(max_inflight)))

    def add_design(self, design: Design, cap, **kw) -> int:
        prm = params(**kw)
        c = np.ascontiguousarray(cap, dtype=np.float32)
        i = ctypes.c_int32()
        check(self.lib.dp_server_add_design(self.handle, design.handle,
                                            c.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm),
                                            ctypes.byref(i)))
        self._designs[i.value] = design
        return i.value

    def submit(self, design_id: int, p, cap_scale=None, backward: bool = False) -> int:
        """Enqueue one query; returns its ticket.  The result arrays are kept
        here until wait() hands them back."""
        d = self._designs[design_id]
        pa = np.ascontiguousarray(p, dtype=np.float32)
        sa = None if cap_scale is None else np.ascontiguousarray(cap_scale, dtype=np.float32)
        power = np.zeros(1, dtype=np.float32)
        dpi = np.zeros(d.n_pi, dtype=np.float32) if backward else None
        q = L.Query(design_id, L.DP_Q_FWD_BWD if backward else L.DP_Q_FWD, pa.ctypes.data,
                    sa.ctypes.data if sa is not None else None, power.ctypes.data,
                    dpi.ctypes.data if dpi is not None else None)
        t = ctypes.c_uint64()
        check(self.lib.dp_submit(self.handle, ctypes.byref(q), ctypes.byref(t)))
        self._live[t.value] = (pa, sa, power, dpi)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32()
        check(self.lib.dp_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(done)))
        return bool(done.value)

    def wait(self, ticket: int):
        """Block until done; returns (power, dP/dp or None, latency seconds)."""
        lat = ctypes.c_double()
        try:
            check(self.lib.dp_wait(self.handle, ctypes.c_uint64(ticket), ctypes.byref(lat)))
        finally:
            live = self._live.pop(ticket, None)
        _, _, power, dpi = live
        return float(power[0]), dpi, lat.value

    def stats(self) -> dict:
        s = L.ServerStats()
        check(self.lib.dp_server_get_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in L.ServerStats._fields_ if k != "reserved"}

    def close(self):
        if self.handle:
            self.lib.dp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
