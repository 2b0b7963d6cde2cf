"""The C-ABI library loads and exports every symbol include/diffpower.h
declares (no GPU needed, no compute calls)."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_2608_03778_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "diffpower.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dp_[a-z_]+)\s*\(", text)))


def _exported():
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines() if " T dp_" in ln})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libdiffpower.so is not built (run python -m paper_2608_03778_amd.build)")
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 30
    assert _exported() == declared
    for name in declared:
        assert hasattr(lib, name)


def test_binding_declares_every_symbol():
    assert sorted(L.SIGNATURES) == _declared()


def test_struct_sizes_match_header_layout():
    # sizes the C compiler gives the structs (natural alignment, x86-64)
    assert ctypes.sizeof(L.Params) == 5 * 8 + 2 * 4 + 8 + 8
    assert ctypes.sizeof(L.Netlist) == 8 + 3 * 8
    assert ctypes.sizeof(L.FwdOut) == 9 * 8 + 8
    assert ctypes.sizeof(L.DesignInfo) == 4 * 4 + 8 + 4 + 4 + 8
    assert ctypes.sizeof(L.ServerStats) == 3 * 8 + 8 + 8 + 4 + 4 + 3 * 8


def test_defaults_and_version(lib):
    p = L.Params()
    lib.dp_params_default(ctypes.byref(p))
    assert (p.vdd, p.fclk, p.energy_factor) == (1.0, 1.0, 0.5)
    assert (p.beta_min, p.beta_max) == (0.1, 10.0)
    assert p.mode == L.DP_MODELED and p.beta_grad == L.DP_BETA_LOCAL
    assert p.n_sim == 4096 and p.seed == 1
    assert b"gfx950" in lib.dp_version()
    assert lib.dp_last_error() == b""


def test_null_arguments_are_rejected_without_a_gpu(lib):
    assert lib.dp_design_info(None, None) == L.DP_E_INVALID
    assert b"NULL" in lib.dp_last_error()
    assert lib.dp_forward(None, None) == L.DP_E_INVALID
    assert lib.dp_backward(None, None, None, None, None, 0) == L.DP_E_INVALID
    assert lib.dp_eval_set_schedule(None, 0, 0, 0) == L.DP_E_INVALID


def test_one_hip_runtime_per_process():
    """Loading the library after torch binds it to torch's HIP runtime: a
    fresh process that loads the binding holds a single libamdhip64."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2608_03778_amd import _lib\n"
            "_lib.load()\n"
            "maps = open('/proc/self/maps').read().split('\\n')\n"
            "paths = {l.split()[-1] for l in maps if 'libamdhip64' in l}\n"
            "print(len(paths))\n") % (os.path.dirname(HEADER).rsplit("/include", 1)[0],)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"
