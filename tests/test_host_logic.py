"""The library's host code without a GPU: its C++ sources built with g++
against a CPU stand-in for the HIP runtime (tests/hoststub), whose launchers
check every launch's extents and compute nothing.  Covered here: compile and
levelization (levels against the oracle's) for fixed cells, library cells,
trees and flop-cut sequential netlists; every compile and parse error; the
setters' validation and state errors; every schedule's host path (graph
capture bookkeeping, chunks, concurrent simulation streams, the persistent
schedule and its refusal for library cells); the stimulus model's setters;
design groups' merged tables and branches; the serving scheduler's batching,
errors and budget.  Each scenario runs in a process of its own, which loads
only the stand-in runtime."""
from __future__ import annotations

import json
import os
import subprocess
import sys

import pytest

from tests.hoststub import build as stub_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def stub_lib(tmp_path_factory):
    if not stub_build.available():
        pytest.skip("g++ or the HIP headers are missing")
    return stub_build.build(str(tmp_path_factory.mktemp("hoststub")))


def _run(lib, scenario):
    p = subprocess.run([sys.executable, "-m", "tests.hoststub.scenarios", lib, scenario],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-4000:]
    return json.loads(p.stdout.strip().splitlines()[-1])


def test_compile_and_levelization(stub_lib):
    r = _run(stub_lib, "compile")
    for name in ("fixed", "library", "flop_cut", "tree"):
        assert r[f"{name}_levels_match"] and r[f"{name}_depth_match"], name
    assert r["expressions_levels_match"]
    assert r["cycle"] == "DP_E_CYCLE"
    for k in ("bad_arity", "bad_op", "bad_net", "cell_arity", "cell_missing"):
        assert r[k] == "DP_E_INVALID", k
    want = {"A&": "operand", "(A|B": "')'", "A $ B": "character", "A B": "after",
            "a&b&c&d&e&f&g": "6 inputs", "&".join(["A"] * 20): "32 operations",
            "A|(B|(C|(D|(E|(F|(A|(B|C)))))))": "8 stack", "1": "no inputs"}
    for text, what in want.items():
        st, msg = r["parse"][text]
        assert st == "DP_E_INVALID" and what in msg, (text, msg)


def test_eval_flows_and_validation(stub_lib):
    r = _run(stub_lib, "flows")
    assert r["fixed_runs"] == 46 and r["library_runs"] == 40
    for name in ("fixed", "library"):
        assert r[f"{name}_backward_first"] == "DP_E_STATE"
        assert r[f"{name}_forward_no_inputs"] == "DP_E_STATE"
        for k in ("p_range", "cap_range", "rates_range", "streams_range", "schedule_bad"):
            assert r[f"{name}_{k}"] == "DP_E_INVALID", (name, k)
        assert r[f"{name}_virus_hybrid"] == "DP_E_UNSUPPORTED"
    assert r["fixed_persistent"] == "OK"
    assert r["library_persistent"] == "DP_E_UNSUPPORTED"


def test_groups_and_serving(stub_lib):
    r = _run(stub_lib, "group_serving")
    assert r["group_results"] == 3
    assert r["served"] == 60 and r["completed"] >= 60 and r["batched"]
    assert r["nan_size"] == "DP_E_INVALID" and r["bad_p"] == "DP_E_INVALID"
    assert r["unknown_ticket"] == "DP_E_NOTFOUND" and r["budget"] == "DP_E_BUDGET"


def test_capture_order_under_the_capture_model(stub_lib):
    """Groups and serving, then the autotuner and graph-captured multi-column
    hybrid sweeps and a captured hybrid design group, in one process, under
    the stand-in's capture model (forks and joins, calls a capturing thread
    may not make, event reuse across captures, graph launches touching only
    live allocations).  Captures record one stream, so nothing forks."""
    r = _run(stub_lib, "capture_order")
    assert r["capture_order_done"] and r["served"] == 60
    assert r["captures"] > 20 and r["graph_launches"] > 100
    assert r["forks"] == 0
