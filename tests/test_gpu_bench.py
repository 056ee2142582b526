"""The benchmark's JSON line end to end on a small workload (12-qubit
molecular (3,3) sector): one line with the contract's fields, the pipelined
steps ending on the same energy bits as the serial ones, the complex64
product within its bound of complex128 on the same input, and the roofline
and CPU-baseline objects in their documented shapes."""

import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "molecular-12q-sector", "--steps", "3",
           "--warmup", "1"]
    print("[bench] " + " ".join(cmd[1:]), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert res.returncode == 0, res.stderr[-2000:]
    lines = [ln for ln in res.stdout.splitlines() if ln.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1 and d["higher_is_better"] is True
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["ms_per_step_serial"] > 0
    assert d["config"]["workload"] == "molecular-12q-sector" and d["config"]["dim"] == 400
    assert d["pipelined_equals_serial"] is True
    assert d["rel_err_c64_vs_c128_same_input"] < 1e-6
    shares = d["apply_ms_c64_row_shares_of_8"]
    assert len(shares) == 8 and min(shares) > 0
    r = d["roofline"]
    assert r["bound"] in ("alu", "hbm") and r["peak"] > 0 and r["apply_ms"] > 0
    assert 100.0 < r["measured_copy_GBs"] < 16000.0  # a plain copy, against the 8 TB/s HBM peak
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]
