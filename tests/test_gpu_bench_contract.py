"""bench.py at a small size: one JSON line with the benchmark contract's
fields, the roofline of the dominant kernel and the oracle baseline."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_contract_line():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench.py, 32 x 1 GeV e-", flush=True)
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "2", "--warmup", "1",
           "--workload", "cal_1GeV_e-_x32", "--mixed-workload", "cal_1GeV_e-_x32", "--capacity", str(1 << 20),
           "--mixed-capacity", str(1 << 20), "--extra-workload=", "--no-serve", "--graph-check", "1",
           "--cpu-events", "8", "--error-events", "8"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1 and d["value"] > 0
    assert d["unit"] == "primaries/s" and d["higher_is_better"] is True and d["dtype"] == "f64"
    assert d["config"]["workload"] == "cal_1GeV_e-_x32" and d["config"]["events"] == 32
    roof = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in roof, k
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["achieved"] > 0 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    assert roof["traffic"] is None  # counters are committed for the full-size workloads only
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["unit"] == "primaries/s"
    assert d["mixed"]["value"] > 0 and d["value_graph_replay"] > 0
