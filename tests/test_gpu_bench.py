"""bench.py end to end on the GPU: one short run, the JSON line's contract."""
import json
import os
import subprocess
import sys

import pytest

from parity_util import announce

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    announce("bench.py short run")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20",
                        "--warmup", "3", "--cpu-seconds", "1", "--surrogate-steps", "0",
                        "--variant-steps", "10"],
                       capture_output=True, text=True, timeout=280, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 20 and d["warmup"] == 3
    assert d["value"] > 0 and d["unit"] == "pair interactions/s" and d["dtype"] == "f32"
    assert d["config"]["particles"] > 1_000_000 and "workload" in d["config"]
    roof = d["roofline"]
    assert roof["bound"] == "alu" and 0 < roof["frac"] < 1 and roof["peak"] == 157.3
    assert abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-12
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1
    assert set(d["variants"]) == {"cubic", "symplectic", "cubic_symplectic"}
    assert all(v["status"] == 0 for v in d["variants"].values())
