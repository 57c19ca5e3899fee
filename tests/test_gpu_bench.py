"""The benchmark's one JSON line keeps its contract: a short default run
(32^4, a fixed launch shape, a few steps) in a child process prints one line
with the metric, the whole-job value, the roofline of the heat-bath kernel,
the 64^4 control, the binary64 form and the serial oracle baseline."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_contract():
    cmd = [sys.executable, "-u", os.path.join(ROOT, "bench.py"), "--steps", "8", "--warmup", "2",
           "--launch", "128,0,1,1", "--cpu-sweeps", "1", "--cpu-threads", "2", "--no-copy-probe"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1, r.stdout[-2000:]
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 8 and d["warmup"] == 2 and d["dtype"] == "f32"
    assert d["value"] > 0 and d["higher_is_better"] is True and d["vs_baseline"] is None
    assert "workload" in d["config"] and d["config"]["launch"]["block"] == 128
    rf = d["roofline"]
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["achieved"] > 0 and abs(rf["frac"] - rf["achieved"] / rf["peak"]) < 1e-12
    assert rf["traffic"] is None or rf["traffic"] > rf["bytes_per_launch"]
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0 and cb["sample"]
    assert rf["avg_launch_source"] and 0 < rf["step_frac"] < 1 and rf["links_in_infinity_cache"] is True
    ko = rf["kernel_only"]
    assert 0 < ko["avg_launch_us"] and abs(ko["frac"] - rf["bytes_per_launch"] / ko["avg_launch_us"] / 8e6) < 1e-9
    assert len(d["timing"]["rep_ms_per_step"]) == 11
    assert d["overrelax"]["frac"] > 0 and d["fp64_plain"]["default"]["value"] > 0
    c = d["control64"]
    assert c["avg_launch_us"] > 0 and 0 < c["frac"] < 1 and c["bytes_per_launch"] == 64 ** 4 // 2 * 128
