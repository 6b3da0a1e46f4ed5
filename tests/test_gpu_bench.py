"""The benchmark's output contract on the GPU: one JSON line with the
required keys, a positive throughput consistent with its step time, and the
roofline and CPU-baseline objects in their documented shapes."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_contract():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] bench contract", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "3",
                        "--warmup", "1", "--large-target-spp", "4", "--no-extras"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["data"] == "synthetic"
    assert d["value"] > 0 and d["ms_per_step"] > 0
    npix = d["config"]["pixels"]
    assert abs(d["value"] - 4 * npix / (d["ms_per_step"] / 1e3)) <= 1e-6 * d["value"]
    assert "workload" in d["config"]
    assert d["config"]["triangles"] == 999698 and d["config"]["params"] == 1310720
    for rf in (d["roofline"], d["roofline_other_kernel"]):
        assert rf["bound"] in ("hbm", "mfma", "alu") and rf["peak"] > 0
        assert rf["kernel"] in ("k_forward", "k_adjoint") and rf["kernel_ms"] > 0
        assert rf["achieved"] is None or abs(rf["frac"] - rf["achieved"] / rf["peak"]) <= 1e-9
    assert d["roofline"]["kernel_ms"] >= d["roofline_other_kernel"]["kernel_ms"]
    assert d["roofline"]["traffic"] is None or d["roofline"]["traffic"] > 0
    adj = [rf for rf in (d["roofline"], d["roofline_other_kernel"])
           if rf["kernel"] == "k_adjoint"][0]
    assert adj["bound"] == "hbm" and adj["achieved"] > 0 and adj["atomics_per_s"] > 0
    ub = d["microbenchmarks"]
    assert ub["copy_GBs"] > 1000
    assert ub["atomic_ops_per_s_lines"] > 0 and ub["atomic_ops_per_s_same_address"] > 0
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["value"] > 0 and cb["cores"] >= 1 and cb["sample"]
