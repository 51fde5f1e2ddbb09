"""The benchmark's one-line JSON record on the GPU: every field of the
contract, the roofline object of the main kernel and the consistency of its
figures (a short run of the single-channel workload), and the default run on
the large channel with the ensemble / adjoint comparison."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_line_contract():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench.py --workload single --steps 300 --warmup 20 --no-cpu", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "single", "--steps", "300",
                        "--warmup", "20", "--no-cpu"], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 300 and d["warmup"] == 20
    assert d["unit"] == "MLUPS" and d["higher_is_better"] is True and d["data"] == "synthetic"
    assert d["dtype"] == "f32" and d["vs_baseline"] is None
    c = d["config"]
    assert "64x64x256" in c["workload"] and c["nodes"] == 64 * 64 * 256 and not c["unstable"]
    # value is node updates per second over the timed steps
    assert abs(d["value"] - c["nodes"] / (d["ms_per_step"] * 1e-3) / 1e6) <= 1e-3 * d["value"]
    ro = d["roofline"]
    assert ro["bound"] == "hbm" and ro["unit"] == "GB/s" and ro["peak"] == 8000.0
    assert ro["bytes_per_launch"] == c["nodes"] * 304
    assert abs(ro["achieved"] - ro["bytes_per_launch"] / (ro["kernel_ms"] * 1e-3) / 1e9) <= 1e-3 * ro["achieved"]
    assert abs(ro["frac"] - ro["achieved"] / ro["peak"]) <= 1e-3
    assert 0.0 < ro["frac"] < 1.0
    # the main kernel is part of a step, not more than a step
    assert ro["kernel_ms"] < d["ms_per_step"]
    assert ro["launches"] >= 300 // 10
    if ro["traffic"] is not None:
        assert ro["traffic"] >= ro["bytes_per_launch"] * 0.95
    print(json.dumps(ro), flush=True)


def test_default_bench_line_large_channel_and_forms():
    """The default run (large channel, FP16 storage) with a short timed region
    times every main launch and carries the forms comparison."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("bench.py --steps 20 --warmup 5 --no-cpu", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--steps", "20", "--warmup", "5",
                        "--no-cpu"], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    c = d["config"]
    assert "192x192x1024" in c["workload"] and c["nodes"] == 192 * 192 * 1024 and not c["unstable"]
    assert d["dtype"] == "f16-storage/f32" and c["precision"] == "fp16"
    ro = d["roofline"]
    assert ro["launches"] == 20 and ro["bytes_per_launch"] == c["nodes"] * 152
    assert "valu" in d
    if d["valu"] is not None:
        v = d["valu"]
        assert v["peak"] == 614.4 and 0.0 < v["frac"] < 1.0 and 0.0 < v["busy"] < 1.0
    f = d["forms"]
    assert f["plain"]["MLUPS"] > 0 and f["ensemble"]["vs_plain"] > 0 and f["adjoint"]["cost_vs_plain"] > 1.0
    gr = f["ensemble"]["graph"]
    assert gr["steps_per_graph"] == 50 and gr["MLUPS"] > 0 and gr["vs_plain_launches"] > 0
    print(json.dumps({"roofline": ro, "valu": d["valu"], "forms": f}), flush=True)
