"""Host side of the benchmark (no GPU): the one-GPU guard and the committed
main-kernel counter summaries that give the bench line its measured HBM
traffic."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
COUNTER_FILES = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_main_*_counters.json")))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_counter_summaries_exist():
    names = {os.path.basename(p)[len("k_main_"):-len("_counters.json")] for p in COUNTER_FILES}
    assert "single" in names


@pytest.mark.parametrize("path", COUNTER_FILES, ids=lambda p: os.path.basename(p))
def test_counter_summary_consistent(path):
    with open(path) as fh:
        d = json.load(fh)
    name = d["workload"]
    assert os.path.basename(path) == f"k_main_{name}_counters.json"
    assert glob.glob(os.path.join(ROOT, "profiles", f"k_main_{name}_*counters.md"))
    # HBM bytes per launch = scaled FETCH_SIZE + scaled WRITE_SIZE (KiB)
    hbm = (d["fetch_kib_per_dispatch"] * d["fetch_scale"] + d["write_kib_per_dispatch"] * d["write_scale"]) * 1024
    assert abs(hbm - d["hbm_bytes_per_launch"]) <= 1e-3 * hbm
    # a launch reads and writes every population at least once
    reps, prec, _ = bench.workload(name)
    nodes = sum(p["nx"] * p["ny"] * p["nz"] for p in reps)
    algorithmic = nodes * 2 * 19 * 2 * STORE_BYTES[prec]
    assert d["hbm_bytes_per_launch"] >= 0.95 * algorithmic
    assert d["hbm_bytes_per_launch"] <= 3.0 * algorithmic
    assert all("rocprofv3 --pmc" in c and "bench.py" in c for c in d["commands"])
    for e in d.get("shapes", []):
        hbm = (e["fetch_kib_per_dispatch"] * d["fetch_scale"] + e["write_kib_per_dispatch"] * d["write_scale"]) * 1024
        assert abs(hbm - e["hbm_bytes_per_launch"]) <= 1e-3 * hbm
        assert algorithmic * 0.95 <= e["hbm_bytes_per_launch"] <= 3.0 * algorithmic


@pytest.mark.parametrize("path", COUNTER_FILES, ids=lambda p: os.path.basename(p))
def test_traffic_only_for_the_profiled_shape(path):
    with open(path) as fh:
        d = json.load(fh)
    name = d["workload"]
    profiled = {(d["block"], d["zchunk"]): d["hbm_bytes_per_launch"]}
    for e in d.get("shapes", []):
        profiled.setdefault((e["block"], e["zchunk"]), e["hbm_bytes_per_launch"])
    current = d["kernel_hash"] == bench.kernel_hash()
    for block in (256, 512, 1024):
        for cz in (1, 2, 3, 4, 8, 16, 32):
            got = bench.traffic_from_profile(name, block, cz)
            if current and (block, cz) in profiled:
                assert got == profiled[(block, cz)]
            else:  # another shape, or counters taken on other kernel sources
                assert got is None


def test_cpu_baseline_leg():
    reps, prec, _ = bench.workload("parity")
    cb = bench.cpu_baseline(reps, budget_s=0.5)
    assert set(cb) == {"value", "unit", "cores", "kind", "sample"}
    assert cb["unit"] == "MLUPS" and cb["kind"] == "oracle" and cb["cores"] == bench.oracle_threads()
    assert cb["value"] > 0.0
    p = reps[0]
    assert f"{p['nx']}x{p['ny']}x{p['nz']}" in cb["sample"] and "FP64" in cb["sample"]
    assert "one replica" in cb["sample"]


def test_cpu_baseline_slab_of_a_large_replica():
    """A replica above max_nodes is sampled as a slab of slab_nz planes with
    the same cross-section and sphere."""
    reps, _, _ = bench.workload("parity")
    cb = bench.cpu_baseline(reps, budget_s=0.2, max_nodes=1000, slab_nz=16)
    assert "24x24x16" in cb["sample"] and "slab" in cb["sample"] and cb["value"] > 0.0


def test_timing_interval():
    assert bench.timing_every(20) == 1 and bench.timing_every(99) == 1 and bench.timing_every(100) == 10


def test_valu_peak():
    # 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles each, 2.4 GHz
    assert abs(bench.VALU_PEAK_GINSTR - 614.4) < 1e-9
