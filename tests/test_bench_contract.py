"""Host-side pieces of bench.py: the one-GPU guard, the counter table's source hashes, and
the CPU baseline's reported fields (on a tiny workload)."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_1410_1921_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counter_entries_match_their_sources():
    # a committed counter figure is reported only for the sources it was taken on; after
    # a kernel edit the bench reports traffic null until the counters are taken again
    for kernel, c in bench.COUNTERS.items():
        h = hashlib.sha256()
        for f in c["files"]:
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != c["sha"]:
            assert bench.traffic_gb(kernel, c["workload"]) is None
            pytest.skip(f"{kernel}: counter figures predate the current sources")
        gb = bench.traffic_gb(kernel, c["workload"])
        assert gb == pytest.approx((c["fetch_kib"] * bench.FETCH_FACTOR +
                                    c["write_kib"] * bench.WRITE_FACTOR) * 1024 / 1e9, rel=1e-4)
        assert bench.traffic_gb(kernel, "another workload") is None
    assert bench.traffic_gb("no such kernel", "recon128_eps0.40_d12_mis_ch4_400K") is None


def test_counter_traffic_exceeds_algorithmic_bytes():
    # L2-miss traffic can only add to the algorithmic bytes of the profiled launch
    nf = {"recon128_eps0.40_d12_mis_ch4_400K": 839927, "recon512_eps0.25_d16": 33554434}
    per_update = {"k_sweep7": bench.BYTES_D3Q7, "k_sweep19": bench.BYTES_D3Q19}
    for kernel, c in bench.COUNTERS.items():
        algo = nf[c["workload"]] * per_update[kernel.split("<")[0]] / 1e9
        gb = (c["fetch_kib"] * bench.FETCH_FACTOR + c["write_kib"] * bench.WRITE_FACTOR) * 1024 / 1e9
        assert algo < gb < 1.5 * algo, kernel


def test_cpu_baseline_fields():
    w = dict(W.SMALL_32, name="recon32_eps0.35_d8")
    w["recon"] = dict(w["recon"], psd="chord13")
    out = bench.cpu_baseline(W, w, 5)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "5 D3Q19 BGK steps of the whole lattice" in out["sample"]
