"""Host-side bookkeeping of bench.py, checked without a GPU.

The roofline's `traffic` comes from the committed rocprofv3 counter summaries,
keyed by the hot kernel's configuration and valid only for the kernel source
the counters were taken on; a multi-GPU request is refused before any device is
touched.
"""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

HOT_C3 = {"hot_group": 8, "hot_pages": True, "hot_fp32": False, "hot_tile": 2048,
          "hot_threads": 1024}


def _profile_value(cfg, key):
    """The number after `key:` in a committed counter summary, read with a
    regular expression of its own (not bench's parser)."""
    text = open(os.path.join(ROOT, "profiles", f"spgemm_hbm_traffic_{cfg}.txt")).read()
    m = re.search(r"^" + re.escape(key) + r":\s*([0-9.eE+-]+)\s*$", text, re.M)
    return float(m.group(1)) if m else None


@pytest.mark.parametrize("name", ["spgemm_hbm_traffic_c3.txt", "spgemm_hbm_traffic_c2.txt",
                                  "spgemm_group_counters_c3.txt",
                                  "spgemm_group_counters_c2.txt"])
def test_counter_summaries_match_the_kernel_source(name):
    """The committed counters of the product kernels were taken on the committed
    kernel source: a kernel change is re-profiled before it is committed."""
    text = open(os.path.join(ROOT, "profiles", name)).read()
    m = re.search(r"^kernel_source_sha256_16:\s*([0-9a-f]{16})\s*$", text, re.M)
    assert m, name
    assert m.group(1) == bench.kernel_hash(), name


@pytest.mark.parametrize("cfg", ["c3", "c2"])
def test_traffic_of_the_hot_kernel(cfg):
    """The lookup returns the copy-calibrated bytes per launch of the hot kernel
    (groups of 8, page windows, FP64, 2048-column windows)."""
    want = _profile_value(cfg, "group8_pages_f64_tile2048_hbm_bytes_per_launch")
    assert want is not None and want > 1e9
    assert bench.read_traffic(HOT_C3, cfg, 0) == want


def test_traffic_of_other_kernels_and_workloads_is_none():
    st = dict(HOT_C3, hot_tile=4096)           # no summary line for this configuration
    assert bench.read_traffic(st, "c3", 0) is None
    assert bench.read_traffic(HOT_C3, "c3", 1) is None                  # mixed precision
    assert bench.read_traffic(HOT_C3, "c3", 0, grid=256) is None         # another size
    assert bench.read_traffic(HOT_C3, "c3", 0, method="newton") is None  # another method
    assert bench.read_traffic(HOT_C3, "c4", 0) is None                  # no summary


def test_traffic_is_none_once_the_kernel_changed(monkeypatch):
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.read_traffic(HOT_C3, "c3", 0) is None


def test_kernel_name():
    assert bench.kernel_name(HOT_C3, 2048) == "k_spgemm_rows<double,8,2048,1024,pages>"
    st = dict(HOT_C3, hot_group=4, hot_pages=False, hot_fp32=True)
    assert bench.kernel_name(st, 4096) == "k_spgemm_rows<float,4,4096,1024>"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
