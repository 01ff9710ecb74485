"""CPU checks of the benchmark's command line: it measures one GPU only and
says so before touching a device; the committed counter summary has the
fields the bench line reads."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


import pytest


@pytest.mark.parametrize("name", ["round_kernel_slab_block_counters.json",
                                  "round_kernel_batched_1024_counters.json"])
def test_counter_summary_has_the_fields_the_bench_reads(name):
    d = json.load(open(os.path.join(ROOT, "profiles", name)))
    for k in ("kernel", "source_hash", "fetch_kib_per_launch", "write_kib_per_launch",
              "fetch_scale", "write_scale", "hbm_bytes_per_launch", "commands"):
        assert k in d
    # the scales come from a 1 GiB copy: bytes moved / counter reading
    assert abs(d["fetch_scale"] - 1048576.0 / d["copy_1GiB_fetch_kib"]) < 1e-9
    assert abs(d["write_scale"] - 1048576.0 / d["copy_1GiB_write_kib"]) < 1e-9
    hbm = (d["fetch_kib_per_launch"] * d["fetch_scale"] +
           d["write_kib_per_launch"] * d["write_scale"]) * 1024
    assert abs(hbm - d["hbm_bytes_per_launch"]) <= 1e-6 * hbm
