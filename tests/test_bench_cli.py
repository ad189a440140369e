"""bench.py's command-line contract and its link to the committed profiles (CPU only).

- More than one GPU is refused with a message, before anything touches a GPU.
- An unknown section is refused.
- The committed HBM-counter summary was taken with the current kernel sources
  (its source hash matches), so the bench line's `traffic` is the counted
  figure, not null; a kernel change without a new profile fails here.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_unknown_section_is_refused():
    r = _run("--sections", "nosuchsection")
    assert r.returncode != 0
    assert "unknown section" in r.stderr


def test_counter_profile_matches_the_kernel_sources():
    txt = open(os.path.join(ROOT, bench.TRAFFIC_SUMMARY)).read()
    assert f"kernel_source_sha256_16: {bench.kernel_source_hash()}" in txt
    for label in ("fp64_state_fp32_dir:resid", "fp64:pre_inv"):
        t = bench.measured_traffic(label)
        assert t is not None and t > 1e8, (label, t)
