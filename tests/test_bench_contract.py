"""The benchmark script's contract on the host (no GPU): one GPU only, and every traffic figure it
reports names the kernel-source digest of a committed profile."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_figures_come_from_committed_profiles():
    texts = "".join(open(p).read() for p in glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    for key, prof in list(bench.TRAFFIC.items()) + list(bench.TRAFFIC3D.items()):
        assert prof["bytes"] > 0, key
        assert f"`{prof['kernel_sha']}`" in texts, (key, prof["kernel_sha"])


def test_kernel_digest_covers_the_step_kernel_sources():
    # the digest changes with the sources it covers and with nothing else
    a = bench._kernel_source_sha()
    assert a == bench._kernel_source_sha(("lbm_step.hpp", "lbm_device.hpp")) and len(a) == 16
    assert bench._kernel_source_sha(bench.KERNEL3D_SOURCES) != a
