"""Host-side parts of bench.py (no GPU): the one-GPU contract, and the rule that
measured HBM traffic is reported only while the kernel sources still hash to the
value recorded beside the counters."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr


def test_kernel_sources_exist_and_hash_is_stable():
    for rel in bench.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(ROOT, rel)), rel
    h = bench.sources_hash()
    assert len(h) == 16 and h == bench.sources_hash()


def _summary(path, sha, hbm):
    with open(path, "w") as f:
        f.write("# counters\n#   k = 1 (a comment line is not a key)\n")
        f.write("kernel_sources_sha256 = %s\nworkload = jet128 fp32\nhbm_bytes_per_launch = %s\n" % (sha, hbm))


def test_traffic_reported_only_for_the_current_kernel(tmp_path, monkeypatch):
    path = str(tmp_path / "traffic.txt")
    monkeypatch.setitem(bench.TRAFFIC_FILES, "jet128", path)
    _summary(path, bench.sources_hash(), "768183226")
    assert bench.measured_traffic("jet128", "fp32") == 768183226.0
    assert bench.measured_traffic("jet128", "fp16") is None  # counters cover binary32 storage only
    assert bench.measured_traffic("no-such-workload", "fp32") is None
    _summary(path, "0" * 16, "768183226")  # counters taken on another kernel
    assert bench.measured_traffic("jet128", "fp32") is None
    _summary(path, bench.sources_hash(), "not-a-number")
    assert bench.measured_traffic("jet128", "fp32") is None


@pytest.mark.parametrize("name", sorted(bench.TRAFFIC_FILES))
def test_committed_traffic_summaries_parse(name):
    """Every committed summary carries the keys the bench reads (its hash may be
    older than the sources; then the bench reports null)."""
    path = bench.TRAFFIC_FILES[name]
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    assert len(kv["kernel_sources_sha256"]) == 16
    assert float(kv["hbm_bytes_per_launch"]) > 0


def test_smooth_state_covers_every_node():
    """inputs.smooth_state, the busy-state start the bench times beside the
    headline: library layout (z, y, x), binary32, phi inside (0, 1) everywhere and
    velocity, density and stress deviations of the stated sizes."""
    from paper_2403_15773_amd import inputs
    st = inputs.smooth_state(48, 40, 36)
    assert st["phi"].shape == (36, 40, 48) and st["u"].shape == (3, 36, 40, 48) and st["P"].shape == (6, 36, 40, 48)
    assert all(v.dtype == np.float32 for v in st.values())
    assert 0.09 < st["phi"].min() and st["phi"].max() < 0.91
    assert np.abs(st["u"]).max() <= 0.02 and np.abs(st["rho_dev"]).max() <= 1e-3 and np.abs(st["P"]).max() <= 1e-4
    assert np.abs(st["u"]).max() > 0.015 and np.abs(st["P"]).max() > 5e-5
    # no quiescent region: almost every node moves, and the phase field varies through the lattice
    assert (np.abs(st["u"]).max(axis=0) < 1e-4).mean() < 0.01
    assert st["phi"].std() > 0.1
