"""Host-side checks of bench.py that need no GPU: the one-GPU rule, the
roofline's lower bound, and how committed counter summaries are matched to
the kernel sources, plan and launch length they were taken on."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    sys.path.insert(0, ROOT)
    import bench as _bench
    return _bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_lower_bound_per_attempt(bench):
    # a quarter of a Philox4x32-10 block with the counter's words 1-3 and the
    # key uniform (18 multiply-adds and 19 three-input XORs per block), plus
    # one compare
    assert bench.PHILOX_VALU_PER_BLOCK == 18 + 19
    assert bench.SLOTS_PER_ATTEMPT == pytest.approx(10.25)


SPLIT_PLAN = {"mode": 3, "tile_planes": 256, "sweeps_per_launch": 1, "block_threads": 1024}


def test_counter_summary_matches_only_its_own_kernel_sources(bench, tmp_path, monkeypatch):
    """The default workload's committed summaries are read while the kernel
    sources hash to the recorded value, for the recorded plan and launch
    length, and ignored otherwise."""
    f = bench.profile_fields("k_persist_split", "ising2d_L1024_R64", SPLIT_PLAN, 100)
    if f is None:
        pytest.skip("the committed summary was taken on other kernel sources")
    assert int(f["traffic_bytes_per_launch"]) > 16 * 2**20  # at least the lattices' read and write
    assert bench.measured_traffic("k_persist_split", "ising2d_L1024_R64", SPLIT_PLAN, 100) > 0
    assert bench.measured_valu_insts("k_persist_split", "ising2d_L1024_R64", SPLIT_PLAN, 100) > 0
    # another plan or launch length: not this summary's
    other = dict(SPLIT_PLAN, block_threads=512)
    assert bench.profile_fields("k_persist_split", "ising2d_L1024_R64", other, 100) is None
    assert bench.profile_fields("k_persist_split", "ising2d_L1024_R64", SPLIT_PLAN, 50) is None
    # other kernel sources: a changed source file changes the hash
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.profile_fields("k_persist_split", "ising2d_L1024_R64", SPLIT_PLAN, 100) is None
    assert bench.measured_traffic("k_persist_split", "ising2d_L1024_R64", SPLIT_PLAN, 100) is None
