"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/pt.h declares, sizes workspaces and rejects invalid
configurations synchronously (pt_create validates before any HIP call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pt():
    from paper_2512_03825_amd import pt as _pt
    return _pt


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(pt):
    names = declared_functions()
    assert len(names) >= 10
    lib = C.CDLL(pt.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(pt.EXPORTS) == names


def test_workspace_bytes(pt):
    beta = np.linspace(0.3, 0.55, 64)
    n = pt.pt_workspace_bytes(pt.Config(0, 1024, 64, beta, record_every=1, max_records=10000))
    lattice = 64 * 1024 * 1024 // 8
    series = 2 * 10000 * 64 * 4
    assert 2 * lattice + series < n < 2 * lattice + series + 4 * 2**20
    # uploads need a staging area of one byte per site
    s0 = np.ones((64, 1024 * 1024), np.int8)
    n2 = pt.pt_workspace_bytes(pt.Config(0, 1024, 64, beta, init_spins=s0, record_every=1,
                                         max_records=10000))
    assert n2 >= n + 64 * 1024 * 1024


@pytest.mark.parametrize("kw, msg", [
    (dict(model=0, L=12, R=4), "power of two"),
    (dict(model=0, L=4, R=4), "power of two"),
    (dict(model=1, L=128, R=4), "power of two"),
    (dict(model=0, L=16, R=0), "R = 0"),
    (dict(model=0, L=16, R=5000), "R = 5000"),
    (dict(model=2, L=16, R=4), "unknown model"),
    (dict(model=0, L=16, R=4, beta=[0.3, -1, 0.4, 0.5]), "beta[1]"),
    (dict(model=0, L=16, R=4, beta=[0.3, float("nan"), 0.4, 0.5]), "beta[1]"),
    (dict(model=0, L=16, R=4, beta=[0.3, 100.0, 0.4, 0.5]), "underflow"),
])
def test_invalid_configs(pt, kw, msg):
    beta = kw.pop("beta", [0.3] * kw["R"]) if kw["R"] <= 16 else np.full(kw["R"], 0.3)
    cfg = pt.Config(kw["model"], kw["L"], kw["R"], np.asarray(beta, np.float64))
    with pytest.raises(pt.PTError, match=re.escape(msg)):
        pt.pt_workspace_bytes(cfg)
    with pytest.raises(pt.PTError) as e:
        pt.pt_create(cfg, 0, 256, 1 << 30)
    assert e.value.status == -1


def test_field_is_accepted_and_must_be_finite(pt):
    assert pt.pt_workspace_bytes(pt.Config(0, 16, 2, np.array([0.3, 0.4]), h=0.05)) > 0
    with pytest.raises(pt.PTError, match="h is not finite"):
        pt.pt_workspace_bytes(pt.Config(0, 16, 2, np.array([0.3, 0.4]), h=float("inf")))


def test_create_checks_buffers_before_device_work(pt):
    cfg = pt.Config(0, 16, 2, np.array([0.3, 0.4]))
    with pytest.raises(pt.PTError, match="aligned"):
        pt.pt_create(cfg, 0, 0x1001, 1 << 30)
    with pytest.raises(pt.PTError, match="NULL"):
        pt.pt_create(cfg, 0, 0, 1 << 30)
    bad = np.ones((2, 256), np.int8)
    bad[1, 7] = 0
    with pytest.raises(pt.PTError, match=r"init_spins\[263\]"):
        pt.pt_create(pt.Config(0, 16, 2, np.array([0.3, 0.4]), init_spins=bad), 0, 256, 1 << 30)
    with pytest.raises(pt.PTError, match="workspace of 1024 bytes"):
        pt.pt_create(cfg, 0, 256, 1024)


def test_server_options_are_checked(pt):
    """Server options are validated on the host: the table size grows with the
    batched lanes the size classes add, and bad options are refused."""
    one = pt.pt_server_overhead_bytes(pt.server_opts(class_sites=()))
    two = pt.pt_server_overhead_bytes(pt.server_opts(class_sites=(4096,)))
    three = pt.pt_server_overhead_bytes(pt.server_opts(class_sites=(4096, 65536)))
    assert one < two < three
    for kw, msg in [(dict(class_sites=(4096, 4096)), "ascend"),
                    (dict(class_sites=(65536, 4096)), "ascend"),
                    (dict(class_sites=(0, 4096)), "after a zero entry"),
                    (dict(tiled_lanes=0), "tiled_lanes"),
                    (dict(depth=9), "depth"),
                    (dict(cycle_sweeps=17), "cycle_sweeps"),
                    (dict(max_jobs=0), "max_jobs")]:
        with pytest.raises(pt.PTError, match=msg):
            pt.pt_server_overhead_bytes(pt.server_opts(**kw))
