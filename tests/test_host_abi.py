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


@pytest.mark.parametrize("kw, msg, status", [
    (dict(model=0, L=13, R=4), "must be even", -1),
    (dict(model=0, L=2, R=4), "must be even, in [4", -1),
    (dict(model=0, L=32768, R=4), "must be even, in [4", -1),
    (dict(model=1, L=128, R=4), "must be even, in [4, 64]", -1),
    (dict(model=1, L=12, R=4), "3D kernels need a power of two", -5),
    (dict(model=0, L=1000, R=4), "whole replicas in LDS", -5),
    (dict(model=0, L=16, R=0), "R = 0", -1),
    (dict(model=0, L=16, R=5000), "R = 5000", -1),
    (dict(model=2, L=16, R=4), "unknown model", -1),
    (dict(model=0, L=16, R=4, beta=[0.3, -1, 0.4, 0.5]), "beta[1]", -1),
    (dict(model=0, L=16, R=4, beta=[0.3, float("nan"), 0.4, 0.5]), "beta[1]", -1),
    (dict(model=0, L=16, R=4, beta=[0.3, 100.0, 0.4, 0.5]), "underflow", -1),
])
def test_invalid_configs(pt, kw, msg, status):
    beta = kw.pop("beta", [0.3] * kw["R"]) if kw["R"] <= 16 else np.full(kw["R"], 0.3)
    cfg = pt.Config(kw["model"], kw["L"], kw["R"], np.asarray(beta, np.float64))
    with pytest.raises(pt.PTError, match=re.escape(msg)):
        pt.pt_workspace_bytes(cfg)
    with pytest.raises(pt.PTError) as e:
        pt.pt_create(cfg, 0, 256, 1 << 30)
    assert e.value.status == status


@pytest.mark.parametrize("L", [4, 6, 10, 12, 20, 24, 100, 300, 520])
def test_even_sides_that_are_not_powers_of_two_are_accepted(pt, L):
    """2D sides that are even but not powers of two (the paper's 300 among
    them) size a workspace: packed spins of ceil(L^2/32) words per walker."""
    R = 3
    n = pt.pt_workspace_bytes(pt.Config(0, L, R, np.array([0.3, 0.4, 0.5])))
    assert n >= 2 * R * 4 * ((L * L + 31) // 32)


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


def test_static_scratch_sizes(pt):
    """pt_create_static: the size query gives the workspace less its sweep
    scratch (tallies, mailboxes, boundary posts), configurations whose scratch
    exceeds the fixed array are refused, and so is a workspace below the
    queried size -- all before any device call."""
    beta = np.linspace(0.3, 0.55, 64)
    cfg = pt.Config(0, 1024, 64, beta, record_every=1, max_records=100)
    full, state = pt.pt_workspace_bytes(cfg), pt.pt_static_state_bytes(cfg)
    posts = 2 * 64 * 8 * (4 * 1024 // 32 + 2) * 8       # split-plan posts of 1024^2 x 64
    assert state + posts < full <= state + pt.PT_STATIC_SCRATCH_BYTES
    big = pt.Config(0, 1024, 512, np.full(512, 0.4))   # posts alone exceed 4 MiB
    with pytest.raises(pt.PTError, match="scratch") as e:
        pt.pt_static_state_bytes(big)
    assert e.value.status == -2
    with pytest.raises(pt.PTError, match="workspace of 1024 bytes") as e:
        pt.pt_create_static(cfg, 0, 256, 1024)
    assert e.value.status == -2
    with pytest.raises(pt.PTError, match="aligned"):
        pt.pt_create_static(cfg, 0, 0x1001, state)
    with pytest.raises(pt.PTError, match="L = 13"):
        pt.pt_static_state_bytes(pt.Config(0, 13, 2, np.array([0.3, 0.4])))


def test_probe_library_exports_its_entry_point(pt):
    """The VALU issue-rate probe (bench.py --form probe) is built beside the
    library and rejects launch shapes that do not fit its output buffer."""
    path = os.path.join(os.path.dirname(pt.LIB_PATH), "libptprobe.so")
    lib = C.CDLL(path)
    f = lib.ptprobe_run
    f.restype = C.c_int
    f.argtypes = [C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_size_t, C.c_void_p,
                  C.POINTER(C.c_float)]
    ms = C.c_float()
    assert f(0, 4, 256, 1, C.c_void_p(256), 1023, None, C.byref(ms)) != 0   # 1024 threads, 1023 words
    assert f(4, 1, 64, 1, C.c_void_p(256), 64, None, C.byref(ms)) != 0      # no such kind
    assert f(0, 1, 96, 1, C.c_void_p(256), 96, None, C.byref(ms)) != 0      # not whole waves


def test_header_constants_match_the_binding(pt):
    """The binding's copies of the header's numeric constants agree with it."""
    src = open(os.path.join(ROOT, "include", "pt.h")).read()
    for name in ("PT_MAX_SWEEPS_PER_LAUNCH", "PT_STATIC_SCRATCH_BYTES"):
        m = re.search(r"#define\s+%s\s+\(?(\d+)u(?:\s*<<\s*(\d+))?\)?" % name, src)
        assert m, name
        value = int(m.group(1)) << int(m.group(2) or 0)
        assert getattr(pt, name) == value, name
