"""ctypes binding of the C ABI in include/pt.h (argument marshalling only).

Every step of the method runs inside libptmi.so (gfx950 kernels + host
library).  PyTorch only provides the device workspace and the stream.  If the
library has not been built this module raises at import: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptmi.so")

PT_ABI_VERSION = 1
PT_ALL_SLOTS = 0xFFFFFFFF
PT_MAX_SWEEPS_PER_LAUNCH = 16
PT_ISING2D, PT_EA3D = 0, 1
PT_PLAN_AUTO, PT_PLAN_FUSED, PT_PLAN_TILED, PT_PLAN_PERSISTENT, PT_PLAN_LANES, PT_PLAN_WAVE = 0, 1, 2, 3, 4, 5
STATUS = {0: "PT_OK", -1: "PT_EINVAL", -2: "PT_ENOMEM", -3: "PT_EDEVICE", -4: "PT_ESTATE",
          -5: "PT_EUNSUPPORTED"}

# Every symbol include/pt.h declares.
EXPORTS = ("pt_workspace_bytes", "pt_create", "pt_create_static", "pt_set_plan", "pt_get_plan", "pt_set_wait_limit", "pt_sweep",
           "pt_exchange", "pt_run", "pt_observables", "pt_flip_thresholds", "pt_swap_threshold",
           "pt_destroy", "pt_last_error", "pt_batch_workspace_bytes", "pt_batch_create",
           "pt_batch_run", "pt_batch_observables", "pt_batch_group_plan", "pt_batch_destroy",
           "pt_server_overhead_bytes", "pt_server_create", "pt_server_submit", "pt_server_step",
           "pt_server_done", "pt_server_result", "pt_server_release", "pt_server_stats_get",
           "pt_server_clock", "pt_server_destroy")
PT_JOB_KEEP_SPINS = 1
PT_STATIC_SCRATCH_BYTES = 4 << 20


class PTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class pt_config(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32), ("model", C.c_uint32), ("L", C.c_uint32), ("R", C.c_uint32),
        ("beta", C.POINTER(C.c_double)), ("J", C.c_double), ("h", C.c_double),
        ("seed", C.c_uint32), ("stream_id", C.c_uint32), ("coupling_seed", C.c_uint32),
        ("init_spins", C.POINTER(C.c_int8)), ("couplings", C.POINTER(C.c_int8)),
        ("record_every", C.c_uint32), ("max_records", C.c_uint32),
    ]


class pt_plan(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("tile_planes", C.c_uint32),
                ("sweeps_per_launch", C.c_uint32), ("block_threads", C.c_uint32)]


class pt_obs(C.Structure):
    _fields_ = [
        ("E_series", C.POINTER(C.c_int32)), ("M_series", C.POINTER(C.c_int32)),
        ("E_slot", C.POINTER(C.c_int32)), ("M_slot", C.POINTER(C.c_int32)),
        ("swap_att", C.POINTER(C.c_uint64)), ("swap_acc", C.POINTER(C.c_uint64)),
        ("walker_at", C.POINTER(C.c_uint32)), ("spins", C.POINTER(C.c_int8)),
        ("spins_slot", C.c_uint32), ("sweeps_done", C.c_uint64), ("exchanges_done", C.c_uint64),
        ("n_records", C.c_uint32),
    ]


class pt_server_opts(C.Structure):
    _fields_ = [("max_jobs", C.c_uint32), ("max_walkers", C.c_uint32), ("tiled_lanes", C.c_uint32),
                ("depth", C.c_uint32), ("cycle_sweeps", C.c_uint32), ("tiled_sweeps", C.c_uint32),
                ("class_sites", C.c_uint32 * 3)]


class pt_job_info(C.Structure):
    _fields_ = [("job_id", C.c_uint64), ("arrival", C.c_double), ("admitted", C.c_double),
                ("finished", C.c_double), ("attempts", C.c_uint64), ("lane", C.c_uint32),
                ("pad", C.c_uint32)]


class pt_server_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "submitted", "pending", "resident", "finished", "arena_bytes", "arena_used", "arena_peak",
        "walkers_resident", "batched_cycles", "tiled_steps", "attempts_finished")]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libptmi.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2512_03825_amd/build.py" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    P = C.POINTER
    sig = {
        "pt_workspace_bytes": (C.c_size_t, [P(pt_config)]),
        "pt_create": (st, [P(pt_config), vp, vp, C.c_size_t, P(vp)]),
        "pt_create_static": (st, [P(pt_config), vp, vp, P(C.c_size_t), P(vp)]),
        "pt_set_plan": (st, [vp, P(pt_plan)]),
        "pt_get_plan": (st, [vp, P(pt_plan)]),
        "pt_set_wait_limit": (st, [vp, C.c_uint32]),
        "pt_sweep": (st, [vp, C.c_uint32]),
        "pt_exchange": (st, [vp]),
        "pt_run": (st, [vp, C.c_uint32, C.c_uint32]),
        "pt_observables": (st, [vp, P(pt_obs)]),
        "pt_flip_thresholds": (st, [vp, P(C.c_uint32)]),
        "pt_swap_threshold": (st, [vp, C.c_uint32, C.c_int64, P(C.c_uint64)]),
        "pt_destroy": (None, [vp]),
        "pt_last_error": (C.c_char_p, []),
        "pt_batch_workspace_bytes": (C.c_size_t, [P(pt_config), C.c_uint32]),
        "pt_batch_create": (st, [P(pt_config), C.c_uint32, vp, vp, C.c_size_t, P(vp)]),
        "pt_batch_run": (st, [vp, C.c_uint32, C.c_uint32]),
        "pt_batch_observables": (st, [vp, C.c_uint32, P(pt_obs)]),
        "pt_batch_group_plan": (st, [vp, C.c_uint32, P(C.c_uint32), P(C.c_uint32), P(C.c_uint32),
                                     P(C.c_uint32)]),
        "pt_batch_destroy": (None, [vp]),
        "pt_server_overhead_bytes": (C.c_size_t, [P(pt_server_opts)]),
        "pt_server_create": (st, [P(pt_server_opts), vp, C.c_size_t, P(vp)]),
        "pt_server_submit": (st, [vp, P(pt_config), C.c_uint64, C.c_uint32, C.c_uint32, C.c_double,
                                  P(C.c_uint64)]),
        "pt_server_step": (st, [vp, C.c_uint32, P(C.c_uint32)]),
        "pt_server_done": (st, [vp, P(pt_job_info), C.c_uint32, P(C.c_uint32)]),
        "pt_server_result": (st, [vp, C.c_uint64, P(pt_obs)]),
        "pt_server_release": (st, [vp, C.c_uint64]),
        "pt_server_stats_get": (st, [vp, P(pt_server_stats)]),
        "pt_server_clock": (C.c_double, [vp]),
        "pt_server_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status):
    if status != 0:
        raise PTError(status, _lib.pt_last_error().decode())


def _p(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class Config:
    """Owns a pt_config and the host arrays it points to."""

    def __init__(self, model, L, R, beta, J=1.0, h=0.0, seed=1, stream_id=0, coupling_seed=None,
                 init_spins=None, couplings=None, record_every=0, max_records=0):
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        if self.beta.shape != (int(R),):
            raise ValueError("beta must have shape (R,)")
        c = pt_config()
        c.abi_version, c.model, c.L, c.R = PT_ABI_VERSION, int(model), int(L), int(R)
        c.beta = _p(self.beta, C.c_double)
        c.J, c.h = float(J), float(h)
        c.seed, c.stream_id = int(seed), int(stream_id)
        c.coupling_seed = int(seed if coupling_seed is None else coupling_seed)
        self.init_spins = self.couplings = None
        if init_spins is not None:
            self.init_spins = np.ascontiguousarray(init_spins, dtype=np.int8)
            c.init_spins = _p(self.init_spins, C.c_int8)
        if couplings is not None:
            self.couplings = np.ascontiguousarray(couplings, dtype=np.int8)
            c.couplings = _p(self.couplings, C.c_int8)
        c.record_every, c.max_records = int(record_every), int(max_records)
        self.c = c
        self.dim = 3 if int(model) == PT_EA3D else 2
        self.N = int(L) ** self.dim
        self.R = int(R)


def pt_workspace_bytes(cfg: Config) -> int:
    n = _lib.pt_workspace_bytes(C.byref(cfg.c))
    if n == 0:
        raise PTError(-1, _lib.pt_last_error().decode())
    return int(n)


def pt_create(cfg: Config, hip_stream: int, workspace_ptr: int, workspace_bytes: int):
    out = C.c_void_p()
    _check(_lib.pt_create(C.byref(cfg.c), C.c_void_p(hip_stream), C.c_void_p(workspace_ptr),
                          C.c_size_t(workspace_bytes), C.byref(out)))
    return out


def pt_static_state_bytes(cfg: Config) -> int:
    """Size query of pt_create_static (d_state = NULL)."""
    n = C.c_size_t(0)
    _check(_lib.pt_create_static(C.byref(cfg.c), None, None, C.byref(n), None))
    return int(n.value)


def pt_create_static(cfg: Config, hip_stream: int, state_ptr: int, state_bytes: int):
    out = C.c_void_p()
    n = C.c_size_t(state_bytes)
    _check(_lib.pt_create_static(C.byref(cfg.c), C.c_void_p(hip_stream), C.c_void_p(state_ptr),
                                 C.byref(n), C.byref(out)))
    return out


def pt_set_plan(ctx, mode, tile_planes=0, sweeps_per_launch=0, block_threads=0):
    p = pt_plan(int(mode), int(tile_planes), int(sweeps_per_launch), int(block_threads))
    _check(_lib.pt_set_plan(ctx, C.byref(p)))


def pt_get_plan(ctx) -> dict:
    p = pt_plan()
    _check(_lib.pt_get_plan(ctx, C.byref(p)))
    return {"mode": p.mode, "tile_planes": p.tile_planes,
            "sweeps_per_launch": p.sweeps_per_launch, "block_threads": p.block_threads}


def pt_set_wait_limit(ctx, polls: int):
    _check(_lib.pt_set_wait_limit(ctx, int(polls)))


def pt_sweep(ctx, n_sweeps: int):
    _check(_lib.pt_sweep(ctx, int(n_sweeps)))


def pt_exchange(ctx):
    _check(_lib.pt_exchange(ctx))


def pt_run(ctx, n_sweeps: int, exchange_every: int):
    _check(_lib.pt_run(ctx, int(n_sweeps), int(exchange_every)))


def pt_observables(ctx, R: int, N: int, max_records: int, spins=None, series=True) -> dict:
    """spins: None, a slot index, or "all" (slot order)."""
    return _observe(lambda o: _lib.pt_observables(ctx, C.byref(o)), R, N, max_records, spins, series)


def _observe(call, R, N, max_records, spins, series):
    o = pt_obs()
    E_slot = np.zeros(R, np.int32)
    M_slot = np.zeros(R, np.int32)
    att = np.zeros((R, R), np.uint64)
    acc = np.zeros((R, R), np.uint64)
    wat = np.zeros(R, np.uint32)
    o.E_slot, o.M_slot = _p(E_slot, C.c_int32), _p(M_slot, C.c_int32)
    o.swap_att, o.swap_acc = _p(att, C.c_uint64), _p(acc, C.c_uint64)
    o.walker_at = _p(wat, C.c_uint32)
    Es = Ms = None
    if series:
        Es = np.zeros((max(max_records, 1), R), np.int32)
        Ms = np.zeros((max(max_records, 1), R), np.int32)
        o.E_series, o.M_series = _p(Es, C.c_int32), _p(Ms, C.c_int32)
    sp = None
    if spins is not None:
        if spins == "all":
            sp = np.zeros((R, N), np.int8)
            o.spins_slot = PT_ALL_SLOTS
        else:
            sp = np.zeros(N, np.int8)
            o.spins_slot = int(spins)
        o.spins = _p(sp, C.c_int8)
    _check(call(o))
    n = int(o.n_records)
    return {"E_slot": E_slot, "M_slot": M_slot, "swap_att": att, "swap_acc": acc,
            "walker_at": wat, "spins": sp,
            "E_series": Es[:n] if Es is not None else None,
            "M_series": Ms[:n] if Ms is not None else None,
            "sweeps_done": int(o.sweeps_done), "exchanges_done": int(o.exchanges_done),
            "n_records": n}


def pt_flip_thresholds(ctx, R: int) -> np.ndarray:
    out = np.zeros((R, 16), np.uint32)
    _check(_lib.pt_flip_thresholds(ctx, _p(out, C.c_uint32)))
    return out


def pt_swap_threshold(ctx, k: int, d: int) -> int:
    T = C.c_uint64()
    _check(_lib.pt_swap_threshold(ctx, int(k), int(d), C.byref(T)))
    return int(T.value)


def pt_destroy(ctx):
    _lib.pt_destroy(ctx)


def pt_last_error() -> str:
    return _lib.pt_last_error().decode()


class Simulation:
    """A context plus a torch-owned device workspace on the current torch stream.

    static_scratch=True creates it with pt_create_static: the workspace then
    holds only the state, and the sweep scratch is the library's fixed array."""

    def __init__(self, cfg: Config, device="cuda", stream=None, static_scratch=False):
        import torch
        self.cfg = cfg
        self.nbytes = pt_static_state_bytes(cfg) if static_scratch else pt_workspace_bytes(cfg)
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        ptr = self.workspace.data_ptr()
        ptr = (ptr + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        create = pt_create_static if static_scratch else pt_create
        self.ctx = create(cfg, self.stream.cuda_stream, ptr, self.nbytes)

    def set_plan(self, mode, tile_planes=0, sweeps_per_launch=0, block_threads=0):
        pt_set_plan(self.ctx, mode, tile_planes, sweeps_per_launch, block_threads)

    def plan(self):
        return pt_get_plan(self.ctx)

    def set_wait_limit(self, polls):
        pt_set_wait_limit(self.ctx, polls)

    def sweep(self, n):
        pt_sweep(self.ctx, n)

    def exchange(self):
        pt_exchange(self.ctx)

    def run(self, n, every):
        pt_run(self.ctx, n, every)

    def observables(self, spins=None, series=True):
        return pt_observables(self.ctx, self.cfg.R, self.cfg.N, self.cfg.c.max_records,
                              spins=spins, series=series)

    def close(self):
        if getattr(self, "ctx", None):
            try:
                pt_destroy(self.ctx)
            except TypeError:  # interpreter shutdown already tore down ctypes
                pass
            self.ctx = None

    def __del__(self):
        self.close()


def pt_batch_workspace_bytes(cfgs) -> int:
    arr = (pt_config * len(cfgs))(*[c.c for c in cfgs])
    n = _lib.pt_batch_workspace_bytes(arr, len(cfgs))
    if n == 0:
        raise PTError(-1, _lib.pt_last_error().decode())
    return int(n)


class Batch:
    """Many instances advanced together (pt_batch_*), torch-owned workspace."""

    def __init__(self, cfgs, device="cuda", stream=None):
        import torch
        self.cfgs = list(cfgs)
        self._arr = (pt_config * len(self.cfgs))(*[c.c for c in self.cfgs])
        self.nbytes = pt_batch_workspace_bytes(self.cfgs)
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        out = C.c_void_p()
        _check(_lib.pt_batch_create(self._arr, len(self.cfgs), C.c_void_p(self.stream.cuda_stream),
                                    C.c_void_p(ptr), C.c_size_t(self.nbytes), C.byref(out)))
        self.b = out

    def run(self, n_sweeps, exchange_every):
        _check(_lib.pt_batch_run(self.b, int(n_sweeps), int(exchange_every)))

    def observables(self, i, spins=None, series=True):
        c = self.cfgs[i]
        return _observe(lambda o: _lib.pt_batch_observables(self.b, int(i), C.byref(o)), c.R, c.N,
                        c.c.max_records, spins, series)

    def group_plans(self):
        out, g = [], 0
        while True:
            L, W, T, K = C.c_uint32(), C.c_uint32(), C.c_uint32(), C.c_uint32()
            if _lib.pt_batch_group_plan(self.b, g, C.byref(L), C.byref(W), C.byref(T), C.byref(K)) != 0:
                return out
            out.append({"L": L.value, "walkers_per_wg": W.value, "block_threads": T.value,
                        "sweeps_per_cycle": K.value})
            g += 1

    def close(self):
        if getattr(self, "b", None):
            try:
                _lib.pt_batch_destroy(self.b)
            except TypeError:
                pass
            self.b = None

    def __del__(self):
        self.close()


def server_opts(max_jobs=1024, max_walkers=32768, tiled_lanes=1, depth=2, cycle_sweeps=10,
                tiled_sweeps=5, class_sites=(4096, 65536)) -> pt_server_opts:
    cs = list(class_sites) + [0] * (3 - len(class_sites))
    return pt_server_opts(int(max_jobs), int(max_walkers), int(tiled_lanes), int(depth),
                          int(cycle_sweeps), int(tiled_sweeps), (C.c_uint32 * 3)(*map(int, cs)))


def pt_server_overhead_bytes(opts: pt_server_opts) -> int:
    n = _lib.pt_server_overhead_bytes(C.byref(opts))
    if n == 0:
        raise PTError(-1, _lib.pt_last_error().decode())
    return int(n)


class Server:
    """Served form (pt_server_*): jobs admitted by device-memory budget into a
    torch-owned arena of arena_bytes, advanced together as they arrive."""

    def __init__(self, arena_bytes, device="cuda", **opts):
        import torch
        self.opts = server_opts(**opts)
        self.nbytes = pt_server_overhead_bytes(self.opts) + int(arena_bytes)
        self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        torch.cuda.synchronize(device)
        out = C.c_void_p()
        _check(_lib.pt_server_create(C.byref(self.opts), C.c_void_p(ptr), C.c_size_t(self.nbytes),
                                     C.byref(out)))
        self.sv = out
        self.jobs = {}

    def submit(self, cfg: Config, n_sweeps, exchange_every, keep_spins=False, arrival=-1.0) -> int:
        jid = C.c_uint64()
        _check(_lib.pt_server_submit(self.sv, C.byref(cfg.c), int(n_sweeps), int(exchange_every),
                                     PT_JOB_KEEP_SPINS if keep_spins else 0, float(arrival),
                                     C.byref(jid)))
        self.jobs[jid.value] = cfg
        return jid.value

    def step(self, wait_us=0) -> int:
        n = C.c_uint32()
        _check(_lib.pt_server_step(self.sv, int(wait_us), C.byref(n)))
        return n.value

    def done(self, cap=256):
        arr = (pt_job_info * cap)()
        n = C.c_uint32()
        _check(_lib.pt_server_done(self.sv, arr, cap, C.byref(n)))
        return [{"job_id": a.job_id, "arrival": a.arrival, "admitted": a.admitted,
                 "finished": a.finished, "attempts": a.attempts, "lane": a.lane}
                for a in arr[:n.value]]

    def result(self, job_id, spins=None, series=True):
        c = self.jobs[job_id]
        return _observe(lambda o: _lib.pt_server_result(self.sv, int(job_id), C.byref(o)), c.R, c.N,
                        c.c.max_records, spins, series)

    def release(self, job_id):
        _check(_lib.pt_server_release(self.sv, int(job_id)))
        self.jobs.pop(job_id, None)

    def stats(self) -> dict:
        s = pt_server_stats()
        _check(_lib.pt_server_stats_get(self.sv, C.byref(s)))
        return {n: int(getattr(s, n)) for n, _ in pt_server_stats._fields_}

    def clock(self) -> float:
        return float(_lib.pt_server_clock(self.sv))

    def close(self):
        if getattr(self, "sv", None):
            try:
                _lib.pt_server_destroy(self.sv)
            except TypeError:
                pass
            self.sv = None

    def __del__(self):
        self.close()
