"""Plain CPU oracle for Metropolis-Hastings with Parallel Tempering (ctypes wrapper).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU
baseline leg may use this package; the product path (the HIP library and its
binding) never imports it.  The arithmetic lives in ``oracle.c``; this module only
builds that file with gcc and marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ISING2D = 0
EA3D = 1


def compile_source(src: str, out: str) -> str:
    """gcc one oracle source file into a shared library (FP contraction off)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call([
        "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
        "-shared", "-Wall", "-Wextra", "-I", _HERE, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


class _Config(C.Structure):
    _fields_ = [
        ("model", C.c_int32), ("L", C.c_int32), ("R", C.c_int32),
        ("beta", C.POINTER(C.c_double)), ("J", C.c_double), ("h", C.c_double),
        ("seed", C.c_uint32), ("stream_id", C.c_uint32), ("coupling_seed", C.c_uint32),
        ("init_spins", C.POINTER(C.c_int8)), ("couplings", C.POINTER(C.c_int8)),
        ("record_every", C.c_uint32), ("max_records", C.c_uint32),
    ]


_libs = {}


def lib(path: str = None):
    """The loaded oracle library (the default build, or another compiled copy)."""
    path = path or _LIB_PATH
    if path not in _libs:
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(_Config)]
        L.orc_destroy.argtypes = [vp]
        L.orc_sweep.argtypes = [vp, C.c_uint64]
        L.orc_exchange.argtypes = [vp]
        L.orc_run.argtypes = [vp, C.c_uint64, C.c_uint32]
        for name, rt in [("orc_num_sites", C.c_int64), ("orc_sweeps_done", C.c_uint64),
                         ("orc_exchanges_done", C.c_uint64), ("orc_n_records", C.c_uint32)]:
            getattr(L, name).restype = rt
            getattr(L, name).argtypes = [vp]
        for name in ["orc_get_spins", "orc_get_couplings", "orc_get_labels"]:
            getattr(L, name).argtypes = [vp, vp]
        for name in ["orc_get_energy", "orc_get_series", "orc_get_swaps", "orc_recount"]:
            getattr(L, name).argtypes = [vp, vp, vp]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_flip_accept.restype = C.c_int
        L.orc_flip_accept.argtypes = [C.c_double, C.c_double, C.c_uint32]
        L.orc_swap_accept.restype = C.c_int
        L.orc_swap_accept.argtypes = [C.c_double, C.c_double, C.c_double, C.c_uint32]
        _libs[path] = L
    return _libs[path]


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: counter (4 words), key (2 words) -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def flip_accept(beta: float, dE: float, r: int) -> bool:
    return bool(lib().orc_flip_accept(beta, dE, r))


def swap_accept(beta_k: float, beta_k1: float, dE: float, r: int) -> bool:
    return bool(lib().orc_swap_accept(beta_k, beta_k1, dE, r))


class Oracle:
    """One parallel-tempering simulation held by the C oracle."""

    lib_path = None  # subclasses bound to another compiled copy override this

    def __init__(self, model, L, R, beta, J=1.0, h=0.0, seed=1, stream_id=0,
                 coupling_seed=None, init_spins=None, couplings=None,
                 record_every=0, max_records=0):
        self._L = lib(self.lib_path)
        self.model, self.L, self.R = int(model), int(L), int(R)
        self.dim = 3 if self.model == EA3D else 2
        self.N = self.L ** self.dim
        self._beta = np.ascontiguousarray(beta, dtype=np.float64)
        assert self._beta.shape == (self.R,)
        cfg = _Config()
        cfg.model, cfg.L, cfg.R = self.model, self.L, self.R
        cfg.beta = self._beta.ctypes.data_as(C.POINTER(C.c_double))
        cfg.J, cfg.h = float(J), float(h)
        cfg.seed, cfg.stream_id = int(seed), int(stream_id)
        cfg.coupling_seed = int(seed if coupling_seed is None else coupling_seed)
        keep = []
        if init_spins is not None:
            a = np.ascontiguousarray(init_spins, dtype=np.int8).reshape(self.R, self.N)
            keep.append(a)
            cfg.init_spins = a.ctypes.data_as(C.POINTER(C.c_int8))
        if couplings is not None:
            a = np.ascontiguousarray(couplings, dtype=np.int8).reshape(3, self.N)
            keep.append(a)
            cfg.couplings = a.ctypes.data_as(C.POINTER(C.c_int8))
        cfg.record_every, cfg.max_records = int(record_every), int(max_records)
        self._st = self._L.orc_create(C.byref(cfg))
        if not self._st:
            raise ValueError("oracle rejected the configuration")

    def __del__(self):
        st = getattr(self, "_st", None)
        if st:
            self._L.orc_destroy(st)
            self._st = None

    # -- dynamics -----------------------------------------------------------
    def sweep(self, n=1):
        self._L.orc_sweep(self._st, int(n))

    def exchange(self):
        self._L.orc_exchange(self._st)

    def run(self, n, every=0):
        self._L.orc_run(self._st, int(n), int(every))

    # -- state ----------------------------------------------------------------
    @property
    def sweeps_done(self):
        return int(self._L.orc_sweeps_done(self._st))

    @property
    def exchanges_done(self):
        return int(self._L.orc_exchanges_done(self._st))

    @property
    def n_records(self):
        return int(self._L.orc_n_records(self._st))

    def spins(self):
        out = np.empty((self.R, self.N), dtype=np.int8)
        self._L.orc_get_spins(self._st, _ptr(out))
        return out

    def couplings(self):
        out = np.empty((3, self.N), dtype=np.int8)
        self._L.orc_get_couplings(self._st, _ptr(out))
        return out

    def labels(self):
        out = np.empty(self.R, dtype=np.uint32)
        self._L.orc_get_labels(self._st, _ptr(out))
        return out

    def energy(self):
        E = np.empty(self.R, dtype=np.int64)
        M = np.empty(self.R, dtype=np.int64)
        self._L.orc_get_energy(self._st, _ptr(E), _ptr(M))
        return E, M

    def recount(self):
        E = np.empty(self.R, dtype=np.int64)
        M = np.empty(self.R, dtype=np.int64)
        self._L.orc_recount(self._st, _ptr(E), _ptr(M))
        return E, M

    def series(self):
        n = self.n_records
        E = np.empty((n, self.R), dtype=np.int32)
        M = np.empty((n, self.R), dtype=np.int32)
        if n:
            self._L.orc_get_series(self._st, _ptr(E), _ptr(M))
        return E, M

    def swaps(self):
        n = max(self.R - 1, 0)
        att = np.zeros(max(n, 1), dtype=np.uint64)
        acc = np.zeros(max(n, 1), dtype=np.uint64)
        self._L.orc_get_swaps(self._st, _ptr(att), _ptr(acc))
        return att[:n], acc[:n]


def bind(lib_path: str):
    """The oracle API bound to another compiled copy of oracle.c."""
    from types import SimpleNamespace

    class _Bound(Oracle):
        pass
    _Bound.lib_path = lib_path
    L = lib(lib_path)

    def _philox(ctr, key):
        c = np.ascontiguousarray(ctr, dtype=np.uint32)
        k = np.ascontiguousarray(key, dtype=np.uint32)
        out = np.zeros(4, dtype=np.uint32)
        L.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
        return out

    return SimpleNamespace(
        Oracle=_Bound, philox4x32_10=_philox, ISING2D=ISING2D, EA3D=EA3D,
        flip_accept=lambda b, dE, r: bool(L.orc_flip_accept(b, dE, r)),
        swap_accept=lambda bk, bk1, dE, r: bool(L.orc_swap_accept(bk, bk1, dE, r)))
