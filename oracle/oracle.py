"""ctypes front end of the reference CPU simulator in oracle.c.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline leg of bench.py.  The product library never imports this module.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.environ.get("DPSNN_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcConfig(C.Structure):
    _fields_ = [
        ("grid_x", C.c_uint32), ("grid_y", C.c_uint32), ("neurons_per_column", C.c_uint32),
        ("exc_fraction", C.c_float), ("synapses_per_neuron", C.c_uint32),
        ("conn_mode", C.c_uint32), ("own_fraction", C.c_float), ("max_delay", C.c_uint32),
        ("w_exc_init", C.c_float), ("w_inh", C.c_float), ("w_max", C.c_float),
        ("a_plus", C.c_float), ("a_minus", C.c_float), ("tau_plus", C.c_float),
        ("tau_minus", C.c_float), ("weight_update_period", C.c_uint32),
        ("wu_bias", C.c_float), ("sd_decay", C.c_float), ("thalamic_rate", C.c_float),
        ("thalamic_current", C.c_float), ("seed", C.c_uint64), ("sum_mode", C.c_uint32),
    ]


def to_cfg(d: dict) -> OrcConfig:
    c = OrcConfig()
    for name, _ in OrcConfig._fields_:
        setattr(c, name, d[name])
    return c


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        L.orc_philox.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_synapse.argtypes = [P(OrcConfig), C.c_uint32, C.c_uint32, P(C.c_uint32),
                                  P(C.c_uint32), P(C.c_float)]
        L.orc_thalamic.argtypes = [P(OrcConfig), C.c_uint32, C.c_uint32, P(C.c_uint32), C.c_uint32]
        L.orc_thalamic.restype = C.c_uint32
        L.orc_tp.argtypes = [P(OrcConfig), C.c_uint32]
        L.orc_tp.restype = C.c_float
        L.orc_tm.argtypes = [P(OrcConfig), C.c_uint32]
        L.orc_tm.restype = C.c_float
        L.orc_neuron_step.argtypes = [P(C.c_float), P(C.c_float)] + [C.c_float] * 5
        L.orc_neuron_step.restype = C.c_int
        L.orc_single_neuron.argtypes = [C.c_int, C.c_float, C.c_uint32, P(C.c_uint32), C.c_uint32,
                                        P(C.c_float), P(C.c_float)]
        L.orc_single_neuron.restype = C.c_uint32
        L.orc_create.argtypes = [P(OrcConfig), C.c_uint32]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_stimulus.argtypes = [C.c_void_p, P(C.c_uint32), P(C.c_uint32), P(C.c_float),
                                       C.c_uint64]
        L.orc_set_stimulus.restype = C.c_int
        L.orc_run.argtypes = [C.c_void_p, C.c_uint32]
        L.orc_run.restype = C.c_int
        L.orc_time.argtypes = [C.c_void_p]
        L.orc_time.restype = C.c_uint32
        L.orc_raster_count.argtypes = [C.c_void_p]
        L.orc_raster_count.restype = C.c_uint64
        L.orc_get_raster.argtypes = [C.c_void_p, P(C.c_uint32), P(C.c_uint32)]
        L.orc_get_synapses.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, P(C.c_uint32),
                                       P(C.c_uint8), P(C.c_float), P(C.c_float), P(C.c_float)]
        L.orc_get_state.argtypes = [C.c_void_p, P(C.c_float), P(C.c_float)]
        L.orc_get_counters.argtypes = [C.c_void_p, P(C.c_uint64)]
        L.orc_num_neurons.argtypes = [C.c_void_p]
        L.orc_num_neurons.restype = C.c_uint32
        L.orc_exc_per_column.argtypes = [P(OrcConfig)]
        L.orc_exc_per_column.restype = C.c_uint32
        L.orc_paper_blocks.argtypes = [C.c_uint32, P(C.c_uint32)]
        L.orc_q32.argtypes = [C.c_float]
        L.orc_q32.restype = C.c_int64
        L.orc_dq32.argtypes = [C.c_int64]
        L.orc_dq32.restype = C.c_float
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return tuple(o)


def synapse(cfg: dict, i: int, j: int):
    cc = to_cfg(cfg)
    t, d, w = C.c_uint32(), C.c_uint32(), C.c_float()
    lib().orc_synapse(C.byref(cc), i, j, C.byref(t), C.byref(d), C.byref(w))
    return t.value, d.value, w.value


def thalamic(cfg: dict, c: int, t: int):
    cc = to_cfg(cfg)
    buf = (C.c_uint32 * 1024)()
    n = lib().orc_thalamic(C.byref(cc), c, t, buf, 1024)
    return [buf[k] for k in range(min(n, 1024))]


def tp(cfg: dict, delta: int) -> float:
    cc = to_cfg(cfg)
    return lib().orc_tp(C.byref(cc), delta)


def tm(cfg: dict, delta: int) -> float:
    cc = to_cfg(cfg)
    return lib().orc_tm(C.byref(cc), delta)


def exc_per_column(cfg: dict) -> int:
    cc = to_cfg(cfg)
    return lib().orc_exc_per_column(C.byref(cc))


def paper_blocks(M: int):
    o = (C.c_uint32 * 13)()
    lib().orc_paper_blocks(M, o)
    return list(o)


def q32(x: float) -> int:
    return lib().orc_q32(x)


def dq32(a: int) -> float:
    return lib().orc_dq32(a)


def single_neuron(fs: bool, I: float, T: int, cap: int = 100000):
    buf = np.zeros(cap, dtype=np.uint32)
    v, u = C.c_float(), C.c_float()
    n = lib().orc_single_neuron(int(fs), I, T, _p(buf, C.c_uint32), cap, C.byref(v), C.byref(u))
    return buf[:min(n, cap)].copy(), v.value, u.value


def neuron_step(v: float, u: float, I: float, a: float, b: float, c: float, d: float):
    vv, uu = C.c_float(v), C.c_float(u)
    f = lib().orc_neuron_step(C.byref(vv), C.byref(uu), I, a, b, c, d)
    return vv.value, uu.value, bool(f)


class Net:
    """One oracle network; run() advances it by whole 1 ms steps."""

    def __init__(self, cfg: dict, t_cap: int):
        self.cfg = dict(cfg)
        self._cc = to_cfg(cfg)
        self.h = lib().orc_create(C.byref(self._cc), t_cap)
        if not self.h:
            raise MemoryError("oracle network allocation failed")
        self.N = lib().orc_num_neurons(self.h)
        self.M = cfg["synapses_per_neuron"]

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_stimulus(self, t, ids, mv):
        t = np.ascontiguousarray(t, dtype=np.uint32)
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        mv = np.ascontiguousarray(mv, dtype=np.float32)
        rc = lib().orc_set_stimulus(self.h, _p(t, C.c_uint32), _p(ids, C.c_uint32),
                                    _p(mv, C.c_float), len(t))
        if rc != 0:
            raise ValueError(f"orc_set_stimulus failed: {rc}")

    def run(self, n: int):
        rc = lib().orc_run(self.h, n)
        if rc != 0:
            raise RuntimeError(f"orc_run failed: {rc}")

    @property
    def t(self) -> int:
        return lib().orc_time(self.h)

    def raster(self):
        n = lib().orc_raster_count(self.h)
        tt = np.zeros(n, dtype=np.uint32)
        ii = np.zeros(n, dtype=np.uint32)
        if n:
            lib().orc_get_raster(self.h, _p(tt, C.c_uint32), _p(ii, C.c_uint32))
        return tt, ii

    def synapses(self, first: int = 0, count: int | None = None):
        if count is None:
            count = self.N * self.M - first
        tgt = np.zeros(count, dtype=np.uint32)
        dly = np.zeros(count, dtype=np.uint8)
        w = np.zeros(count, dtype=np.float32)
        P = np.zeros(count, dtype=np.float32)
        D = np.zeros(count, dtype=np.float32)
        lib().orc_get_synapses(self.h, first, count, _p(tgt, C.c_uint32), _p(dly, C.c_uint8),
                               _p(w, C.c_float), _p(P, C.c_float), _p(D, C.c_float))
        return dict(tgt=tgt, dly=dly, w=w, P=P, D=D)

    def state(self):
        v = np.zeros(self.N, dtype=np.float32)
        u = np.zeros(self.N, dtype=np.float32)
        lib().orc_get_state(self.h, _p(v, C.c_float), _p(u, C.c_float))
        return v, u

    def counters(self) -> dict:
        o = (C.c_uint64 * 6)()
        lib().orc_get_counters(self.h, o)
        keys = ("events", "ltp_visits", "ltp_updates", "ltd_updates", "spikes", "thalamic")
        return {k: int(o[i]) for i, k in enumerate(keys)}
