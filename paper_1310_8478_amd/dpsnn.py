"""Python binding of libdpsnn.so: the C ABI of include/dpsnn.h with the same
names, argument marshalling only.  Every simulation step runs in the HIP
kernels of the library; PyTorch only supplies device memory (its caching
allocator) and the stream.

Raises RuntimeError on import of the library if libdpsnn.so has not been
built (python -m paper_1310_8478_amd.build); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdpsnn.so")

E_INVAL, E_NOMEM, E_DEVICE, E_RANGE, E_BUFSZ, E_TIMEOUT, E_CANCELED = -1, -2, -3, -4, -5, -6, -7
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3
SUM_ORDERED, SUM_ATOMIC, SUM_FIXED = 0, 1, 2


class DpsnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dpsnn error {code}: {msg}")
        self.code = code


class dpsnn_config(C.Structure):
    _fields_ = [
        ("grid_x", C.c_uint32), ("grid_y", C.c_uint32), ("neurons_per_column", C.c_uint32),
        ("exc_fraction", C.c_float), ("synapses_per_neuron", C.c_uint32),
        ("conn_mode", C.c_uint32), ("own_fraction", C.c_float), ("max_delay", C.c_uint32),
        ("w_exc_init", C.c_float), ("w_inh", C.c_float), ("w_max", C.c_float),
        ("a_plus", C.c_float), ("a_minus", C.c_float), ("tau_plus", C.c_float),
        ("tau_minus", C.c_float), ("weight_update_period", C.c_uint32),
        ("wu_bias", C.c_float), ("sd_decay", C.c_float), ("thalamic_rate", C.c_float),
        ("thalamic_current", C.c_float), ("seed", C.c_uint64), ("sum_mode", C.c_uint32),
        ("raster_steps", C.c_uint32),
    ]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class dpsnn_device(C.Structure):
    _fields_ = [("device", C.c_int), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("ctx", C.c_void_p)]


class dpsnn_stats(C.Structure):
    _fields_ = [
        ("steps", C.c_uint64), ("spikes", C.c_uint64), ("events", C.c_uint64),
        ("ltp_visits", C.c_uint64), ("consolidations", C.c_uint64), ("events_exc", C.c_uint64),
        ("ms_ltp", C.c_double), ("ms_deliver", C.c_double), ("ms_neuron", C.c_double),
        ("ms_wupdate", C.c_double),
        ("n_ltp", C.c_uint64), ("n_deliver", C.c_uint64), ("n_neuron", C.c_uint64),
        ("n_wupdate", C.c_uint64), ("graph_steps", C.c_uint64),
    ]


class dpsnn_job_info(C.Structure):
    _fields_ = [
        ("id", C.c_uint64), ("status", C.c_int32), ("error", C.c_int32), ("steps", C.c_uint32),
        ("steps_launched", C.c_uint32), ("footprint", C.c_uint64), ("t_submit", C.c_double),
        ("t_admit", C.c_double), ("t_built", C.c_double), ("t_done", C.c_double),
        ("net", C.c_void_p), ("message", C.c_char * 160),
    ]


class dpsnn_server_stats(C.Structure):
    _fields_ = [
        ("submitted", C.c_uint64), ("completed", C.c_uint64), ("failed", C.c_uint64),
        ("released", C.c_uint64), ("queued", C.c_uint64), ("running", C.c_uint64),
        ("quanta", C.c_uint64), ("set_steps", C.c_uint64), ("job_steps", C.c_uint64),
        ("budget_bytes", C.c_uint64), ("reserved_bytes", C.c_uint64),
        ("peak_reserved_bytes", C.c_uint64), ("peak_running", C.c_uint64),
    ]


EXPORTS = [
    "dpsnn_default_config", "dpsnn_footprint_bytes", "dpsnn_build_network", "dpsnn_step",
    "dpsnn_sync", "dpsnn_time", "dpsnn_read_spikes", "dpsnn_read_weights",
    "dpsnn_read_weights_noalloc",
    "dpsnn_read_connectivity", "dpsnn_read_state", "dpsnn_get_stats", "dpsnn_set_stimulus",
    "dpsnn_set_probes", "dpsnn_read_probes",
    "dpsnn_set_timing", "dpsnn_set_tuning", "dpsnn_autotune", "dpsnn_destroy",
    "dpsnn_get_config", "dpsnn_checkpoint_bytes", "dpsnn_save", "dpsnn_load",
    "dpsnn_batch_create", "dpsnn_batch_step", "dpsnn_batch_get_stats", "dpsnn_batch_set_timing",
    "dpsnn_batch_set_tuning", "dpsnn_batch_autotune", "dpsnn_batch_destroy",
    "dpsnn_server_create", "dpsnn_server_submit", "dpsnn_server_query", "dpsnn_server_wait",
    "dpsnn_server_wait_any", "dpsnn_server_cancel", "dpsnn_server_release", "dpsnn_server_get_stats", "dpsnn_server_clock",
    "dpsnn_server_destroy", "dpsnn_last_error",
]
_VOID = ("dpsnn_destroy", "dpsnn_batch_destroy", "dpsnn_server_destroy", "dpsnn_last_error")

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_1310_8478_amd.build`")
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.dpsnn_default_config.argtypes = [P(dpsnn_config)]
        L.dpsnn_footprint_bytes.argtypes = [P(dpsnn_config), P(C.c_uint64)]
        L.dpsnn_build_network.argtypes = [P(dpsnn_config), P(dpsnn_device), P(vp)]
        L.dpsnn_step.argtypes = [vp, C.c_uint32]
        L.dpsnn_sync.argtypes = [vp]
        L.dpsnn_time.argtypes = [vp, P(C.c_uint32)]
        L.dpsnn_read_spikes.argtypes = [vp, C.c_uint32, C.c_uint32, P(C.c_uint32), P(C.c_uint32),
                                        C.c_size_t, P(C.c_size_t)]
        L.dpsnn_read_weights.argtypes = [vp, C.c_uint64, C.c_uint64, P(C.c_float), P(C.c_float),
                                         P(C.c_float)]
        L.dpsnn_read_weights_noalloc.argtypes = [vp, C.c_uint64, C.c_uint64, P(C.c_float),
                                                 P(C.c_float), P(C.c_float)]
        L.dpsnn_read_connectivity.argtypes = [vp, C.c_uint64, C.c_uint64, P(C.c_uint32),
                                              P(C.c_uint8)]
        L.dpsnn_read_state.argtypes = [vp, P(C.c_float), P(C.c_float)]
        L.dpsnn_get_stats.argtypes = [vp, P(dpsnn_stats)]
        L.dpsnn_set_stimulus.argtypes = [vp, P(C.c_uint32), P(C.c_uint32), P(C.c_float), C.c_size_t]
        L.dpsnn_set_probes.argtypes = [vp, P(C.c_uint32), C.c_uint32]
        L.dpsnn_read_probes.argtypes = [vp, C.c_uint32, C.c_uint32, P(C.c_float), P(C.c_float)]
        L.dpsnn_set_timing.argtypes = [vp, C.c_int]
        L.dpsnn_set_tuning.argtypes = [vp, C.c_uint32, C.c_uint32]
        L.dpsnn_autotune.argtypes = [vp, C.c_uint32]
        L.dpsnn_destroy.argtypes = [vp]
        L.dpsnn_destroy.restype = None
        L.dpsnn_get_config.argtypes = [vp, P(dpsnn_config)]
        L.dpsnn_checkpoint_bytes.argtypes = [vp, P(C.c_uint64)]
        L.dpsnn_save.argtypes = [vp, vp, C.c_uint64]
        L.dpsnn_load.argtypes = [vp, C.c_uint64, P(dpsnn_device), P(vp)]
        L.dpsnn_batch_create.argtypes = [P(vp), C.c_uint32, P(vp)]
        L.dpsnn_batch_step.argtypes = [vp, C.c_uint32]
        L.dpsnn_batch_get_stats.argtypes = [vp, P(dpsnn_stats)]
        L.dpsnn_batch_set_timing.argtypes = [vp, C.c_int]
        L.dpsnn_batch_set_tuning.argtypes = [vp, C.c_uint32, C.c_uint32]
        L.dpsnn_batch_autotune.argtypes = [vp, C.c_uint32]
        L.dpsnn_batch_destroy.argtypes = [vp]
        L.dpsnn_batch_destroy.restype = None
        L.dpsnn_server_create.argtypes = [P(dpsnn_device), C.c_uint64, C.c_uint32, C.c_uint32,
                                          P(vp)]
        L.dpsnn_server_submit.argtypes = [vp, P(dpsnn_config), C.c_uint32, P(C.c_uint64)]
        L.dpsnn_server_query.argtypes = [vp, C.c_uint64, P(dpsnn_job_info)]
        L.dpsnn_server_wait.argtypes = [vp, C.c_uint64, C.c_double, P(dpsnn_job_info)]
        L.dpsnn_server_wait_any.argtypes = [vp, C.c_double, P(dpsnn_job_info)]
        L.dpsnn_server_cancel.argtypes = [vp, C.c_uint64]
        L.dpsnn_server_release.argtypes = [vp, C.c_uint64]
        L.dpsnn_server_get_stats.argtypes = [vp, P(dpsnn_server_stats)]
        L.dpsnn_server_clock.argtypes = [vp, P(C.c_double)]
        L.dpsnn_server_destroy.argtypes = [vp]
        L.dpsnn_server_destroy.restype = None
        L.dpsnn_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name not in _VOID:
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise DpsnnError(rc, lib().dpsnn_last_error().decode())


def to_config(cfg: dict) -> dpsnn_config:
    c = dpsnn_config()
    _check(lib().dpsnn_default_config(C.byref(c)))
    for name, _ in dpsnn_config._fields_:
        if name in cfg:
            setattr(c, name, cfg[name])
    return c


def footprint_bytes(cfg: dict) -> int:
    c = to_config(cfg)
    b = C.c_uint64()
    _check(lib().dpsnn_footprint_bytes(C.byref(c), C.byref(b)))
    return b.value


def _ptr(a, ct):
    return None if a is None else a.ctypes.data_as(C.POINTER(ct))


class _TorchAllocator:
    """Routes the library's device allocations through PyTorch's caching
    allocator on the given device."""

    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device

        def _alloc(nbytes, stream, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device,
                                                              stream=stream or 0))
            except Exception:  # allocation failure is reported to the library as NULL
                return None

        def _free(p, nbytes, stream, ctx):
            if p:
                torch.cuda.caching_allocator_delete(int(p))

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class Network:
    """One simulated network on one GPU (dpsnn_build_network .. dpsnn_destroy)."""

    def __init__(self, cfg: dict, device: int = 0, stream=None, torch_alloc: bool = True,
                 allocator=None):
        self.cfg = dict(cfg)
        self._c = to_config(cfg)
        dev = self._device(device, stream, torch_alloc, allocator)
        h = C.c_void_p()
        _check(lib().dpsnn_build_network(C.byref(self._c), C.byref(dev), C.byref(h)))
        self._adopt(h)

    def _device(self, device, stream, torch_alloc, allocator=None):
        """allocator: an object with ctypes `alloc` / `free` callbacks
        (ALLOC_FN, FREE_FN) serving every device allocation of the network;
        by default PyTorch's caching allocator (torch_alloc) or hipMalloc."""
        self._allocator = None
        dev = dpsnn_device()
        dev.device = device
        if stream is None:
            try:
                import torch
                torch.cuda.set_device(device)
                stream = torch.cuda.current_stream(device).cuda_stream
            except Exception:
                stream = 0
        dev.stream = stream or None
        if allocator is not None:
            self._allocator = allocator
        elif torch_alloc:
            self._allocator = _TorchAllocator(device)
        if self._allocator is not None:
            dev.alloc = self._allocator.alloc
            dev.free = self._allocator.free
        dev.ctx = None
        self._dev = dev
        return dev

    def _adopt(self, h):
        self.h = h
        self.Ncol = self._c.neurons_per_column
        self.N = self._c.grid_x * self._c.grid_y * self.Ncol
        self.M = self._c.synapses_per_neuron

    def save(self, path=None):
        """Checkpoint (dpsnn_save) as a uint8 array, also written to `path`
        if one is given."""
        n = C.c_uint64()
        _check(lib().dpsnn_checkpoint_bytes(self.h, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        _check(lib().dpsnn_save(self.h, buf.ctypes.data, n.value))
        if path is not None:
            buf.tofile(path)
        return buf

    @classmethod
    def load(cls, src, device: int = 0, stream=None, torch_alloc: bool = True, allocator=None):
        """A network restored from a checkpoint (a path or the bytes of one)."""
        if isinstance(src, (str, os.PathLike)):
            buf = np.fromfile(src, dtype=np.uint8)
        else:
            buf = np.ascontiguousarray(np.frombuffer(src, dtype=np.uint8))
        self = cls.__new__(cls)
        dev = self._device(device, stream, torch_alloc, allocator)
        h = C.c_void_p()
        _check(lib().dpsnn_load(buf.ctypes.data, buf.size, C.byref(dev), C.byref(h)))
        c = dpsnn_config()
        rc = lib().dpsnn_get_config(h, C.byref(c))
        if rc != 0:
            lib().dpsnn_destroy(h)
            _check(rc)
        self._c = c
        self.cfg = {name: getattr(c, name) for name, _ in dpsnn_config._fields_}
        self._adopt(h)
        return self

    @classmethod
    def _view(cls, handle: int, cfg: dict):
        """A Network object over a handle owned elsewhere (a server job);
        close() only forgets the handle."""
        self = cls.__new__(cls)
        self.cfg = dict(cfg)
        self._c = to_config(cfg)
        self._allocator = None
        self._owned = False
        self.h = C.c_void_p(handle)
        self.Ncol = self._c.neurons_per_column
        self.N = self._c.grid_x * self._c.grid_y * self.Ncol
        self.M = self._c.synapses_per_neuron
        return self

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owned", True):
                lib().dpsnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        _check(lib().dpsnn_step(self.h, n))

    def sync(self):
        _check(lib().dpsnn_sync(self.h))

    @property
    def t(self) -> int:
        x = C.c_uint32()
        _check(lib().dpsnn_time(self.h, C.byref(x)))
        return x.value

    def read_spikes(self, t_begin: int = 1, t_end: int | None = None):
        if t_end is None:
            t_end = self.t + 1
        n = C.c_size_t()
        rc = lib().dpsnn_read_spikes(self.h, t_begin, t_end, None, None, 0, C.byref(n))
        if rc not in (0, E_BUFSZ):
            _check(rc)
        times = np.zeros(n.value, dtype=np.uint32)
        ids = np.zeros(n.value, dtype=np.uint32)
        _check(lib().dpsnn_read_spikes(self.h, t_begin, t_end, _ptr(times, C.c_uint32),
                                       _ptr(ids, C.c_uint32), n.value, C.byref(n)))
        return times, ids

    def read_weights(self, first: int = 0, count: int | None = None, w=True, P=True, D=True,
                     noalloc: bool = False):
        """w, P, D of canonical synapses [first, first + count); noalloc uses
        dpsnn_read_weights_noalloc (the library's static workspace)."""
        if count is None:
            count = self.N * self.M - first
        out = {}
        arrs = {}
        for k, want in (("w", w), ("P", P), ("D", D)):
            arrs[k] = np.zeros(count, dtype=np.float32) if want else None
        fn = lib().dpsnn_read_weights_noalloc if noalloc else lib().dpsnn_read_weights
        _check(fn(self.h, first, count, _ptr(arrs["w"], C.c_float),
                  _ptr(arrs["P"], C.c_float), _ptr(arrs["D"], C.c_float)))
        for k, a in arrs.items():
            if a is not None:
                out[k] = a
        return out

    def read_connectivity(self, first: int = 0, count: int | None = None):
        if count is None:
            count = self.N * self.M - first
        tgt = np.zeros(count, dtype=np.uint32)
        dly = np.zeros(count, dtype=np.uint8)
        _check(lib().dpsnn_read_connectivity(self.h, first, count, _ptr(tgt, C.c_uint32),
                                             _ptr(dly, C.c_uint8)))
        return tgt, dly

    def read_state(self):
        v = np.zeros(self.N, dtype=np.float32)
        u = np.zeros(self.N, dtype=np.float32)
        _check(lib().dpsnn_read_state(self.h, _ptr(v, C.c_float), _ptr(u, C.c_float)))
        return v, u

    def stats(self) -> dict:
        s = dpsnn_stats()
        _check(lib().dpsnn_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in dpsnn_stats._fields_}

    def set_stimulus(self, t, ids, mv):
        t = np.ascontiguousarray(t, dtype=np.uint32)
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        mv = np.ascontiguousarray(mv, dtype=np.float32)
        _check(lib().dpsnn_set_stimulus(self.h, _ptr(t, C.c_uint32), _ptr(ids, C.c_uint32),
                                        _ptr(mv, C.c_float), len(t)))

    def set_probes(self, ids):
        """Record v and u of these neurons after every later step."""
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        _check(lib().dpsnn_set_probes(self.h, _ptr(ids, C.c_uint32), len(ids)))
        self._nprobe = len(ids)

    def read_probes(self, t_begin: int, t_end: int):
        """Probed (v, u) after steps t_begin .. t_end - 1, arrays of shape
        (t_end - t_begin, number of probes)."""
        n = getattr(self, "_nprobe", 0)
        v = np.zeros((t_end - t_begin, n), dtype=np.float32)
        u = np.zeros((t_end - t_begin, n), dtype=np.float32)
        _check(lib().dpsnn_read_probes(self.h, t_begin, t_end, _ptr(v, C.c_float), _ptr(u, C.c_float)))
        return v, u

    def set_timing(self, enable: bool = True):
        _check(lib().dpsnn_set_timing(self.h, int(bool(enable))))

    def set_tuning(self, key: int, value: int):
        _check(lib().dpsnn_set_tuning(self.h, key, value))

    def autotune(self, steps_per_trial: int = 5):
        _check(lib().dpsnn_autotune(self.h, steps_per_trial))


class Batch:
    """Several networks advanced together with one launch per kernel
    (dpsnn_batch_create .. dpsnn_batch_destroy).  The networks stay owned by
    their Network objects; close the batch before closing them."""

    def __init__(self, nets):
        self.nets = list(nets)
        arr = (C.c_void_p * len(self.nets))(*[n.h.value for n in self.nets])
        h = C.c_void_p()
        _check(lib().dpsnn_batch_create(arr, len(self.nets), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().dpsnn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        _check(lib().dpsnn_batch_step(self.h, n))

    def stats(self) -> dict:
        s = dpsnn_stats()
        _check(lib().dpsnn_batch_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in dpsnn_stats._fields_}

    def set_timing(self, enable: bool = True):
        _check(lib().dpsnn_batch_set_timing(self.h, int(bool(enable))))

    def set_tuning(self, key: int, value: int):
        _check(lib().dpsnn_batch_set_tuning(self.h, key, value))

    def autotune(self, steps_per_trial: int = 5):
        _check(lib().dpsnn_batch_autotune(self.h, steps_per_trial))


def _info(x: dpsnn_job_info) -> dict:
    return dict(id=x.id, status=x.status, error=x.error, steps=x.steps,
                steps_launched=x.steps_launched, footprint=x.footprint, t_submit=x.t_submit,
                t_admit=x.t_admit, t_built=x.t_built, t_done=x.t_done, net=x.net,
                message=x.message.decode(errors="replace"))


class Server:
    """Continuous-batching job server (dpsnn_server_create .. _destroy): jobs
    are admitted by device footprint against `budget_bytes`, generated on the
    server's build stream and stepped together; a finished job's network stays
    readable through job_network() until release()."""

    def __init__(self, device: int = 0, budget_bytes: int = 0, max_quantum: int = 0,
                 max_jobs: int = 0, torch_alloc: bool = True):
        self._allocator = None
        dev = dpsnn_device()
        dev.device = device
        dev.stream = None
        if torch_alloc:
            import torch
            torch.cuda.set_device(device)
            self._allocator = _TorchAllocator(device)
            dev.alloc = self._allocator.alloc
            dev.free = self._allocator.free
        dev.ctx = None
        self._dev = dev
        self._cfgs = {}
        h = C.c_void_p()
        _check(lib().dpsnn_server_create(C.byref(dev), budget_bytes, max_quantum, max_jobs,
                                         C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().dpsnn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, cfg: dict, steps: int) -> int:
        c = to_config(cfg)
        j = C.c_uint64()
        _check(lib().dpsnn_server_submit(self.h, C.byref(c), steps, C.byref(j)))
        self._cfgs[j.value] = dict(cfg)
        return j.value

    def query(self, job: int) -> dict:
        x = dpsnn_job_info()
        _check(lib().dpsnn_server_query(self.h, job, C.byref(x)))
        return _info(x)

    def wait(self, job: int, timeout: float | None = None) -> dict:
        x = dpsnn_job_info()
        _check(lib().dpsnn_server_wait(self.h, job, -1.0 if timeout is None else timeout,
                                       C.byref(x)))
        return _info(x)

    def wait_any(self, timeout: float | None = None):
        """The next finished job's info, or None if none finished in time."""
        x = dpsnn_job_info()
        rc = lib().dpsnn_server_wait_any(self.h, -1.0 if timeout is None else timeout,
                                         C.byref(x))
        if rc == E_TIMEOUT:
            return None
        _check(rc)
        return _info(x)

    def job_network(self, job: int) -> Network:
        """Read access to a DONE job's network (owned by the server)."""
        info = self.query(job)
        if info["status"] != JOB_DONE or not info["net"]:
            raise DpsnnError(E_INVAL, f"job {job} is not done")
        return Network._view(info["net"], self._cfgs[job])

    def cancel(self, job: int):
        """Ask the server to stop a queued or running job (it becomes FAILED
        with E_CANCELED at the next quantum boundary)."""
        _check(lib().dpsnn_server_cancel(self.h, job))

    def release(self, job: int):
        _check(lib().dpsnn_server_release(self.h, job))
        self._cfgs.pop(job, None)

    def stats(self) -> dict:
        s = dpsnn_server_stats()
        _check(lib().dpsnn_server_get_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in dpsnn_server_stats._fields_}

    def clock(self) -> float:
        x = C.c_double()
        _check(lib().dpsnn_server_clock(self.h, C.byref(x)))
        return x.value
