"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/dpsnn.h, and validates configurations
before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_1310_8478_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "dpsnn.h")).read()
    return sorted(set(re.findall(r"\b(dpsnn_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def dp():
    from paper_1310_8478_amd import dpsnn
    if not os.path.exists(dpsnn._LIB_PATH):
        pytest.skip("libdpsnn.so not built")
    dpsnn.lib()
    return dpsnn


def test_every_declared_symbol_is_exported(dp):
    names = _declared()
    assert len(names) >= 15
    L = C.CDLL(dp._LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dp.EXPORTS)


def test_default_config_and_footprint(dp):
    b_tiny = dp.footprint_bytes(W.tiny())
    b_mid = dp.footprint_bytes(W.mid())
    b_large = dp.footprint_bytes(W.large())
    assert 5e6 < b_tiny < 5e8
    assert 2e9 < b_mid < 1e10
    # 3.2 G synapses: forward (2 + 4 + 4 B), reverse (4 + 4 + 4 B) and
    # forward-to-reverse (4 B) tables
    assert 6e10 < b_large < 8e10
    assert b_large < 288e9


@pytest.mark.parametrize("field,value", [
    ("grid_x", 0), ("neurons_per_column", 1), ("synapses_per_neuron", 0),
    ("max_delay", 0), ("max_delay", 32), ("exc_fraction", 0.0), ("conn_mode", 2),
    ("thalamic_rate", 1024.0), ("thalamic_rate", -1.0), ("tau_plus", 0.0),
    ("w_max", float("nan")), ("sum_mode", 3), ("raster_steps", 5),
])
def test_invalid_configs_rejected(dp, field, value):
    cfg = W.tiny(**{field: value})
    with pytest.raises(dp.DpsnnError) as ei:
        dp.footprint_bytes(cfg)
    assert ei.value.code == dp.E_INVAL
    assert dp.lib().dpsnn_last_error().decode()


def test_size_limits(dp):
    # 64-bit positions: the paper's largest grid (256x128 columns, 6.55 G
    # synapses) is valid and fits one 288 GB device
    big = W.paper_table1(8)
    fp = dp.footprint_bytes(big)
    assert 1.4e11 < fp < 1.8e11
    # ... but not in ORDERED mode (32-bit event slots)
    with pytest.raises(dp.DpsnnError):
        dp.footprint_bytes(dict(big, sum_mode=W.SUM_ORDERED))
    # 2^36 synapses
    with pytest.raises(dp.DpsnnError):
        dp.footprint_bytes(W.make_config(grid_x=256, grid_y=256, neurons_per_column=1000,
                                         synapses_per_neuron=1100))
    # one column's reach (13 x Ncol x M) must stay below 2^31
    with pytest.raises(dp.DpsnnError):
        dp.footprint_bytes(W.make_config(grid_x=1, grid_y=1, neurons_per_column=65535,
                                         synapses_per_neuron=2600))
    # 2^26 neurons is the id limit
    with pytest.raises(dp.DpsnnError):
        dp.footprint_bytes(W.make_config(grid_x=256, grid_y=256, neurons_per_column=1100,
                                         synapses_per_neuron=1))


def test_server_argument_checks(dp):
    # argument checks come before any device work
    L = dp.lib()
    h = C.c_void_p()
    assert L.dpsnn_server_create(None, 0, 0, 0, C.byref(h)) == dp.E_INVAL
    dev = dp.dpsnn_device()
    dev.device = -1
    assert L.dpsnn_server_create(C.byref(dev), 0, 0, 0, C.byref(h)) == dp.E_INVAL
    assert not h.value
    cfg = dp.to_config(W.tiny())
    j = C.c_uint64()
    assert L.dpsnn_server_submit(None, C.byref(cfg), 10, C.byref(j)) == dp.E_INVAL
    info = dp.dpsnn_job_info()
    assert L.dpsnn_server_wait_any(None, 0.0, C.byref(info)) == dp.E_INVAL
    assert L.dpsnn_server_wait(None, 1, 0.0, C.byref(info)) == dp.E_INVAL
    assert L.dpsnn_server_release(None, 1) == dp.E_INVAL
    assert L.dpsnn_server_cancel(None, 1) == dp.E_INVAL
    assert L.dpsnn_server_query(None, 1, C.byref(info)) == dp.E_INVAL
    L.dpsnn_server_destroy(None)
    assert C.sizeof(dp.dpsnn_job_info) == 8 + 4 + 4 + 4 + 4 + 8 + 4 * 8 + 8 + 160


def test_checkpoint_header_checks(dp):
    # rejected before any device work: too short, wrong magic, wrong version
    import ctypes as C
    h = C.c_void_p()
    dev = dp.dpsnn_device()
    for buf in (b"", b"DPSNNCK1", b"X" * 4096):
        arr = (C.c_uint8 * max(1, len(buf))).from_buffer_copy(buf or b"\0")
        rc = dp.lib().dpsnn_load(C.cast(arr, C.c_void_p), len(buf), C.byref(dev), C.byref(h))
        assert rc == dp.E_INVAL, buf[:8]
        assert not h.value
    good = bytearray(b"DPSNNCK1" + b"\0" * 4088)
    good[8] = 99  # version 99
    arr = (C.c_uint8 * len(good)).from_buffer(good)
    assert dp.lib().dpsnn_load(C.cast(arr, C.c_void_p), len(good), C.byref(dev), C.byref(h)) == dp.E_INVAL
    assert "version" in dp.lib().dpsnn_last_error().decode()


def _checkpoint_image(dp, cfg, R, extra=0):
    """A checkpoint of `cfg` with zero state, laid out as dpsnn_save writes it
    (header, then each array padded to 16 bytes); returns (buffer, offset of
    the raster ring, raster words per column)."""
    import struct
    c = dp.to_config(dict(cfg, raster_steps=R))
    Ncol = cfg["neurons_per_column"]
    C_ = cfg["grid_x"] * cfg["grid_y"]
    N, W_ = C_ * Ncol, (Ncol + 63) // 64
    S = N * cfg["synapses_per_neuron"]
    pad = lambda x: (x + 15) & ~15
    head = 16 + C.sizeof(c) + 32
    sizes = [4 * N, 4 * N, 8 * N, 4 * N, 8 * R * C_ * W_, 32 * 64, 4 * S, 4 * S, 4 * S, 0, 0, 0]
    total = pad(head) + sum(pad(b) for b in sizes) + extra
    buf = bytearray(total)
    buf[0:8] = b"DPSNNCK1"
    buf[8:16] = struct.pack("<II", 1, head)
    buf[16:16 + C.sizeof(c)] = bytes(c)
    buf[16 + C.sizeof(c):head] = struct.pack("<QQQQ", 5, 0, 0, total)
    ring = pad(head) + sum(pad(b) for b in sizes[:4])
    return buf, ring, W_


def _load(dp, buf):
    h = C.c_void_p()
    dev = dp.dpsnn_device()
    arr = (C.c_uint8 * len(buf)).from_buffer(buf)
    rc = dp.lib().dpsnn_load(C.cast(arr, C.c_void_p), len(buf), C.byref(dev), C.byref(h))
    if rc == 0:                     # loaded (a device is present): no error message
        dp.lib().dpsnn_destroy(h)
        return rc, ""
    return rc, dp.lib().dpsnn_last_error().decode()


def test_checkpoint_contents_checked_on_host(dp):
    # ragged 65-neuron columns: the last raster word of a column has one valid bit
    cfg = W.make_config(grid_x=2, grid_y=1, neurons_per_column=65, synapses_per_neuron=3)
    R = 24
    buf, ring, W_ = _checkpoint_image(dp, cfg, R)
    rc, msg = _load(dp, buf)
    assert "raster" not in msg and "size" not in msg, msg   # passes the host checks
    # a spike bit beyond the column's last neuron, in any slot or column
    for slot, col, bit in ((0, 0, 1), (R - 1, 1, 63), (7, 1, 5)):
        bad = bytearray(buf)
        pos = ring + ((slot * 2 + col) * W_ + W_ - 1) * 8
        bad[pos:pos + 8] = (1 << bit).to_bytes(8, "little")
        rc, msg = _load(dp, bad)
        assert rc == dp.E_INVAL and "raster" in msg, (slot, col, bit, rc, msg)
    # the valid bit of the last word is accepted by the host checks
    ok = bytearray(buf)
    pos = ring + (W_ - 1) * 8
    ok[pos:pos + 8] = (1).to_bytes(8, "little")
    rc, msg = _load(dp, ok)
    assert "raster" not in msg, msg
    # a total that disagrees with the configuration's array sizes
    big, _, _ = _checkpoint_image(dp, cfg, R, extra=16)
    rc, msg = _load(dp, big)
    assert rc == dp.E_INVAL and "size" in msg, msg


def test_device_allocations_only_in_the_allocator_helpers():
    # every device allocation of the library goes through the network's (or
    # server's) allocator: the only direct runtime allocations are the
    # fallbacks of the helpers used when no callbacks are given
    import re
    csrc = os.path.join(ROOT, "paper_1310_8478_amd", "csrc")
    found = {}
    for fn in sorted(os.listdir(csrc)):
        txt = open(os.path.join(csrc, fn)).read()
        for m in re.finditer(r"\bhip(Malloc|MallocAsync|MallocManaged|ExtMallocWithFlags|HostMalloc)\s*\(", txt):
            # the function the call sits in: the last line that opens a
            # top-level definition before it
            head = txt[:m.start()]
            fdef = re.findall(r"^[A-Za-z].*?\b([A-Za-z_][A-Za-z_0-9]*)\s*\([^;]*$", head, re.M)
            found.setdefault(fn, []).append((m.group(0).split("(")[0], fdef[-1] if fdef else None))
    assert found.get("api.cpp") == [("hipMalloc", "dalloc"), ("hipMalloc", "dev_alloc"),
                                    ("hipHostMalloc", "make_launch_set")], found
    assert found.get("serve.cpp") == [("hipMallocAsync", "ordered_alloc")], found
    assert set(found) == {"api.cpp", "serve.cpp"}, found
