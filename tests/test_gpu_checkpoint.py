"""Checkpoints (dpsnn_save / dpsnn_load): a network saved after T1 steps,
loaded (connectivity regenerated from the seed) and stepped to T must equal,
bit for bit, the same network stepped to T without interruption: raster,
w, P, D, v, u and counters, in both reproducible summation modes, across
consolidations, with a stimulus list, through a file, inside a batch, and on
the full-size mid workload."""
import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1310_8478_amd import dpsnn
    dpsnn.lib()
    return dpsnn


def _snap(net, t0=1):
    tt, ii = net.read_spikes(t0, net.t + 1)
    syn = net.read_weights()
    v, u = net.read_state()
    st = net.stats()
    return dict(tt=tt, ii=ii, v=v, u=u, w=syn["w"], P=syn["P"], D=syn["D"],
                counts=(st["steps"], st["spikes"], st["events"], st["ltp_visits"],
                        st["consolidations"], st["events_exc"]))


def _same(a, b, what):
    np.testing.assert_array_equal(a["tt"], b["tt"], err_msg=what)
    np.testing.assert_array_equal(a["ii"], b["ii"], err_msg=what)
    for k in ("w", "P", "D", "v", "u"):
        np.testing.assert_array_equal(a[k].view(np.uint32), b[k].view(np.uint32),
                                      err_msg=f"{what}: {k}")
    assert a["counts"] == b["counts"], what


def _cfg(mode):
    return W.make_config(grid_x=3, grid_y=2, neurons_per_column=400, synapses_per_neuron=90,
                         thalamic_rate=2.0, w_exc_init=8.0, weight_update_period=70,
                         raster_steps=400, sum_mode=mode, seed=9101)


def _stim(N):
    return W.stimulus_list(N, 300, 200, seed=12)


@pytest.mark.parametrize("mode", [W.SUM_FIXED, W.SUM_ORDERED])
def test_save_load_continues_bit_exact(dp, orc, mode):
    cfg = _cfg(mode)
    T, T1 = 300, 137
    _say(f"checkpoint at step {T1} of {T}, mode {mode}")
    ref = dp.Network(cfg)
    ref.set_stimulus(*_stim(ref.N))
    ref.step(T)
    ref.sync()
    want = _snap(ref)
    ref.close()
    a = dp.Network(cfg)
    a.set_stimulus(*_stim(a.N))
    a.step(T1)
    buf = a.save()
    a.step(T - T1)                      # the saved network itself goes on unchanged
    _same(_snap(a), want, "saved network")
    a.close()
    b = dp.Network.load(buf)
    assert b.t == T1 and b.cfg["sum_mode"] == mode
    b.step(T - T1)
    got = _snap(b)
    _same(got, want, "loaded network")
    b.close()
    if mode == W.SUM_FIXED:
        o = orc.Net(cfg, T)
        o.set_stimulus(*_stim(a.N))
        o.run(T)
        ot, oi = o.raster()
        s = o.synapses()
        o.close()
        np.testing.assert_array_equal(got["tt"], ot)
        np.testing.assert_array_equal(got["ii"], oi)
        np.testing.assert_array_equal(got["w"].view(np.uint32), s["w"].view(np.uint32))


def test_checkpoint_file_into_a_batch(dp, tmp_path):
    cfg = _cfg(W.SUM_FIXED)
    other = W.make_config(grid_x=2, grid_y=2, synapses_per_neuron=60, seed=9102,
                          weight_update_period=50)
    _say("checkpoint file, resumed inside a batch")
    ref = dp.Network(cfg)
    ref.step(260)
    ref.sync()
    want = _snap(ref)
    ref.close()
    a = dp.Network(cfg)
    a.step(100)
    path = tmp_path / "net.ckpt"
    a.save(str(path))
    a.close()
    b = dp.Network.load(str(path))
    c = dp.Network(other)
    c.step(100)
    batch = dp.Batch([b, c])
    batch.step(160)
    batch.close()
    _same(_snap(b), want, "loaded network stepped in a batch")
    b.close()
    c.close()


def test_checkpoint_errors(dp):
    _say("checkpoint errors")
    net = dp.Network(_cfg(W.SUM_FIXED))
    try:
        net.step(20)
        buf = net.save()
        small = np.empty(buf.size - 1, dtype=np.uint8)
        rc = dp.lib().dpsnn_save(net.h, small.ctypes.data, small.size)
        assert rc == dp.E_BUFSZ
        with pytest.raises(dp.DpsnnError) as e:
            dp.Network.load(buf[:-16])
        assert e.value.code == dp.E_INVAL
        bad = buf.copy()
        bad[16:20] = np.frombuffer(np.uint32(7).tobytes(), np.uint8)   # grid_x in the header
        with pytest.raises(dp.DpsnnError) as e:
            dp.Network.load(bad)
        assert e.value.code == dp.E_INVAL
        # the device stays usable and a good checkpoint still loads
        ok = dp.Network.load(buf)
        assert ok.t == 20
        ok.close()
    finally:
        net.close()


def test_checkpoint_mid_full_size(dp):
    cfg = W.mid(weight_update_period=120)
    _say("mid full size: checkpoint at step 90 of 200")
    ref = dp.Network(cfg)
    ref.step(200)
    ref.sync()
    want_t, want_i = ref.read_spikes(101, 201)
    wv, wu = ref.read_state()
    wst = ref.stats()
    ref.close()
    a = dp.Network(cfg)
    a.step(90)
    buf = a.save()
    a.close()
    b = dp.Network.load(buf)
    b.step(110)
    b.sync()
    gt, gi = b.read_spikes(101, 201)
    gv, gu = b.read_state()
    gst = b.stats()
    b.close()
    np.testing.assert_array_equal(gt, want_t)
    np.testing.assert_array_equal(gi, want_i)
    np.testing.assert_array_equal(gv.view(np.uint32), wv.view(np.uint32))
    np.testing.assert_array_equal(gu.view(np.uint32), wu.view(np.uint32))
    for k in ("spikes", "events", "ltp_visits", "consolidations", "events_exc"):
        assert gst[k] == wst[k], k
