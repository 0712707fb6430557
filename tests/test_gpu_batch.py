"""Batched stepping: several independent networks advanced with one launch
per kernel must give, network by network, exactly their solo results."""
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


def _result(net, T):
    tt, ii = net.read_spikes(1, T + 1)
    syn = net.read_weights()
    v, u = net.read_state()
    return dict(tt=tt, ii=ii, v=v, u=u, **syn)


def _same(a, b):
    np.testing.assert_array_equal(a["tt"], b["tt"])
    np.testing.assert_array_equal(a["ii"], b["ii"])
    for k in ("w", "P", "D", "v", "u"):
        np.testing.assert_array_equal(a[k].view(np.uint32), b[k].view(np.uint32), err_msg=k)


MIX = [
    W.make_config(grid_x=2, grid_y=2, synapses_per_neuron=100, thalamic_rate=0.75, seed=2001,
                  weight_update_period=100),
    W.make_config(grid_x=3, grid_y=3, synapses_per_neuron=250, thalamic_rate=1.5, seed=2002,
                  weight_update_period=100),
    W.make_config(grid_x=2, grid_y=2, synapses_per_neuron=625, thalamic_rate=1.0, seed=2003,
                  weight_update_period=100),   # reaches the all-firing regime
    W.make_config(grid_x=4, grid_y=2, neurons_per_column=700, synapses_per_neuron=180,
                  thalamic_rate=2.0, seed=2004, weight_update_period=70),
    W.make_config(grid_x=1, grid_y=1, neurons_per_column=1500, synapses_per_neuron=300,
                  thalamic_rate=0.5, seed=2005, max_delay=12, weight_update_period=100),
]


def test_batch_members_equal_solo_runs(dp):
    T = 200
    pre = [0, 37, 0, 5, 120]  # steps run alone before joining the batch
    _say("batch of 5 uneven networks vs solo runs")
    solo = []
    for cfg in MIX:
        n = dp.Network(cfg)
        n.step(T)
        n.sync()
        solo.append(_result(n, T))
        n.close()
    nets = [dp.Network(cfg) for cfg in MIX]
    for n, k in zip(nets, pre):
        if k:
            n.step(k)
    # members advance together; each leaves the batch when it reaches T
    active = [(n, T - k) for n, k in zip(nets, pre)]
    while active:
        b = dp.Batch([n for n, _ in active])
        s = min(r for _, r in active)
        b.step(s)
        b.close()
        active = [(n, r - s) for n, r in active if r - s > 0]
    for cfg, n, ref in zip(MIX, nets, solo):
        assert n.t == T
        _same(_result(n, T), ref)
        n.close()
    assert (np.bincount(solo[2]["tt"], minlength=T + 1)[100:] == 5000).sum() >= 30


def test_batch_autotune_keeps_results(dp):
    cfgs = [MIX[0], MIX[1], MIX[3]]
    T = 120
    _say("batch autotune invariance")
    refs = []
    for cfg in cfgs:
        n = dp.Network(cfg)
        n.step(T)
        refs.append(_result(n, T))
        n.close()
    nets = [dp.Network(cfg) for cfg in cfgs]
    b = dp.Batch(nets)
    b.set_timing(True)
    b.autotune(steps_per_trial=5)     # 2 rounds x 6 candidates x 5 steps = 60 steps
    b.step(T - 60)
    st = b.stats()
    b.close()
    assert st["n_deliver"] > 0 and st["ms_deliver"] > 0
    for n, ref in zip(nets, refs):
        assert n.t == T
        _same(_result(n, T), ref)
        n.close()


def test_batch_rules(dp):
    a = dp.Network(MIX[0])
    o = dp.Network(W.tiny(sum_mode=W.SUM_ORDERED))
    try:
        with pytest.raises(dp.DpsnnError):
            dp.Batch([a, o])          # mixed summation modes
        b = dp.Batch([a])
        with pytest.raises(dp.DpsnnError):
            a.step(1)                 # stepped only through its batch
        with pytest.raises(dp.DpsnnError):
            dp.Batch([a])             # already in a batch
        b.step(3)
        b.close()
        a.step(2)
        assert a.t == 5
    finally:
        a.close()
        o.close()


def _events_from_raster(tt, ii, dly, M, T, dmax):
    """Deliveries implied by a raster: a spike stamped s reaches its delay-d
    synapses in step s + d - 1, which lies in steps 0 .. T-1 when d <= T - s."""
    d = dly.reshape(-1, M).astype(np.int64)
    cum = np.zeros((d.shape[0], dmax + 1), dtype=np.int64)
    for k in range(1, dmax + 1):
        cum[:, k] = (d <= k).sum(axis=1)
    lim = np.minimum(T - tt.astype(np.int64), dmax)
    ok = lim >= 1
    return int(cum[ii[ok].astype(np.int64), lim[ok]].sum())


def test_batch_atomic_mode(dp):
    # unordered fp32 atomics: not bit-reproducible, so the batch is checked
    # for exact delivery accounting against its own raster and for a mean
    # rate close to the fixed-point run of the same networks
    T = 300
    _say("batch of 5 networks, ATOMIC summation")
    nets = [dp.Network(dict(c, sum_mode=W.SUM_ATOMIC)) for c in MIX]
    b = dp.Batch(nets)
    b.step(T)
    b.close()
    for cfg, n in zip(MIX, nets):
        tt, ii = n.read_spikes(1, T + 1)
        _, dly = n.read_connectivity()
        st = n.stats()
        assert st["events"] == _events_from_raster(tt, ii, dly, cfg["synapses_per_neuron"], T,
                                                   cfg["max_delay"])
        ref = dp.Network(cfg)
        ref.step(T)
        ref.sync()
        rt, _ = ref.read_spikes(1, T + 1)
        ref.close()
        assert abs(len(tt) - len(rt)) <= 0.25 * len(rt) + 100, (len(tt), len(rt))
        n.close()
