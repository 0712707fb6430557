"""The large workload at full size (64x64 columns x 1250 neurons, M = 625,
3.2 G synapses) in ORDERED summation, the mode that addresses synapses and
event slots with 32-bit offsets (at most 2^32 - 1 synapses): forward
positions here run past 2^31.  Checked on sampled neurons of one step in the
rising-rate regime (steps 30 and 40): the input current is rebuilt from the
network's own connectivity, weights and raster and summed in fp32 in the
canonical order (the thalamic picks first, then by delay, source id and
synapse index j), and the oracle's neuron update must then give the GPU's v,
u and spike bit for bit (Sec. 2 loop items 2.3-2.7)."""
import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W
from test_gpu_fullsize import FS, RS, _window_columns

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


def _check_one_step_ordered(net, orc, cols, per_col, seed):
    """Step net once; check sampled neurons of `cols` against the oracle with
    the canonical-order fp32 current.  Returns the number of deliveries summed."""
    cfg = net.cfg
    M, Ncol, Dmax = cfg["synapses_per_neuron"], cfg["neurons_per_column"], cfg["max_delay"]
    Ne = int(round(cfg["exc_fraction"] * Ncol))
    T1 = net.t
    v0, u0 = net.read_state()
    tt, ii = net.read_spikes(T1 - Dmax + 1, T1 + 1)
    spiked = np.zeros((Dmax, net.N), dtype=bool)     # row d-1: stamp T1 - d + 1
    spiked[(T1 - tt.astype(np.int64)), ii] = True
    net.step(1)
    net.sync()
    v1, u1 = net.read_state()
    t2, i2 = net.read_spikes(T1 + 1, T1 + 2)
    fired = np.zeros(net.N, dtype=bool)
    fired[i2] = True
    rng = np.random.default_rng(seed)
    summed = 0
    for ck in cols:
        sample = ck * Ncol + np.sort(rng.choice(Ncol, size=per_col, replace=False))
        contrib = {int(k): [] for k in sample}
        for cs in _window_columns(cfg, ck):
            first = cs * Ncol * M
            tg, dl = net.read_connectivity(first, Ncol * M)
            hit = np.isin(tg, sample)
            if not hit.any():
                continue
            pos = np.nonzero(hit)[0]
            src = cs * Ncol + pos // M
            dly = dl[pos].astype(np.int64)
            live = spiked[dly - 1, src]
            w = net.read_weights(first, Ncol * M, P=False, D=False)["w"]
            for p, k, on, s, d in zip(pos.tolist(), tg[pos].tolist(), live.tolist(),
                                      src.tolist(), dly.tolist()):
                if on:
                    contrib[k].append((d, s, p % M, np.float32(w[p])))
        picks = orc.thalamic(cfg, ck, T1)
        thal = np.float32(cfg["thalamic_current"])
        for k in sample.tolist():
            acc = np.float32(0.0)
            for l in picks:
                if ck * Ncol + l == k:
                    acc = np.float32(acc + thal)
            for _, _, _, wv in sorted(contrib[k], key=lambda e: e[:3]):
                acc = np.float32(acc + wv)
            summed += len(contrib[k])
            a, b, c, d = RS if (k % Ncol) < Ne else FS
            v, u, f = orc.neuron_step(float(v0[k]), float(u0[k]), float(acc), a, b, c, d)
            assert np.float32(v).view(np.uint32) == v1[k].view(np.uint32), (T1, k, v, v1[k])
            assert np.float32(u).view(np.uint32) == u1[k].view(np.uint32), (T1, k, u, u1[k])
            assert f == bool(fired[k]), (T1, k)
    return summed


def test_large_ordered_sampled_steps(dp, orc):
    cfg = W.large(sum_mode=W.SUM_ORDERED)
    S = cfg["grid_x"] * cfg["grid_y"] * cfg["neurons_per_column"] * cfg["synapses_per_neuron"]
    assert 2 ** 31 < S < 2 ** 32
    _say("large, ORDERED: building 3.2 G synapses")
    net = dp.Network(cfg)
    try:
        net.step(30)
        net.sync()
        _say("large, ORDERED: step 30, sampled neurons of 2 columns")
        n1 = _check_one_step_ordered(net, orc, cols=[0, 2081], per_col=24, seed=3)
        net.step(40 - net.t)
        net.sync()
        st = net.stats()
        _say(f"large, ORDERED: step 40 ({st['events']} events so far)")
        n2 = _check_one_step_ordered(net, orc, cols=[4095, 1234], per_col=24, seed=4)
        assert n1 + n2 > 0
        _say(f"large, ORDERED: {n1} + {n2} deliveries summed in canonical order")
    finally:
        net.close()
