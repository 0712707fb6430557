"""The large workload at full size (64x64 columns x 1250 neurons, M = 625,
3.2 G synapses) with the launch shapes the benchmark uses, checked on outputs
the oracle computes one at a time:

  * connectivity: sampled rows against the oracle's per-synapse draw (Sec. 2,
    "Distributed generation of reproducible connections");
  * one step of sampled neurons: the input current is rebuilt from the
    network's own connectivity, weights and raster (every synapse whose
    source spiked d - 1 steps earlier, plus the oracle's thalamic picks, in
    fixed point), and the oracle's neuron update must then give the GPU's v,
    u and spike bit for bit (Sec. 2 loop items 2.3-2.7).

The step is checked early (rates still rising, spiking runs decoded per
delay) and after the network fires in every step (the all-firing path)."""
import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W

pytestmark = pytest.mark.gpu

RS = (0.02, 0.2, -65.0, 8.0)   # regular spiking (excitatory), Sec. 2
FS = (0.1, 0.2, -65.0, 2.0)    # fast spiking (inhibitory)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def dp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1310_8478_amd import dpsnn
    dpsnn.lib()
    return dpsnn


@pytest.fixture(scope="module")
def large(dp):
    _say("large: building 3.2 G synapses")
    net = dp.Network(W.large())
    yield net
    net.close()


def _window_columns(cfg, c, r=3):
    gx, gy = cfg["grid_x"], cfg["grid_y"]
    cx, cy = c % gx, c // gx
    return sorted({((cy + dy) % gy) * gx + (cx + dx) % gx
                   for dx in range(-r, r + 1) for dy in range(-r, r + 1)})


def test_large_connectivity_rows(large, orc):
    cfg = large.cfg
    M = cfg["synapses_per_neuron"]
    rng = np.random.default_rng(11)
    rows = rng.integers(0, large.N, size=24)
    _say("large: 24 sampled rows against the oracle's draws")
    for i in rows.tolist():
        tg, dl = large.read_connectivity(i * M, M)
        w = large.read_weights(i * M, M, P=False, D=False)["w"]
        ref = [orc.synapse(cfg, i, j) for j in range(M)]
        np.testing.assert_array_equal(tg, np.array([r[0] for r in ref], np.uint32))
        np.testing.assert_array_equal(dl, np.array([r[1] for r in ref], np.uint8))
        if large.t < cfg["weight_update_period"]:
            np.testing.assert_array_equal(w.view(np.uint32),
                                          np.array([r[2] for r in ref], np.float32).view(np.uint32))


def _check_one_step(dp, orc, net, cols, per_col=24, seed=0):
    """Step net once and check sampled neurons of `cols` against the oracle."""
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
    for ck in cols:
        sample = ck * Ncol + np.sort(rng.choice(Ncol, size=per_col, replace=False))
        acc = {int(k): 0 for k in sample}
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
            for p, k, on in zip(pos.tolist(), tg[pos].tolist(), live.tolist()):
                if on:
                    acc[k] += orc.q32(float(w[p]))
        picks = orc.thalamic(cfg, ck, T1)
        for l in picks:
            k = ck * Ncol + l
            if k in acc:
                acc[k] += orc.q32(cfg["thalamic_current"])
        for k in sample.tolist():
            a, b, c, d = RS if (k % Ncol) < Ne else FS
            v, u, f = orc.neuron_step(float(v0[k]), float(u0[k]), orc.dq32(acc[k]), a, b, c, d)
            assert np.float32(v).view(np.uint32) == v1[k].view(np.uint32), (T1, k, v, v1[k])
            assert np.float32(u).view(np.uint32) == u1[k].view(np.uint32), (T1, k, u, u1[k])
            assert f == bool(fired[k]), (T1, k)


def test_large_sampled_steps(dp, orc, large):
    cfg = large.cfg
    assert large.t == 0 or large.t < 30
    large.step(30 - large.t)
    large.sync()
    _say("large: step 30, sampled neurons of 2 columns")
    _check_one_step(dp, orc, large, cols=[0, 2081], seed=1)
    large.step(150 - large.t)
    large.sync()
    st = large.stats()
    _, ids = large.read_spikes(151 - cfg["max_delay"], 151)
    _say(f"large: step 150 ({len(ids)} spikes in the last {cfg['max_delay']} stamps)")
    all_firing = len(ids) == large.N * cfg["max_delay"]
    _check_one_step(dp, orc, large, cols=[4095, 1234], seed=2)
    assert st["events"] > 0
    # once every neuron fires in every step, every synapse delivers in every step
    if all_firing:
        s0 = large.stats()["events"]
        large.step(5)
        large.sync()
        assert large.stats()["events"] - s0 == 5 * large.N * cfg["synapses_per_neuron"]


def test_large_consolidation_both_forms(dp):
    # the first consolidation of the full-size network (Sec. 3, Table 2's
    # long-term plasticity block), at step 39 with decay 1: the folded
    # derivative is then the P left behind, so every excitatory weight must
    # equal clamp(w_init + (bias + P)) with D = 0, and inhibitory synapses
    # stay at w_inh with P = D = 0 -- on sampled rows on both sides of
    # position 2^31, for the one-pass forward form and the two-pass form,
    # which must agree bit for bit
    cfg = W.large(weight_update_period=40, sd_decay=1.0)
    M = cfg["synapses_per_neuron"]
    ncol = cfg["neurons_per_column"]
    N = cfg["grid_x"] * cfg["grid_y"] * ncol
    Ne = int(round(cfg["exc_fraction"] * ncol))
    rng = np.random.default_rng(41)
    rows = np.concatenate([rng.integers(0, N, size=10), rng.integers((2 ** 31) // M + 1, N, size=10),
                           [N - 1, ncol * 37 + Ne - 1, ncol * 37 + Ne]]).tolist()
    got = {}
    for form in (1, 0):
        _say(f"large: first consolidation, form {form}")
        net = dp.Network(cfg)
        try:
            net.set_tuning(14, form)
            net.step(40)
            net.sync()
            assert net.stats()["consolidations"] == 1
            if form == 1:
                # add excitatory sources that spiked (their synapses carry P)
                _, ids = net.read_spikes(1, 41)
                exc = np.unique(ids[(ids % ncol) < Ne])
                assert len(exc) >= 6
                rows += exc[:3].tolist() + exc[-3:].tolist()
            got[form] = {i: net.read_weights(i * M, M) for i in rows}
        finally:
            net.close()
    bias = np.float32(cfg["wu_bias"])
    wmax = np.float32(cfg["w_max"])
    w0 = np.float32(cfg["w_exc_init"])
    moved = 0
    for i in rows:
        a = got[1][i]
        for k in ("w", "P", "D"):
            np.testing.assert_array_equal(a[k].view(np.uint32), got[0][i][k].view(np.uint32), err_msg=k)
        assert not a["D"].any()
        if i % ncol < Ne:
            want = np.clip(w0 + (bias + a["P"]), np.float32(0.0), wmax).astype(np.float32)
            np.testing.assert_array_equal(a["w"].view(np.uint32), want.view(np.uint32))
            moved += int((a["P"] != 0).sum())
        else:
            assert (a["w"] == np.float32(cfg["w_inh"])).all() and not a["P"].any()
    assert moved > 0, "some sampled synapse must carry a derivative"


def test_large_sampled_stdp_from_raster(dp):
    # P and D of the full-size network (Sec. 2, the STDP rule and its P / D
    # split) on sampled rows, recomputed from the network's own raster and
    # connectivity by the post-hoc checker: 70 steps, rows of excitatory
    # sources that spiked, random rows and rows beyond position 2^31
    from simref import stdp_posthoc_synapses
    cfg = W.large()
    M = cfg["synapses_per_neuron"]
    ncol = cfg["neurons_per_column"]
    N = cfg["grid_x"] * cfg["grid_y"] * ncol
    Ne = int(round(cfg["exc_fraction"] * ncol))
    T = 70
    _say(f"large: {T} steps, sampled P and D against the post-hoc STDP checker")
    net = dp.Network(cfg)
    try:
        net.step(T)
        net.sync()
        tt, ii = net.read_spikes(1, T + 1)
        exc = np.unique(ii[(ii % ncol) < Ne])
        rng = np.random.default_rng(43)
        rows = np.unique(np.concatenate([exc[:4], exc[-4:], rng.choice(exc, 4),
                                         rng.integers(0, N, size=4),
                                         rng.integers((2 ** 31) // M + 1, N, size=4)])).tolist()
        got = {i: net.read_weights(i * M, M) for i in rows}
        conn = {i: net.read_connectivity(i * M, M) for i in rows}
    finally:
        net.close()
    _say(f"  {len(tt)} spikes, {len(rows)} rows")
    src = np.repeat(np.array(rows, np.int64), M)
    tgt = np.concatenate([conn[i][0] for i in rows])
    dly = np.concatenate([conn[i][1] for i in rows])
    w, P, D = stdp_posthoc_synapses(cfg, tt, ii, src, tgt, dly, T)
    gP = np.concatenate([got[i]["P"] for i in rows])
    gD = np.concatenate([got[i]["D"] for i in rows])
    gw = np.concatenate([got[i]["w"] for i in rows])
    for name, a, b in (("P", gP, P), ("D", gD, D), ("w", gw, w)):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32), err_msg=name)
    _say(f"  {(P != 0).sum()} synapses with P != 0, {(D != 0).sum()} with D != 0")
    assert (P != 0).sum() >= 20 and (D != 0).sum() >= 20, "the sample must carry derivatives"
