"""Steps replayed from captured HIP graphs (tuning key 8) against the same
steps launched one by one.  Bar: rasters, weights (w, P, D), state (v, u)
and counters equal bit for bit at every checkpoint.  The replays are mixed
with the program's own work between them (reads and synchronisations,
stimulus changes, launch-shape changes that force a new capture, timed steps
that bypass the graph, the autotuner), and every checkpoint is compared.
Consolidation steps and the first step always run outside the graph, so the
runs below cross several consolidation boundaries at varying offsets."""
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


def _snap(net):
    tt, ii = net.read_spikes(1, net.t + 1) if net.t >= 1 else (np.zeros(0), np.zeros(0))
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


def _cfg(**over):
    c = W.tiny(weight_update_period=50, seed=7311, thalamic_rate=1.5, **over)
    c["raster_steps"] = 600
    return c


def test_graph_replays_equal_direct_steps(dp, orc):
    chunks = [1, 3, 17, 40, 8, 64, 99, 7, 16, 9, 136]   # 400 steps
    _say("graph replays (G = 8 and 5) vs direct steps, tiny, 11 checkpoints")
    ref = dp.Network(_cfg())
    ref.set_tuning(8, 0)
    g8 = dp.Network(_cfg())
    g5 = dp.Network(_cfg())
    g5.set_tuning(8, 5)
    try:
        for k, n in enumerate(chunks):
            for net in (ref, g8, g5):
                net.step(n)
            a = _snap(ref)
            _same(a, _snap(g8), f"G=8 after chunk {k}")
            _same(a, _snap(g5), f"G=5 after chunk {k}")
        assert ref.stats()["graph_steps"] == 0
        gs8, gs5 = g8.stats()["graph_steps"], g5.stats()["graph_steps"]
        assert gs8 % 8 == 0 and gs5 % 5 == 0
        assert gs8 >= 200 and gs5 >= 200, (gs8, gs5)
        assert ref.stats()["consolidations"] == 8
        # and the oracle
        T = sum(chunks)
        o = orc.Net(_cfg(), T)
        o.run(T)
        ot, oi = o.raster()
        s = o.synapses()
        ov, ou = o.state()
        o.close()
        got = _snap(g8)
        np.testing.assert_array_equal(got["tt"], ot)
        np.testing.assert_array_equal(got["ii"], oi)
        for key, r in (("w", s["w"]), ("P", s["P"]), ("D", s["D"]), ("v", ov), ("u", ou)):
            np.testing.assert_array_equal(got[key].view(np.uint32), r.view(np.uint32), err_msg=key)
    finally:
        for net in (ref, g8, g5):
            net.close()


def test_graph_with_interleaved_changes(dp):
    _say("graph replays mixed with stimulus, shape changes, timing and autotuning")
    ref = dp.Network(_cfg(synapses_per_neuron=160))
    ref.set_tuning(8, 0)
    g = dp.Network(_cfg(synapses_per_neuron=160))
    nets = (ref, g)
    rng = np.random.default_rng(5)
    try:
        def both(fn):
            for net in nets:
                fn(net)

        def check(what):
            _same(_snap(ref), _snap(g), what)

        both(lambda n: n.step(30))
        check("start")
        st, si, sm = W.stimulus_list(ref.N, 200, 300, seed=77)
        st = st + 40   # stimuli in steps 40 .. 239
        both(lambda n: n.set_stimulus(st, si, sm))
        both(lambda n: n.step(25))
        check("after the stimulus was set")
        before = g.stats()["graph_steps"]
        g.set_tuning(0, 512)          # new launch shapes: captured again
        g.set_tuning(1, 512)
        both(lambda n: n.step(40))
        check("after a shape change")
        assert g.stats()["graph_steps"] > before
        g.set_tuning(7, 0)            # LTP and delivery as two kernels
        g.set_tuning(3, int(rng.choice([1, 2, 8])))
        both(lambda n: n.step(33))
        check("unfused")
        g.set_timing(True)            # timed steps run directly
        before = g.stats()["graph_steps"]
        both(lambda n: n.step(20))
        assert g.stats()["graph_steps"] == before
        g.set_timing(False)
        check("timed steps")
        g.set_tuning(8, 16)
        both(lambda n: n.step(61))
        check("G = 16")
        both(lambda n: n.autotune(2))   # 24 direct steps under trial shapes
        both(lambda n: n.step(77))
        check("after autotuning")
        both(lambda n: n.set_stimulus(np.zeros(0, np.uint32), np.zeros(0, np.uint32),
                                      np.zeros(0, np.float32)))
        both(lambda n: n.step(50))
        check("stimulus cleared")
    finally:
        for net in nets:
            net.close()


MIX = [
    W.make_config(grid_x=2, grid_y=2, synapses_per_neuron=100, thalamic_rate=0.75, seed=2101,
                  weight_update_period=40),
    W.make_config(grid_x=3, grid_y=3, synapses_per_neuron=250, thalamic_rate=1.5, seed=2102,
                  weight_update_period=100),
    W.make_config(grid_x=2, grid_y=2, synapses_per_neuron=625, thalamic_rate=1.0, seed=2103,
                  weight_update_period=60),
    W.make_config(grid_x=4, grid_y=2, neurons_per_column=700, synapses_per_neuron=180,
                  thalamic_rate=2.0, seed=2104, weight_update_period=70),
]


def test_graph_batch_equals_direct_solo_runs(dp):
    chunks = [5, 50, 37, 1, 64, 43]   # 200 steps
    _say("batch of 4 uneven networks replayed from graphs vs direct solo runs")
    solo = [dp.Network(c) for c in MIX]
    for n in solo:
        n.set_tuning(8, 0)
    nets = [dp.Network(c) for c in MIX]
    b = dp.Batch(nets)
    try:
        for k, n in enumerate(chunks):
            for s in solo:
                s.step(n)
            b.step(n)
            if k in (1, 3, 5):
                for j, (s, m) in enumerate(zip(solo, nets)):
                    _same(_snap(s), _snap(m), f"member {j} after chunk {k}")
        st = b.stats()
        assert st["graph_steps"] >= 4 * 100, st["graph_steps"]
        assert st["steps"] == 4 * sum(chunks)
    finally:
        b.close()
        for n in solo + nets:
            n.close()


def test_graph_atomic_mode_accounting(dp):
    # unordered fp32 atomics: each delivery still happens exactly once
    T = 250
    _say("graph replays, ATOMIC summation, delivery accounting")
    cfg = dict(_cfg(synapses_per_neuron=200), sum_mode=W.SUM_ATOMIC)
    net = dp.Network(cfg)
    try:
        net.step(T)
        net.sync()
        st = net.stats()
        assert st["graph_steps"] >= 200
        tt, ii = net.read_spikes(1, T + 1)
        dly = net.read_connectivity()[1]
        M, dmax = cfg["synapses_per_neuron"], cfg["max_delay"]
        d = dly.reshape(-1, M).astype(np.int64)
        cum = np.stack([(d <= k).sum(axis=1) for k in range(dmax + 1)], axis=1)
        lim = np.minimum(T - tt.astype(np.int64), dmax)
        ok = lim >= 1
        assert st["events"] == int(cum[ii[ok].astype(np.int64), lim[ok]].sum())
    finally:
        net.close()


def test_graph_autotuned_batch_members_equal_oracle(dp, orc):
    # the batched path as a caller runs it: autotuned launch shapes, then
    # runs of 8 steps replayed from captured graphs (with each member's own
    # consolidations launched directly), every member against the oracle
    T = 230
    _say("autotuned batch of 4 uneven networks replayed from graphs vs the oracle")
    nets = [dp.Network(c) for c in MIX]
    b = dp.Batch(nets)
    try:
        b.autotune(3)             # 2 rounds x 6 shapes x 3 steps = 36 steps
        b.step(T - 36)
        st = b.stats()
        assert st["steps"] == 4 * T
        assert st["graph_steps"] >= 4 * 120, st["graph_steps"]
        b.close()
        for j, (cfg, n) in enumerate(zip(MIX, nets)):
            got = _snap(n)
            o = orc.Net(cfg, T)
            o.run(T)
            ot, oi = o.raster()
            s = o.synapses()
            ov, ou = o.state()
            o.close()
            assert len(ot) > 100
            np.testing.assert_array_equal(got["tt"], ot, err_msg=f"member {j}")
            np.testing.assert_array_equal(got["ii"], oi, err_msg=f"member {j}")
            for key, r in (("w", s["w"]), ("P", s["P"]), ("D", s["D"]), ("v", ov), ("u", ou)):
                np.testing.assert_array_equal(got[key].view(np.uint32), r.view(np.uint32),
                                              err_msg=f"member {j} {key}")
    finally:
        b.close()
        for n in nets:
            n.close()
