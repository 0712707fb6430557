"""Pins of the oracle's network step: delivery, currents, STDP, consolidation.

* an independent dense brute-force simulator reproduces the oracle bit-exactly
  on tiny networks, in both reproducible summation modes;
* a post-hoc checker recomputes P, D and w from the raster and connectivity
  alone (Sec. 2, STDP rule);
* hand-traced spike pairs give the table values worked out by hand;
* exact invariants: delivered events, thalamic count, weight range,
  inhibitory synapses not plastic;
* the fixed-point current is the nearest fp32 to the exact rational sum.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W

from simref import brute_force, ensemble_stats, stdp_posthoc, stdp_posthoc_synapses, tables, qfix, dqfix

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _micro(mode, **over):
    base = dict(grid_x=2, grid_y=2, neurons_per_column=30, synapses_per_neuron=12,
                max_delay=6, w_exc_init=9.0, w_inh=-6.0, weight_update_period=40,
                thalamic_rate=1.5, sum_mode=mode, seed=77)
    base.update(over)
    return W.make_config(**base)


@pytest.mark.parametrize("mode", [W.SUM_FIXED, W.SUM_ORDERED])
@pytest.mark.parametrize("seed", [77, 78])
def test_oracle_equals_brute_force(orc, mode, seed):
    cfg = _micro(mode, seed=seed)
    T = 120
    N = 4 * 30
    st = W.stimulus_list(N, T, 150, seed=seed, mv_range=(10.0, 120.0))
    net = orc.Net(cfg, T)
    net.set_stimulus(*st)
    net.run(T)
    tt, ii = net.raster()
    syn = net.synapses()
    v, u = net.state()
    ref_r, w, P, D, rv, ru = brute_force(orc, cfg, T, stim=st)
    assert len(tt) > 100, "the case must spike"
    assert list(zip(tt.tolist(), ii.tolist())) == [(int(a), int(b)) for a, b in ref_r]
    np.testing.assert_array_equal(syn["w"].view(np.uint32), w.view(np.uint32))
    np.testing.assert_array_equal(syn["P"].view(np.uint32), P.view(np.uint32))
    np.testing.assert_array_equal(syn["D"].view(np.uint32), D.view(np.uint32))
    np.testing.assert_array_equal(v.view(np.uint32), rv.view(np.uint32))
    np.testing.assert_array_equal(u.view(np.uint32), ru.view(np.uint32))
    assert (syn["w"] != np.float32(cfg["w_exc_init"])).any()


@pytest.mark.parametrize("mode", [W.SUM_FIXED, W.SUM_ORDERED])
def test_posthoc_stdp_on_tiny_workload(orc, mode):
    # the 2x2 x 1250, M = 100 workload, 400 steps, consolidation every 150 steps
    cfg = W.tiny(sum_mode=mode, weight_update_period=150)
    T = 400
    net = orc.Net(cfg, T)
    net.run(T)
    tt, ii = net.raster()
    syn = net.synapses()
    assert len(tt) > 1000
    w, P, D = stdp_posthoc(cfg, net.N, tt, ii, syn["tgt"], syn["dly"], T)
    np.testing.assert_array_equal(syn["P"].view(np.uint32), P.view(np.uint32))
    np.testing.assert_array_equal(syn["D"].view(np.uint32), D.view(np.uint32))
    np.testing.assert_array_equal(syn["w"].view(np.uint32), w.view(np.uint32))


def test_posthoc_stdp_on_chosen_synapses(orc):
    # the sampled form used at full size: chosen rows (and a scatter of single
    # synapses) of the tiny workload, against the oracle's arrays
    cfg = W.tiny(weight_update_period=150)
    T = 400
    M = cfg["synapses_per_neuron"]
    net = orc.Net(cfg, T)
    net.run(T)
    tt, ii = net.raster()
    syn = net.synapses()
    net.close()
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([ii[:5], rng.integers(0, 5000, size=7)]))
    sel = np.concatenate([np.arange(i * M, (i + 1) * M) for i in rows.tolist()] +
                         [rng.integers(0, 5000 * M, size=300)])
    w, P, D = stdp_posthoc_synapses(cfg, tt, ii, sel // M, syn["tgt"][sel], syn["dly"][sel], T)
    assert (P != 0).any() and (D != 0).any()
    for name, a, b in (("w", w, syn["w"][sel]), ("P", P, syn["P"][sel]), ("D", D, syn["D"][sel])):
        np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32), err_msg=name)


def test_delivered_events_and_thalamic_invariants(orc):
    cfg = W.tiny()
    T = 300
    net = orc.Net(cfg, T)
    net.run(T)
    tt, ii = net.raster()
    syn = net.synapses()
    M = cfg["synapses_per_neuron"]
    dl = syn["dly"].reshape(-1, M).astype(np.int64)
    # a spike stamped s reaches its delay-d synapses in step s + d - 1 <= T - 1
    want = sum(int((dl[i] <= T - s).sum()) for s, i in zip(tt.tolist(), ii.tolist()))
    c = net.counters()
    assert c["events"] == want
    assert c["thalamic"] == 4 * T          # rate 1: one pick per column per ms
    assert c["spikes"] == len(tt)
    # raster sorted by (stamp, id), stamps within 1..T
    assert (np.diff(tt.astype(np.int64)) >= 0).all()
    same = np.diff(tt.astype(np.int64)) == 0
    assert (np.diff(ii.astype(np.int64))[same] > 0).all()
    assert tt.min() >= 1 and tt.max() <= T


def test_consolidation_invariants(orc):
    cfg = W.tiny(weight_update_period=100)
    T = 300
    net = orc.Net(cfg, T)
    net.run(T)
    syn = net.synapses()
    N, M = net.N, cfg["synapses_per_neuron"]
    exc = (np.repeat(np.arange(N), M) % 1250) < 1000
    assert (syn["w"][exc] >= 0).all() and (syn["w"][exc] <= cfg["w_max"]).all()
    assert (syn["w"][~exc] == np.float32(cfg["w_inh"])).all()
    assert not syn["P"][~exc].any() and not syn["D"][~exc].any()
    # D is cleared by the last consolidation (step 299 -> 300 is a multiple of 100)
    assert not syn["D"].any()
    assert (syn["w"][exc] != np.float32(6.0)).any()


def _golden_stdp():
    out = []
    for line in open(os.path.join(GOLD, "stdp_hand_values.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, dt, v = line.split()
        out.append((k, int(dt), float(v)))
    return out


@pytest.mark.parametrize("kind,dt,val", _golden_stdp())
def test_stdp_amplitudes_hand_values(orc, kind, dt, val):
    cfg = W.tiny()
    got = orc.tp(cfg, dt) if kind == "LTP" else orc.tm(cfg, dt)
    assert got == pytest.approx(val, rel=2e-7)


def _find_synapse(orc, cfg, delay):
    Ncol = cfg["neurons_per_column"]
    Ne = orc.exc_per_column(cfg)
    for i in range(Ne):
        for j in range(cfg["synapses_per_neuron"]):
            k, d, _ = orc.synapse(cfg, i, j)
            if d == delay:
                return i, j, k
    raise AssertionError("no synapse with that delay")


def test_hand_traced_pair(orc):
    # pre stamped 10, delay 5 (first effect at 15), post stamped 12 and 17:
    # LTD at the arrival pairs with post 12: dt = 12 - 10 - 5 = -3 -> D += A- e^{-3/20}
    # LTP at post 17 pairs with the arrival: dt = 17 - 10 - 5 = 2 -> P += A+ e^{-2/20}
    cfg = W.make_config(grid_x=1, grid_y=1, neurons_per_column=20, synapses_per_neuron=4,
                        w_exc_init=0.0, thalamic_rate=0.0, weight_update_period=0)
    i, j, k = _find_synapse(orc, cfg, 5)
    net = orc.Net(cfg, 30)
    net.set_stimulus([9, 11, 16], [i, k, k], [200.0, 200.0, 200.0])
    net.run(30)
    tt, ii = net.raster()
    assert sorted(zip(tt.tolist(), ii.tolist())) == sorted([(10, i), (12, k), (17, k)])
    syn = net.synapses(i * 4 + j, 1)
    assert syn["P"][0] == np.float32(0.1 * np.exp(-0.1)) == orc.tp(cfg, 2)
    assert syn["D"][0] == orc.tm(cfg, 3)
    assert syn["D"][0] == pytest.approx(0.12 * np.exp(-0.15), rel=2e-7)


def test_delayed_chain_fires_after_exact_delay(orc):
    # one strong synapse: a pre forced at stamp s makes the post fire at stamp s + d
    cfg = W.make_config(grid_x=1, grid_y=1, neurons_per_column=20, synapses_per_neuron=4,
                        w_exc_init=400.0, thalamic_rate=0.0, weight_update_period=0)
    for delay in (1, 3, 7):
        i, j, k = _find_synapse(orc, cfg, delay)
        net = orc.Net(cfg, 40)
        net.set_stimulus([4], [i], [300.0])
        net.run(40)
        tt, ii = net.raster()
        got = set(zip(tt.tolist(), ii.tolist()))
        assert (5, i) in got and (5 + delay, k) in got


def test_fixed_point_sum_is_exact(orc):
    rng = np.random.default_rng(5)
    for trial in range(200):
        n = int(rng.integers(1, 60))
        xs = (rng.standard_normal(n) * rng.choice([1e-9, 1e-3, 1.0, 10.0, 100.0])).astype(np.float32)
        q = [orc.q32(float(x)) for x in xs]
        assert q == [qfix(x) for x in xs]
        # each term is the nearest multiple of 2^-32 to x (ties to even)
        for x, a in zip(xs, q):
            ex = Fraction(float(x)) * 2 ** 32
            assert abs(ex - a) <= Fraction(1, 2)
        tot = sum(q)
        got = orc.dq32(tot)
        assert got == dqfix(tot)
        # nearest fp32 to the exact rational value
        exact = Fraction(tot, 2 ** 32)
        cand = [np.nextafter(np.float32(got), np.float32(-np.inf)), np.float32(got),
                np.nextafter(np.float32(got), np.float32(np.inf))]
        errs = [abs(Fraction(float(c)) - exact) for c in cand]
        assert errs[1] <= min(errs)


def test_tables_match_test_side_tables(orc):
    cfg = W.tiny()
    tp, tm = tables(cfg, 2100)
    for k in list(range(0, 40)) + [100, 500, 1000, 1699, 1700, 1701, 1720, 2000]:
        assert np.float32(orc.tp(cfg, k)) == tp[k]
        if k >= 1:
            assert np.float32(orc.tm(cfg, k)) == tm[k]
    assert tp[2000] == 0 and tp[1000] > 0


def _golden_consolidation():
    out = []
    for line in open(os.path.join(GOLD, "consolidation_hand.txt")):
        if line.startswith("#") or not line.strip():
            continue
        head, before, after = line.split("|")
        name, beta, gamma, w0, wmax, posts = head.split()
        out.append(dict(name=name, beta=float(beta), gamma=float(gamma), w0=float(w0),
                        wmax=float(wmax), posts=[int(x) for x in posts.split(",")],
                        before=[int(x, 16) for x in before.split()],
                        after=[int(x, 16) for x in after.split()]))
    return out


@pytest.mark.parametrize("case", _golden_consolidation(), ids=lambda c: c["name"])
def test_consolidation_hand_values(orc, case):
    # the hand-traced pair (pre stamped 10, delay 5, posts forced) followed by
    # one consolidation after step 19; P, D before it and w, P, D after it
    # against values worked by hand (bias sign, decay, both clamps, D reset,
    # the sign of a zero)
    cfg = W.make_config(grid_x=1, grid_y=1, neurons_per_column=20, synapses_per_neuron=4,
                        w_exc_init=case["w0"], w_max=case["wmax"], thalamic_rate=0.0,
                        weight_update_period=20, wu_bias=case["beta"], sd_decay=case["gamma"])
    i, j, k = _find_synapse(orc, cfg, 5)
    stim_t = [9] + [p - 1 for p in case["posts"]]
    stim_id = [i] + [k] * len(case["posts"])
    for T, want in ((19, case["before"][:2] + [None]), (20, case["after"][1:] + [case["after"][0]])):
        net = orc.Net(cfg, T)
        net.set_stimulus(stim_t, stim_id, [200.0] * len(stim_t))
        net.run(T)
        tt, ii = net.raster()
        assert sorted(zip(tt.tolist(), ii.tolist())) == sorted(
            [(10, i)] + [(p, k) for p in case["posts"]]), "only the forced spikes may occur"
        syn = net.synapses(i * 4 + j, 1)
        net.close()
        P, D, w = (int(syn[x].view(np.uint32)[0]) for x in ("P", "D", "w"))
        assert (P, D) == tuple(want[:2]), (hex(P), hex(D))
        if want[2] is not None:
            assert w == want[2], hex(w)
        else:
            assert w == int(np.float32(case["w0"]).view(np.uint32))


STAT_SEEDS = list(range(1311, 1327))


def test_statistical_bar_holds_between_the_reproducible_orders(orc):
    # calibration of the unordered mode's statistical bar: the oracle's two
    # reproducible summation orders (fixed point and ordered fp32) sum the
    # same currents differently; on the tiny workload with consolidation
    # every 100 steps (non-integer weights from step 99) their runs diverge,
    # yet over 16 seeds the median rate deviation stays within 1 % and the
    # pooled weight histogram within L1 0.02
    N, M, T = 5000, 100, 1000
    runs = {}
    for mode in (W.SUM_FIXED, W.SUM_ORDERED):
        runs[mode] = []
        for seed in STAT_SEEDS:
            o = orc.Net(W.tiny(seed=seed, sum_mode=mode, weight_update_period=100), T)
            o.run(T)
            r = o.raster()
            runs[mode].append((len(r[0]), r, o.synapses()["w"]))
            o.close()
    exc = (np.repeat(np.arange(N), M) % 1250) < 1000
    med, l1, differ = ensemble_stats(runs[W.SUM_FIXED], runs[W.SUM_ORDERED], exc)
    assert differ >= len(STAT_SEEDS) // 2, differ
    assert med <= 0.01, med
    assert l1 <= 0.02, l1
