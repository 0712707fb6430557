"""Degenerate and extreme configurations against the oracle, bit-exact in both
reproducible summation modes: the smallest column and fan-out, a network
without inhibitory neurons, a silent network (no thalamic input) with and
without stimulus, no consolidation, the longest delay, all targets in the
own column or none, a fan-out larger than the column, ragged raster words,
the widest column (1024 raster words per column, one delay per chunk), and a
saturated column whose targets receive more than 1024 events per step."""
import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W
from test_gpu_parity import assert_bitexact, gpu_run, oracle_run

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


EDGE = {
    # Ncol = 2 (one excitatory, one inhibitory), M = 1, delay 1 only
    "min_column": (W.make_config(grid_x=1, grid_y=1, neurons_per_column=2, exc_fraction=0.5,
                                 synapses_per_neuron=1, max_delay=1, thalamic_rate=0.7,
                                 w_exc_init=30.0, weight_update_period=40), 200),
    "all_excitatory": (W.make_config(grid_x=3, grid_y=3, neurons_per_column=100,
                                     exc_fraction=1.0, synapses_per_neuron=40,
                                     weight_update_period=60, thalamic_rate=2.0), 200),
    "no_consolidation": (W.make_config(grid_x=2, grid_y=2, neurons_per_column=150,
                                       synapses_per_neuron=50, weight_update_period=0,
                                       thalamic_rate=3.0, w_exc_init=8.0), 250),
    "max_delay_31": (W.make_config(grid_x=2, grid_y=2, neurons_per_column=200,
                                   synapses_per_neuron=60, max_delay=31, thalamic_rate=3.0,
                                   w_exc_init=9.0, weight_update_period=70), 250),
    "own_fraction_0": (W.make_config(grid_x=3, grid_y=2, neurons_per_column=120,
                                     synapses_per_neuron=30, own_fraction=0.0, thalamic_rate=3.0,
                                     w_exc_init=9.0, weight_update_period=50), 200),
    "own_fraction_1": (W.make_config(grid_x=3, grid_y=2, neurons_per_column=120,
                                     synapses_per_neuron=30, own_fraction=1.0, thalamic_rate=3.0,
                                     w_exc_init=9.0, weight_update_period=50), 200),
    "fanout_over_column": (W.make_config(grid_x=1, grid_y=1, neurons_per_column=300,
                                         synapses_per_neuron=1500, w_exc_init=0.6, w_inh=-0.5,
                                         w_max=1.0, thalamic_rate=2.0, weight_update_period=60), 150),
    "ragged_words": (W.make_config(grid_x=2, grid_y=1, neurons_per_column=65,
                                   synapses_per_neuron=20, thalamic_rate=2.0, w_exc_init=12.0,
                                   weight_update_period=45), 200),
    # 13 x Ncol x M above 2^28: the network keeps no forward-to-reverse map
    # and consolidates in the two-pass form; its reverse rows (about 6400
    # entries) go through the long-row sort
    "no_consolidation_map": (W.make_config(grid_x=1, grid_y=1, neurons_per_column=2600,
                                           synapses_per_neuron=8000, w_exc_init=0.05, w_inh=-0.05,
                                           w_max=1.0, thalamic_rate=30.0, thalamic_current=40.0,
                                           weight_update_period=40), 100),
    "widest_column": (W.make_config(grid_x=1, grid_y=1, neurons_per_column=65535,
                                    synapses_per_neuron=3, thalamic_rate=300.0, w_exc_init=10.0,
                                    weight_update_period=40), 120),
    # every neuron fires in every step from step ~20 on and each target then
    # receives 1200-1600 events per step (above the ORDERED fold's LDS sort)
    "saturated_fanout": (W.make_config(grid_x=1, grid_y=1, neurons_per_column=300,
                                       synapses_per_neuron=1500, w_exc_init=10.0, w_inh=-0.5,
                                       w_max=10.0, thalamic_rate=20.0, weight_update_period=60), 120),
}


@pytest.mark.parametrize("mode", [W.SUM_FIXED, W.SUM_ORDERED])
@pytest.mark.parametrize("name", list(EDGE))
def test_edge_configuration_bitexact(dp, orc, name, mode):
    cfg, T = EDGE[name]
    cfg = dict(cfg, sum_mode=mode)
    _say(f"edge {name}, mode {mode}, {T} steps")
    g = gpu_run(dp, cfg, T)
    o = oracle_run(orc, cfg, T)
    assert_bitexact(g, o)
    if name != "widest_column":
        assert len(o["tt"]) > 0, "the case should be active"
    if name == "saturated_fanout":
        per = np.bincount(o["tt"], minlength=T + 1)
        assert (per[40:] == cfg["neurons_per_column"]).sum() >= 60, "the column must saturate"


@pytest.mark.parametrize("mode", [W.SUM_FIXED, W.SUM_ORDERED])
def test_silent_network_and_stimulus(dp, orc, mode):
    # no thalamic input: nothing fires until the stimulus drives a few neurons
    cfg = W.make_config(grid_x=2, grid_y=2, neurons_per_column=200, synapses_per_neuron=60,
                        thalamic_rate=0.0, w_exc_init=9.0, weight_update_period=50, sum_mode=mode)
    T = 150
    _say(f"silent network, mode {mode}")
    g = gpu_run(dp, cfg, T)
    assert len(g["tt"]) == 0
    assert g["stats"]["events"] == 0 and g["stats"]["ltp_visits"] == 0
    o = oracle_run(orc, cfg, T)
    assert_bitexact(g, o)
    t = np.array([10, 10, 11, 60, 61, 62], dtype=np.uint32)
    ids = np.array([0, 5, 401, 777, 3, 0], dtype=np.uint32)
    mv = np.array([40.0, 40.0, 40.0, 40.0, 25.0, 40.0], dtype=np.float32)
    g = gpu_run(dp, cfg, T, stim=(t, ids, mv))
    o = oracle_run(orc, cfg, T, stim=(t, ids, mv))
    assert_bitexact(g, o)
    assert len(o["tt"]) >= 4


@pytest.mark.parametrize("name", list(EDGE))
def test_edge_configuration_sparse_path_bitexact(dp, orc, name):
    # the wavefront-level sparse LTP and delivery paths forced on, on every
    # degenerate shape (queue rounds, 32-bit targets, no LDS window for the
    # widest column, inhibitory fan-out beyond one pass of a wavefront)
    cfg, T = EDGE[name]
    cfg = dict(cfg, sum_mode=W.SUM_FIXED)
    _say(f"edge {name}, sparse paths, {T} steps")
    o = oracle_run(orc, cfg, T)
    g = gpu_run(dp, cfg, T, tuning=((12, 1),))
    assert_bitexact(g, o)
    assert g["stats"]["events"] == o["counters"]["events"]
    assert g["stats"]["ltp_visits"] == o["counters"]["ltp_visits"]
    # the sparse LTP beside the run-based delivery, with the partial-window
    # ages, and consolidation as the two reverse-order passes
    g = gpu_run(dp, cfg, T, tuning=((11, 1), (2, 2), (4, 1), (14, 0)))
    assert_bitexact(g, o)
    assert g["stats"]["events"] == o["counters"]["events"]
    assert g["stats"]["ltp_visits"] == o["counters"]["ltp_visits"]
