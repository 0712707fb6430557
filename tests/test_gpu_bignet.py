"""The paper's largest Table 1 grid (256 x 128 columns of 1000 neurons,
M = 200: 6.55 G synapses, 64-bit synapse positions) on one device, checked on
outputs the oracle computes one at a time:

  * connectivity, weights and accumulators of sampled rows, including rows
    whose canonical and forward positions lie beyond 2^32, against the
    oracle's per-synapse draws;
  * one step of sampled neurons against the oracle's neuron update fed with
    the current rebuilt from the network's own connectivity, weights and
    raster (Sec. 2 loop items 2.3-2.7);
  * the first consolidation (Table 2's long-term plasticity block) on sampled
    rows: with a decay of 1 the derivative it folds in is the P it leaves
    behind, so every excitatory weight must equal clamp(w + (bias + P)) and
    its D must be 0, and inhibitory weights must not move.  This exercises
    the reverse-to-forward map across the whole 64-bit forward range."""
import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W
from test_gpu_fullsize import _check_one_step

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


def test_paper_largest_grid(dp, orc):
    cfg = W.paper_table1(8, sd_decay=1.0, weight_update_period=200, raster_steps=64)
    N = cfg["grid_x"] * cfg["grid_y"] * cfg["neurons_per_column"]
    M = cfg["synapses_per_neuron"]
    Ne = int(round(cfg["exc_fraction"] * cfg["neurons_per_column"]))
    assert N * M >= 2 ** 32
    _say(f"paper 256x128 grid: building {N * M / 1e9:.2f} G synapses")
    net = dp.Network(cfg)
    try:
        rng = np.random.default_rng(31)
        rows = np.concatenate([rng.integers(0, N, size=12),
                               rng.integers((2 ** 32) // M + 1, N, size=12), [N - 1]])
        for i in rows.tolist():
            tg, dl = net.read_connectivity(i * M, M)
            ref = [orc.synapse(cfg, i, j) for j in range(M)]
            np.testing.assert_array_equal(tg, np.array([r[0] for r in ref], np.uint32))
            np.testing.assert_array_equal(dl, np.array([r[1] for r in ref], np.uint8))
            wv = net.read_weights(i * M, M, P=False, D=False)["w"]
            np.testing.assert_array_equal(wv.view(np.uint32),
                                          np.array([r[2] for r in ref], np.float32).view(np.uint32))
        net.step(25)
        net.sync()
        _say("paper 256x128 grid: sampled neurons of step 25")
        _check_one_step(dp, orc, net, cols=[0, 32767, 20000], per_col=16, seed=5)
        # up to the step before the first consolidation, then through it
        net.step(cfg["weight_update_period"] - 1 - net.t)
        net.sync()
        before = {i: net.read_weights(i * M, M, P=False, D=False) for i in rows.tolist()}
        net.step(1)
        net.sync()
        assert net.stats()["consolidations"] == 1
        bias = np.float32(cfg["wu_bias"])
        wmax = np.float32(cfg["w_max"])
        moved = 0
        for i in rows.tolist():
            a, b = before[i], net.read_weights(i * M, M)
            if i % cfg["neurons_per_column"] < Ne:
                want = np.clip(a["w"] + (bias + b["P"]), np.float32(0.0), wmax).astype(np.float32)
                np.testing.assert_array_equal(b["w"].view(np.uint32), want.view(np.uint32))
                assert not b["D"].any()
                moved += int((b["w"] != a["w"]).sum())
            else:
                np.testing.assert_array_equal(b["w"].view(np.uint32), a["w"].view(np.uint32))
        assert moved > 0
        _say(f"paper 256x128 grid: {net.stats()['spikes']} spikes in {net.t} steps")
    finally:
        net.close()
