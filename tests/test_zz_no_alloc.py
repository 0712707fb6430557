"""dpsnn_read_weights_noalloc: the read of dpsnn_read_weights for callers that
cannot allocate device memory, with its scratch in the library's static
device workspace.  Its output must equal dpsnn_read_weights' bit for bit, on
two calls in a row (the second with a smaller input), and it must make no
allocation through the network's allocator."""
import sys

import numpy as np
import pytest

from paper_1310_8478_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1310_8478_amd import dpsnn
    dpsnn.lib()
    return dpsnn


class CountingAllocator:
    def __init__(self, dp):
        import torch
        self.calls = 0

        def _alloc(nbytes, stream, ctx):
            self.calls += 1
            return int(torch.cuda.caching_allocator_alloc(int(nbytes), device=0, stream=stream or 0))

        def _free(p, nbytes, stream, ctx):
            if p:
                torch.cuda.caching_allocator_delete(int(p))

        self.alloc = dp.ALLOC_FN(_alloc)
        self.free = dp.FREE_FN(_free)


def _same(a, b):
    for k in ("w", "P", "D"):
        np.testing.assert_array_equal(a[k].view(np.uint32), b[k].view(np.uint32), err_msg=k)


def test_noalloc_read_equals_allocating_read(dp):
    # the large workload's column shape on a 4x4 grid (3.1 MB of P per
    # column), then a smaller read, then a different network
    cfg = W.large(grid_x=4, grid_y=4)
    _say("no-allocation read: 4x4 grid of large columns")
    ca = CountingAllocator(dp)
    net = dp.Network(cfg, allocator=ca)
    try:
        net.step(80)
        net.sync()
        S = net.N * net.M
        big = (3 * 1250 * 625 + 17, 9 * 1250 * 625 + 555)   # spans 7 columns
        small = (12 * 1250 * 625 + 40 * 625 + 3, 200)        # part of two rows
        ref_big = net.read_weights(*big)
        ref_small = net.read_weights(*small)
        before = ca.calls
        got_big = net.read_weights(*big, noalloc=True)
        got_small = net.read_weights(*small, noalloc=True)
        assert ca.calls == before, "the no-allocation read called the allocator"
        _same(got_big, ref_big)
        _same(got_small, ref_small)
        assert (ref_big["P"] != 0).any() and (ref_big["D"] != 0).any()
        # the whole network, then one synapse
        _same(net.read_weights(noalloc=True), net.read_weights())
        _same(net.read_weights(S - 1, 1, noalloc=True), net.read_weights(S - 1, 1))
        with pytest.raises(dp.DpsnnError) as e:
            net.read_weights(S - 5, 10, noalloc=True)
        assert e.value.code == dp.E_RANGE
    finally:
        net.close()
    # another network on the same workspace: a smaller column shape
    cfg2 = W.tiny(seed=77, weight_update_period=50)
    net = dp.Network(cfg2)
    try:
        net.step(120)
        net.sync()
        _same(net.read_weights(noalloc=True), net.read_weights())
        _same(net.read_weights(777, 3, noalloc=True), net.read_weights(777, 3))
    finally:
        net.close()


def test_noalloc_rejects_a_column_beyond_the_workspace(dp):
    # one column's P of 10240 x 1000 floats (41 MB) does not fit 32 MiB
    cfg = W.make_config(grid_x=1, grid_y=1, neurons_per_column=10240, synapses_per_neuron=1000,
                        thalamic_rate=0.0)
    net = dp.Network(cfg)
    try:
        with pytest.raises(dp.DpsnnError) as e:
            net.read_weights(0, 10, noalloc=True)
        assert e.value.code == dp.E_INVAL
        assert "workspace" in str(e.value)
        # without P the staging alone fits
        r = net.read_weights(0, 10, P=False, noalloc=True)
        np.testing.assert_array_equal(r["w"], net.read_weights(0, 10, P=False)["w"])
    finally:
        net.close()
