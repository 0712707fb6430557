"""Device memory ownership at the boundary: every device allocation of a
network goes through the caller's allocator callbacks, read-backs take a
bounded scratch that is freed before they return, and an allocator that
fails part-way through a build leaves nothing allocated."""
import ctypes as C
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
    """PyTorch's caching allocator behind callbacks that log every call and
    can be told to fail (return NULL) on their k-th allocation."""

    def __init__(self, dp, fail_at=None):
        import torch
        self.live = {}
        self.log = []          # sizes of the allocations, in order
        self.calls = 0
        self.fail_at = fail_at

        def _alloc(nbytes, stream, ctx):
            self.calls += 1
            if self.fail_at is not None and self.calls == self.fail_at:
                return None
            p = int(torch.cuda.caching_allocator_alloc(int(nbytes), device=0, stream=stream or 0))
            self.live[p] = int(nbytes)
            self.log.append(int(nbytes))
            return p

        def _free(p, nbytes, stream, ctx):
            if p:
                assert self.live.pop(int(p)) == int(nbytes), "freed with another size"
                torch.cuda.caching_allocator_delete(int(p))

        self.alloc = dp.ALLOC_FN(_alloc)
        self.free = dp.FREE_FN(_free)


def test_read_scratch_is_bounded_and_goes_through_the_allocator(dp):
    # the large workload's column shape (1250 neurons, M = 625: 3.1 MB of P
    # per column) on a 4x4 grid
    cfg = W.large(grid_x=4, grid_y=4)
    _say("read-back scratch through the callbacks, 4x4 grid of large columns")
    ca = CountingAllocator(dp)
    net = dp.Network(cfg, allocator=ca)
    try:
        net.step(60)
        net.sync()
        built = len(ca.log)
        footprint = dp.footprint_bytes(cfg)
        assert sum(ca.live.values()) <= footprint
        # 200 synapses of one row: one scratch of P for one column + staging
        r = net.read_weights(7 * 1250 * 625 + 300 * 625, 200)
        assert len(ca.log) == built + 1, ca.log[built:]
        colb = 1250 * 625 * 4
        assert ca.log[-1] <= colb + (1 << 20), ca.log[-1]
        assert sum(ca.live.values()) <= footprint, "scratch must be freed"
        # the whole network: groups of columns, never more than the bound
        full = net.read_weights()
        assert len(ca.log) == built + 2
        assert ca.log[-1] <= (32 << 20) + (8 << 20) + 4096, ca.log[-1]
        for k in ("w", "P", "D"):
            np.testing.assert_array_equal(full[k][7 * 1250 * 625 + 300 * 625:][:200].view(np.uint32),
                                          r[k].view(np.uint32))
        assert (full["P"] != 0).any() and (full["D"] != 0).any()
        # connectivity reads stage only
        net.read_connectivity(5 * 625, 1000)
        assert ca.log[-1] <= 1000 * 5 + 4096
        # a checkpoint takes its P buffer through the callbacks too
        n0 = len(ca.log)
        buf = net.save()
        assert len(ca.log) == n0 + 1 and ca.log[-1] <= (1 << 30)
        assert sum(ca.live.values()) <= footprint
        ca2 = CountingAllocator(dp)
        back = dp.Network.load(buf, allocator=ca2)
        try:
            rb = back.read_weights(7 * 1250 * 625 + 300 * 625, 200)
            for k in ("w", "P", "D"):
                np.testing.assert_array_equal(rb[k].view(np.uint32), r[k].view(np.uint32))
        finally:
            back.close()
        assert not ca2.live, "a closed network leaves nothing allocated"
    finally:
        net.close()
    assert not ca.live, "a closed network leaves nothing allocated"


def test_failing_allocator_during_build(dp):
    # an allocator that returns NULL on its k-th call, for every k of a
    # build: DPSNN_E_NOMEM, and every block allocated before it is freed
    cfg = W.tiny(sum_mode=W.SUM_ORDERED)
    ok = CountingAllocator(dp)
    net = dp.Network(cfg, allocator=ok)
    n_build = len(ok.log)
    net.close()
    assert not ok.live
    _say(f"failing allocator: {n_build} allocations in a build")
    assert n_build > 20
    for k in range(1, n_build + 1):
        ca = CountingAllocator(dp, fail_at=k)
        with pytest.raises(dp.DpsnnError) as e:
            dp.Network(cfg, allocator=ca)
        assert e.value.code == dp.E_NOMEM, (k, e.value)
        assert not ca.live, f"allocation {k} failed: {len(ca.live)} blocks left"
    # and a failure inside a read-back is reported, with nothing left over
    ca = CountingAllocator(dp)
    net = dp.Network(cfg, allocator=ca)
    try:
        net.step(20)
        ca.fail_at = ca.calls + 1
        with pytest.raises(dp.DpsnnError) as e:
            net.read_weights()
        assert e.value.code == dp.E_NOMEM
        ca.fail_at = None
        net.read_weights()           # works again
    finally:
        net.close()
    assert not ca.live
