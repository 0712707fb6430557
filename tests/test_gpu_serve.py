"""GPU tests of the continuous-batching job server (dpsnn_server_*).

Bar: every finished job's raster, weights (w, P, D) and state (v, u) equal,
bit for bit, those of the same configuration built and stepped alone; two
small jobs are also checked against the oracle.  Admission respects the byte
budget and the submission order; errors are reported, never fatal.
"""
import ctypes as C
import sys
import time

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


def bits(a):
    return np.ascontiguousarray(a).view(np.uint32)


def snapshot(net, steps):
    tt, ii = net.read_spikes(1, steps + 1)
    syn = net.read_weights()
    v, u = net.read_state()
    return dict(tt=tt, ii=ii, w=syn["w"], P=syn["P"], D=syn["D"], v=v, u=u,
                stats=net.stats())


def solo(dp, cfg, steps):
    c = dict(cfg)
    c["raster_steps"] = max(steps + 1, c["max_delay"] + 1)
    net = dp.Network(c)
    try:
        net.step(steps)
        net.sync()
        return snapshot(net, steps)
    finally:
        net.close()


def assert_same(a, b, what):
    np.testing.assert_array_equal(a["tt"], b["tt"], err_msg=what)
    np.testing.assert_array_equal(a["ii"], b["ii"], err_msg=what)
    for k in ("w", "P", "D", "v", "u"):
        np.testing.assert_array_equal(bits(a[k]), bits(b[k]), err_msg=f"{what}: {k}")
    assert a["stats"]["events"] == b["stats"]["events"], what


# uneven jobs: grid, column size, M, rate, period, mode, target width
JOBS = [
    (W.make_config(grid_x=3, grid_y=3, synapses_per_neuron=120, weight_update_period=100,
                   seed=4001), 260),
    (W.make_config(grid_x=2, grid_y=2, neurons_per_column=400, synapses_per_neuron=60,
                   thalamic_rate=1.7, weight_update_period=50, seed=4002), 120),
    (W.make_config(grid_x=4, grid_y=2, synapses_per_neuron=200, weight_update_period=90,
                   seed=4003), 300),
    (W.make_config(grid_x=2, grid_y=2, neurons_per_column=300, synapses_per_neuron=40,
                   weight_update_period=35, sum_mode=W.SUM_ORDERED, seed=4004), 90),
    (W.make_config(grid_x=1, grid_y=1, neurons_per_column=5200, synapses_per_neuron=30,
                   weight_update_period=70, seed=4005), 150),
    (W.make_config(grid_x=5, grid_y=5, neurons_per_column=250, synapses_per_neuron=80,
                   max_delay=12, thalamic_rate=0.8, weight_update_period=60, seed=4006), 200),
    (W.make_config(grid_x=2, grid_y=3, synapses_per_neuron=100, conn_mode=W.CONN_PAPER,
                   weight_update_period=45, seed=4007), 33),
    (W.make_config(grid_x=2, grid_y=2, neurons_per_column=300, synapses_per_neuron=40,
                   weight_update_period=25, sum_mode=W.SUM_ORDERED, seed=4008), 61),
    (W.make_config(grid_x=3, grid_y=2, synapses_per_neuron=150, weight_update_period=80,
                   seed=4009), 1),
    (W.make_config(grid_x=2, grid_y=2, synapses_per_neuron=100, weight_update_period=100,
                   seed=4010), 410),
]


def run_stream(dp, srv, jobs, first_batch=4):
    """Submit the first jobs at once, the rest while those run; collect."""
    ids = []
    for cfg, steps in jobs[:first_batch]:
        ids.append(srv.submit(cfg, steps))
    srv.wait(ids[0], timeout=120.0)
    for cfg, steps in jobs[first_batch:]:
        ids.append(srv.submit(cfg, steps))
        time.sleep(0.003)
    out = {}
    for j, (cfg, steps) in zip(ids, jobs):
        info = srv.wait(j, timeout=120.0)
        assert info["status"] == dp.JOB_DONE, info
        assert info["steps_launched"] == steps
        assert info["t_submit"] <= info["t_admit"] <= info["t_built"] <= info["t_done"]
        net = srv.job_network(j)
        assert net.t == steps
        out[j] = snapshot(net, steps)
    return ids, out


def test_jobs_equal_solo_runs(dp, orc):
    _say("serve: 10 uneven jobs against solo runs")
    srv = dp.Server(max_quantum=7)
    try:
        ids, got = run_stream(dp, srv, JOBS)
        st = srv.stats()
        assert st["completed"] == len(JOBS) and st["failed"] == 0
        assert st["peak_running"] >= 2, "jobs must have run together"
        for j in ids:
            srv.release(j)
        assert srv.stats()["reserved_bytes"] == 0
    finally:
        srv.close()
    for (cfg, steps), j in zip(JOBS, ids):
        _say(f"  job {j}: solo comparison")
        assert_same(got[j], solo(dp, cfg, steps), f"job {j}")
    # two jobs also against the oracle (ordered fp32 and fixed point)
    for k in (3, 1):
        cfg, steps = JOBS[k]
        n = orc.Net(cfg, steps)
        n.run(steps)
        ot, oi = n.raster()
        s = n.synapses()
        ov, ou = n.state()
        n.close()
        g = got[ids[k]]
        np.testing.assert_array_equal(g["tt"], ot)
        np.testing.assert_array_equal(g["ii"], oi)
        for key, ref in (("w", s["w"]), ("P", s["P"]), ("D", s["D"]), ("v", ov), ("u", ou)):
            np.testing.assert_array_equal(bits(g[key]), bits(ref), err_msg=key)


def test_stream_ordered_allocation_path(dp):
    _say("serve: library allocation (no callbacks)")
    jobs = [JOBS[0], JOBS[3], JOBS[5], JOBS[9]]
    srv = dp.Server(torch_alloc=False, max_quantum=16)
    try:
        ids, got = run_stream(dp, srv, jobs, first_batch=2)
        for j in ids:
            srv.release(j)
    finally:
        srv.close()
    for (cfg, steps), j in zip(jobs, ids):
        assert_same(got[j], solo(dp, cfg, steps), f"job {j}")


def test_budget_admits_in_order(dp):
    _say("serve: budget admits one job at a time, in order")
    jobs = [(W.make_config(grid_x=3, grid_y=3, synapses_per_neuron=120, weight_update_period=60,
                           seed=4100 + k), steps) for k, steps in enumerate((100, 150, 80, 120))]
    fps = [dp.footprint_bytes(dict(c, raster_steps=s + 1)) for c, s in jobs]
    budget = max(fps) + 1
    assert all(a + b > budget for a in fps for b in fps), "the budget must hold one job only"
    srv = dp.Server(budget_bytes=budget, max_quantum=5)
    try:
        ids = [srv.submit(c, s) for c, s in jobs]
        infos = []
        for j in ids:
            infos.append(srv.wait(j, timeout=120.0))
            srv.release(j)   # frees the budget for the next job
        st = srv.stats()
        assert st["peak_running"] == 1
        assert st["peak_reserved_bytes"] <= budget
        admits = [i["t_admit"] for i in infos]
        assert admits == sorted(admits)
        for a, b in zip(infos, infos[1:]):
            assert b["t_admit"] >= a["t_done"]
        with pytest.raises(dp.DpsnnError) as e:
            srv.submit(W.make_config(grid_x=8, grid_y=8, synapses_per_neuron=400), 10)
        assert e.value.code == dp.E_NOMEM
    finally:
        srv.close()


def test_errors_and_ownership(dp):
    _say("serve: errors, timeouts and ownership")
    srv = dp.Server(max_quantum=8)
    try:
        with pytest.raises(dp.DpsnnError) as e:
            srv.submit(W.tiny(max_delay=40), 10)
        assert e.value.code == dp.E_INVAL
        with pytest.raises(dp.DpsnnError) as e:
            srv.submit(W.tiny(), 0)
        assert e.value.code == dp.E_INVAL
        long_job = srv.submit(W.tiny(), 3000)
        with pytest.raises(dp.DpsnnError) as e:
            srv.release(long_job)
        assert e.value.code == dp.E_INVAL
        with pytest.raises(dp.DpsnnError) as e:
            srv.wait(long_job, timeout=0.0)
        assert e.value.code == dp.E_TIMEOUT
        assert srv.query(long_job)["status"] in (dp.JOB_QUEUED, dp.JOB_RUNNING)
        short = srv.submit(W.tiny(), 20)
        first = srv.wait_any(timeout=120.0)
        assert first is not None and first["id"] == short
        info = srv.wait(long_job, timeout=120.0)
        assert info["status"] == dp.JOB_DONE
        # collected by wait(): wait_any does not hand it out a second time
        assert srv.wait_any(timeout=0.05) is None
        # a job's network is freed by the server only
        net = srv.job_network(long_job)
        dp.lib().dpsnn_destroy(net.h)
        assert "server" in dp.lib().dpsnn_last_error().decode()
        assert len(net.read_spikes(2990, 3001)[0]) > 0
        # finished networks can be stepped further by the client
        net.step(5)
        net.sync()
        assert net.t == 3005
        srv.release(long_job)
        srv.release(short)
        with pytest.raises(dp.DpsnnError):
            srv.release(short)
        with pytest.raises(dp.DpsnnError):
            srv.query(short)
    finally:
        srv.close()


def test_shutdown_with_jobs_in_flight(dp):
    _say("serve: destroy with queued and running jobs")
    srv = dp.Server(max_quantum=4)
    ids = [srv.submit(W.tiny(seed=5000 + k), 2000) for k in range(6)]
    time.sleep(0.05)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 60.0
    assert len(ids) == 6
    # the device is still usable afterwards
    got = solo(dp, W.tiny(), 30)
    assert len(got["tt"]) > 0


def test_mixed_summation_modes(dp):
    # fixed-point, ordered and atomic jobs in one server: three groups step
    # side by side; the reproducible ones equal their solo runs, the atomic
    # one delivers exactly the events its raster implies
    _say("serve: fixed, ordered and atomic jobs together")
    jobs = [JOBS[0], JOBS[3],
            (dict(JOBS[2][0], sum_mode=W.SUM_ATOMIC), 180),
            (dict(JOBS[9][0], sum_mode=W.SUM_ATOMIC), 120)]
    srv = dp.Server(max_quantum=6)
    try:
        ids, got = run_stream(dp, srv, jobs, first_batch=4)
        dlys = {}
        for j, (cfg, steps) in zip(ids, jobs):
            if cfg["sum_mode"] == W.SUM_ATOMIC:
                dlys[j] = srv.job_network(j).read_connectivity()[1]
            srv.release(j)
    finally:
        srv.close()
    for (cfg, steps), j in zip(jobs, ids):
        g = got[j]
        if cfg["sum_mode"] != W.SUM_ATOMIC:
            assert_same(g, solo(dp, cfg, steps), f"job {j}")
            continue
        M = cfg["synapses_per_neuron"]
        d = dlys[j].reshape(-1, M).astype(np.int64)
        cum = np.stack([(d <= k).sum(axis=1) for k in range(cfg["max_delay"] + 1)], axis=1)
        lim = np.minimum(steps - g["tt"].astype(np.int64), cfg["max_delay"])
        ok = lim >= 1
        assert g["stats"]["events"] == int(cum[g["ii"][ok].astype(np.int64), lim[ok]].sum())


def test_cancel_running_and_queued_jobs(dp):
    # a long job is cancelled while it runs, another while it waits for
    # memory: both become FAILED (E_CANCELED), their memory returns to the
    # budget on release, and the jobs that ran beside them equal their solo
    # runs bit for bit
    _say("serve: cancel a running and a queued job")
    long_cfg = W.make_config(grid_x=4, grid_y=4, synapses_per_neuron=200, seed=4101,
                             raster_steps=1024)
    keep = [JOBS[0], JOBS[2], JOBS[5]]
    fp_long = dp.footprint_bytes(long_cfg)
    fp_keep = sum(dp.footprint_bytes(dict(c, raster_steps=max(s + 1, c["max_delay"] + 1)))
                  for c, s in keep)
    # the budget holds the long job and the kept jobs, not a second long job
    srv = dp.Server(max_quantum=4, budget_bytes=fp_long + fp_keep + (64 << 20))
    try:
        j_long = srv.submit(long_cfg, 200000)
        ids = [srv.submit(c, s) for c, s in keep]
        j_queued = srv.submit(long_cfg, 100)   # waits: no room beside j_long
        t0 = time.time()
        while srv.query(j_long)["steps_launched"] < 50:
            assert time.time() - t0 < 60, "the long job did not start"
            time.sleep(0.01)
        assert srv.query(j_queued)["status"] == dp.JOB_QUEUED
        srv.cancel(j_queued)
        info = srv.query(j_queued)
        assert info["status"] == dp.JOB_FAILED and info["error"] == dp.E_CANCELED
        srv.cancel(j_long)
        info = srv.wait(j_long, timeout=60.0)
        assert info["status"] == dp.JOB_FAILED and info["error"] == dp.E_CANCELED
        assert info["steps_launched"] < 200000
        with pytest.raises(dp.DpsnnError) as e:
            srv.cancel(j_long)            # already finished
        assert e.value.code == dp.E_INVAL
        before = srv.stats()["reserved_bytes"]
        srv.release(j_long)
        srv.release(j_queued)
        assert before - srv.stats()["reserved_bytes"] == info["footprint"]
        got = {}
        for j, (c, s) in zip(ids, keep):
            i = srv.wait(j, timeout=120.0)
            assert i["status"] == dp.JOB_DONE, i
            got[j] = snapshot(srv.job_network(j), s)
        # wait() collected them: wait_any returns only the uncollected ones
        assert srv.wait_any(timeout=0.0) is None
        for j in ids:
            srv.release(j)
        assert srv.stats()["reserved_bytes"] == 0
    finally:
        srv.close()
    for j, (c, s) in zip(ids, keep):
        assert_same(got[j], solo(dp, c, s), f"job {j} beside the cancelled ones")
