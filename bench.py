"""Benchmark of the DPSNN-STDP 1 ms step on one MI355X.

One bench step is one 1 ms simulation step of the whole hot path: LTP of the
previous step's spikes, delivery + current injection + LTD, the neuron update
with thalamic input and raster, and (every 1000th step) the weight
consolidation.  Inputs are synthetic and seeded (the paper's workloads are
themselves synthetic); the network is generated on the device before timing
and is resident in HBM when the timed region starts.

Prints one JSON line: synaptic events/s over the timed steps, plus the
roofline of the dominant kernel (algorithmic bytes / its average duration,
measured with HIP events on the library's stream) and the CPU oracle's
events/s on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per unit of work, for a plain layout with a 4-byte
# target index, a weight per synapse and a separate delay byte (state that
# stays cache-resident -- spike history, currents, offsets, tables -- is not
# counted).  The device layout stores less than this (a 2-byte target
# window index, no weight for inhibitory synapses, a packed 4-byte
# source/delay entry: 14 / 2 / 12 bytes), so these figures are an upper
# bound of what the kernels must move.
BYTES_EXC_EVENT = 4 + 4 + 8         # target, weight, LTD accumulator read + write
BYTES_INH_EVENT = 4 + 4             # target, weight
BYTES_LTP_VISIT = 4 + 1 + 8         # forward position, delay, P read + write
BYTES_NEURON = 44                   # v, u, current, spike history, latest stamp
BYTES_CONSOLIDATION = 24            # per excitatory synapse: w, P, D

KERNELS = ("ltp", "deliver", "neuron", "wupdate")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_ltp_deliver_large_hbm_traffic.json")


def measured_traffic(workload, steps, first, mode, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when that summary is for another window (workload, timed
    steps, first timed step, summation mode) or for kernel sources that have
    changed since the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sha256"]:
            return None
        if (rec["workload"], rec["steps"], rec["first_timed_step"], rec["sum_mode"]) != (workload, steps, first, mode):
            return None
        return rec["traffic_bytes_per_launch"].get(kernel)
    except (OSError, KeyError, ValueError):
        return None


def _describe(name, cfg):
    return (f"{name}: {cfg['grid_x']}x{cfg['grid_y']} columns x {cfg['neurons_per_column']} "
            f"Izhikevich neurons (80% RS / 20% FS), M={cfg['synapses_per_neuron']} synapses/neuron, "
            f"delays 1-{cfg['max_delay']} ms, STDP, thalamic {cfg['thalamic_rate']:g}/column/ms")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cfg, budget_s: float, evolve: int = 0):
    """The oracle, as it stands, on a 2x2-column patch of the workload (same
    column size, M and constants), on one host core (the calling thread is
    pinned to it): evolved `evolve` steps untimed, so that it is in the same
    activity regime as the timed GPU window, then stepped until about
    budget_s seconds of CPU work; events per second of oracle stepping."""
    from oracle import oracle as O
    patch = dict(cfg)
    patch["grid_x"], patch["grid_y"] = 2, 2
    patch["sum_mode"] = 2
    cap = evolve + 5000
    aff = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
    core = min(aff) if aff else None
    if core is not None:
        os.sched_setaffinity(0, {core})
    try:
        net = O.Net(patch, cap)
        if evolve:
            net.run(evolve)
        c0 = net.counters()
        steps, elapsed = 0, 0.0
        chunk = 5
        while elapsed < budget_s and evolve + steps + chunk <= cap:
            t0 = time.perf_counter()
            net.run(chunk)
            elapsed += time.perf_counter() - t0
            steps += chunk
        c1 = net.counters()
        net.close()
    finally:
        if aff:
            os.sched_setaffinity(0, aff)
    ev = c1["events"] - c0["events"]
    n_neu = 4 * cfg["neurons_per_column"]
    rate = (c1["spikes"] - c0["spikes"]) / n_neu / (steps / 1000.0) if steps else None
    return {
        "value": ev / elapsed if elapsed > 0 else None, "unit": "synaptic events/s",
        "cores": 1, "kind": "oracle",
        "sample": (f"oracle (plain C, one thread pinned to host core {core}) on a 2x2-column patch of "
                   f"the workload (same column size, M and constants), evolved {evolve} steps "
                   f"untimed, then steps {evolve}..{evolve + steps - 1} timed: {ev} events in "
                   f"{elapsed:.1f} s at {rate:.1f} Hz"),
        "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(),
                 "pinned_core": core},
        "rate_hz": rate,
    }


def _kernel_table(d, bytes_k):
    """Per-kernel launches, average duration, algorithmic bytes per launch and
    achieved GB/s.  When LTP ran inside the delivery launch (k_ltp_deliver,
    the library's default) the delivery timer covers both, so the entry is
    named ltp_deliver and carries the bytes of both."""
    kern = {}
    fused = d["n_ltp"] == 0 and d["n_deliver"] > 0 and bytes_k["ltp"] > 0
    for k in KERNELS:
        ms, n = d[f"ms_{k}"], d[f"n_{k}"]
        if n == 0:
            continue
        name, b = k, bytes_k[k]
        if fused and k == "deliver":
            name, b = "ltp_deliver", bytes_k["deliver"] + bytes_k["ltp"]
        kern[name] = {"launches": n, "total_ms": round(ms, 3), "avg_us": round(1000 * ms / n, 3),
                      "algo_bytes_per_launch": b / n,
                      "achieved_GBs": round(b / (ms / 1000.0) / 1e9, 1) if ms > 0 else None}
    return kern


def run_batched(n_nets, warmup, steps, mode, mode_name):
    """Many independent networks of uneven size advanced together (one launch
    per kernel for all of them), against the same networks stepped one at a
    time.  Both sets start from t = 0 and are timed over the same steps."""
    import torch
    from paper_1310_8478_amd import dpsnn as dp
    from paper_1310_8478_amd import workloads as W

    cfgs = [dict(c, sum_mode=mode) for c in W.batched_mix(n_nets)]
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    nets = [dp.Network(c, device=0) for c in cfgs]
    build_s = time.perf_counter() - t0
    N = sum(n.N for n in nets)
    S = sum(n.N * n.M for n in nets)
    print(f"[bench] built {len(nets)} networks ({N} neurons, {S} synapses) in {build_s:.2f} s",
          file=sys.stderr, flush=True)
    batch = dp.Batch(nets)
    tune_steps = 0
    if warmup >= 36:
        batch.autotune(steps_per_trial=3)       # 2 rounds x 6 shapes x 3 steps
        tune_steps = 36
    if warmup > tune_steps:
        batch.step(warmup - tune_steps)
    batch.set_timing(True)
    s0 = batch.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        k = min(100, steps - done)
        batch.step(k)
        done += k
        if done % 500 == 0 or done == steps:
            torch.cuda.synchronize()
            print(f"[bench] batched {done}/{steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = batch.stats()
    batch.close()
    for n in nets:
        n.close()
    d = {k: s1[k] - s0[k] for k in s1 if isinstance(s1[k], (int, float))}

    # the same networks, stepped one network at a time
    seq = [dp.Network(c, device=0) for c in cfgs]
    for n in seq:
        n.step(warmup)
    torch.cuda.synchronize()
    e0 = sum(n.stats()["events"] for n in seq)
    t0 = time.perf_counter()
    for step in range(steps):
        for n in seq:
            n.step(1)
        if (step + 1) % 500 == 0:
            torch.cuda.synchronize()
            print(f"[bench] one-by-one {step + 1}/{steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall_seq = time.perf_counter() - t0
    e1 = sum(n.stats()["events"] for n in seq)
    for n in seq:
        n.close()

    exc_ev = d["events_exc"]
    inh_ev = d["events"] - exc_ev
    Nexc_syn = sum(int(c["grid_x"] * c["grid_y"] * round(c["exc_fraction"] * c["neurons_per_column"])
                       * c["synapses_per_neuron"]) for c in cfgs)
    bytes_k = {
        "deliver": exc_ev * BYTES_EXC_EVENT + inh_ev * BYTES_INH_EVENT,
        "ltp": d["ltp_visits"] * BYTES_LTP_VISIT,
        "neuron": d["n_neuron"] * N * BYTES_NEURON,
        "wupdate": Nexc_syn * BYTES_CONSOLIDATION * (d["n_wupdate"] / max(1, len(cfgs))),
    }
    kern = _kernel_table(d, bytes_k)
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    ach = kern[dom]["achieved_GBs"]
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4) if ach else None, "traffic": None,
            "kernel": f"k_{dom}", "avg_launch_us": kern[dom]["avg_us"],
            "algo_bytes_per_launch": kern[dom]["algo_bytes_per_launch"]}
    sides = sorted(c["grid_x"] for c in cfgs)
    rate_hz = d["spikes"] / N / (steps / 1000.0)
    return {
        "metric": "synaptic events/s",
        "value": d["events"] / wall,
        "unit": "events/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": 1000.0 * wall / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if mode != W.SUM_FIXED else "f32+i64acc",
        "data": "synthetic (seeded Philox networks and thalamic input, as in the paper)",
        "config": {
            "workload": (f"batched: {len(cfgs)} independent networks, square grids of side "
                         f"{sides[0]}..{sides[-1]} x 1250 neurons, M 100-400, thalamic 0.5-2/column/ms, "
                         f"seeds 2000+b, one launch per kernel for all networks, autotuned shapes"),
            "neurons": N, "synapses": S, "sum_mode": mode_name,
            "timed_steps": f"{warmup}..{warmup + steps - 1}",
        },
        "one_by_one_events_per_s": (e1 - e0) / wall_seq,
        "batch_speedup": (d["events"] / wall) / ((e1 - e0) / wall_seq) if e1 > e0 else None,
        "rate_hz": rate_hz,
        "build_s": build_s,
        "kernels": kern,
        "roofline": roof,
        "first_config": cfgs[0],
    }


def bench_batched(args, mode):
    out = run_batched(args.nets, args.warmup, args.steps, mode, args.mode)
    cfg0 = out.pop("first_config")
    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg0, args.cpu_seconds)
    out["cpu_baseline"] = cpu
    print(json.dumps(out))


def run_serving(reqs, budget_gb, quantum, warmup_jobs, mode, mode_name, jobs_out="", label=""):
    """Continuous-batching serving: a Poisson stream of jobs (uneven networks)
    submitted at their arrival times to a job server that admits them by
    device footprint and steps every admitted job together.  Latency = result
    readable (last step completed) - submission, build included.  Throughput
    = events of all jobs / (last completion - first submission)."""
    import threading

    import numpy as np
    import torch
    from paper_1310_8478_amd import dpsnn as dp
    from paper_1310_8478_amd import workloads as W

    torch.cuda.set_device(0)
    for r in reqs:
        r["config"] = dict(r["config"], sum_mode=mode)
    srv = dp.Server(device=0, budget_bytes=int(budget_gb * 1e9), max_quantum=quantum)
    # warm-up jobs (not timed): load the kernels and fill the allocator's cache
    warm = [srv.submit(W.make_config(grid_x=4, grid_y=4, synapses_per_neuron=300, sum_mode=mode,
                                     seed=9000 + k), 50) for k in range(max(0, warmup_jobs))]
    for j in warm:
        srv.wait(j)
        srv.release(j)
    while srv.wait_any(timeout=0.0) is not None:
        pass

    done = []
    lock = threading.Lock()
    errors = []

    def consume():
        n = 0
        while n < len(reqs):
            info = srv.wait_any(timeout=600.0)
            if info is None:
                errors.append("no job finished within 600 s")
                return
            n += 1
            if info["status"] != dp.JOB_DONE:
                errors.append(f"job {info['id']} failed: {info['message']}")
                srv.release(info["id"])
                continue
            net = srv.job_network(info["id"])
            ev = net.stats()["events"]
            spikes = net.stats()["spikes"]
            srv.release(info["id"])
            with lock:
                done.append(dict(info, events=ev, spikes=spikes, net=None))
            if n % 25 == 0 or n == len(reqs):
                print(f"[bench] serving: {n}/{len(reqs)} jobs done", file=sys.stderr, flush=True)

    th = threading.Thread(target=consume)
    th.start()
    start = time.perf_counter()
    lag = 0.0
    for r in reqs:
        delay = r["arrival"] - (time.perf_counter() - start)
        if delay > 0:
            time.sleep(delay)
        lag = max(lag, (time.perf_counter() - start) - r["arrival"])
        srv.submit(r["config"], r["steps"])
    th.join()
    st = srv.stats()
    srv.close()
    if errors:
        raise RuntimeError("; ".join(errors[:5]))

    if jobs_out:
        with open(jobs_out, "w") as f:
            json.dump([dict(d, grid=reqs[d["id"] - len(warm) - 1]["config"]["grid_x"],
                            M=reqs[d["id"] - len(warm) - 1]["config"]["synapses_per_neuron"])
                       for d in done], f)
    lat = np.array([d["t_done"] - d["t_submit"] for d in done])
    queue_s = np.array([d["t_admit"] - d["t_submit"] for d in done])
    build = np.array([d["t_built"] - d["t_admit"] for d in done])
    first = min(d["t_submit"] for d in done)
    last = max(d["t_done"] for d in done)
    span = last - first
    events = sum(d["events"] for d in done)
    job_steps = sum(r["steps"] for r in reqs)
    syn = [r["config"]["grid_x"] * r["config"]["grid_y"] * r["config"]["neurons_per_column"]
           * r["config"]["synapses_per_neuron"] for r in reqs]
    sides = [r["config"]["grid_x"] for r in reqs]
    durs = [r["steps"] for r in reqs]
    rate = len(reqs) / reqs[-1]["arrival"] if reqs[-1]["arrival"] > 0 else None
    out = {
        "metric": "synaptic events/s",
        "value": events / span,
        "unit": "events/s",
        "n_gpus": 1, "steps": job_steps, "warmup": len(warm),
        "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if mode != W.SUM_FIXED else "f32+i64acc",
        "data": "synthetic (seeded Philox networks and thalamic input, as in the paper)",
        "config": {
            "workload": (f"serving{label}: {len(reqs)} jobs, Poisson arrivals (offered "
                         f"{rate:.2f}/s), square grids of side {min(sides)}..{max(sides)} x 1250 "
                         f"neurons, M 100-625, {min(durs)}-{max(durs)} steps, seeds 3000+k, "
                         f"admission by footprint within {budget_gb:g} GB"),
            "sum_mode": mode_name, "max_quantum": quantum,
            "synapses_per_job_mean": float(np.mean(syn)),
            "events_per_job_mean": events / max(1, len(done)),
        },
        "serve_p50_s": float(np.percentile(lat, 50)),
        "serve_p99_s": float(np.percentile(lat, 99)),
        "serve_max_s": float(lat.max()),
        "queue_wait_mean_s": float(queue_s.mean()),
        "build_mean_s": float(build.mean()),
        "jobs_per_s": len(done) / span,
        "span_s": span,
        "submit_lag_max_s": lag,
        "arrivals_span_s": reqs[-1]["arrival"],
        "peak_running": st["peak_running"],
        "peak_reserved_GB": st["peak_reserved_bytes"] / 1e9,
        "quanta": st["quanta"],
        "roofline": None,
        "cpu_baseline": None,
    }
    return out


def bench_serving(args, mode):
    from paper_1310_8478_amd import workloads as W
    reqs = W.serving_stream(args.requests, lam=args.rate)
    out = run_serving(reqs, args.budget_gb, args.quantum, args.warmup_jobs, mode, args.mode,
                      jobs_out=args.jobs_out)
    print(json.dumps(out))


def bench_consolidation(args, mode):
    """Consolidation alone (Sec. 3, Table 2, "long term synaptic plasticity"):
    Table 1's 128x128 grid and the large workload, consolidating every 40
    steps for 121 steps (three passes), in the one-pass forward form (tuning
    key 14 = 1) and the two-pass form (0), timed by the per-kernel timers."""
    import torch
    from paper_1310_8478_amd import dpsnn as dp
    from paper_1310_8478_amd import workloads as W

    torch.cuda.set_device(0)
    rows = {}
    for name, make in (("paper128", W.paper128), ("large", W.large)):
        cfg = make(weight_update_period=40, sum_mode=mode)
        exc_syn = cfg["grid_x"] * cfg["grid_y"] * round(cfg["exc_fraction"] * cfg["neurons_per_column"]) \
            * cfg["synapses_per_neuron"]
        for key in (1, 0):
            net = dp.Network(cfg, device=0)
            try:
                net.set_tuning(14, key)
                net.set_timing(True)
                net.step(121)
                net.sync()
                st = net.stats()
            finally:
                net.close()
            ms = st["ms_wupdate"] / max(1, st["n_wupdate"])
            gbs = exc_syn * BYTES_CONSOLIDATION / (ms * 1e-3) / 1e9
            rows[f"{name}_{'forward' if key else 'two_pass'}"] = {
                "ms_per_pass": ms, "passes": st["n_wupdate"], "algo_bytes": exc_syn * BYTES_CONSOLIDATION,
                "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
            print(f"[bench] consolidation {name}, key 14 = {key}: {ms:.2f} ms per pass",
                  file=sys.stderr, flush=True)
    head = rows["paper128_forward"]
    print(json.dumps({
        "metric": "consolidation time per pass", "value": head["ms_per_pass"], "unit": "ms",
        "n_gpus": 1, "steps": 121, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if mode != W.SUM_FIXED else "f32+i64acc",
        "data": "synthetic (seeded Philox networks and thalamic input, as in the paper)",
        "config": {"workload": "consolidation every 40 steps, 121 steps: Table 1 128x128 grid and the "
                               "large workload, forward and two-pass forms"},
        "roofline": {"bound": "hbm", "achieved": head["achieved_GBs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["frac"], "traffic": None, "kernel": "k_consolidate"},
        "runs": rows, "cpu_baseline": None}))


def bench_paper(args, mode):
    """The paper's own experiment shapes on one GPU: the Table 1 scaling grids
    (1000-neuron columns, M = 200, 76/12/8/4 % projection) and the Table 3
    synapses-per-neuron sweep, each timed over args.paper_steps steps after
    args.paper_warmup steps of evolution (the paper: 2 s after 8 s)."""
    import torch
    from paper_1310_8478_amd import dpsnn as dp
    from paper_1310_8478_amd import workloads as W

    torch.cuda.set_device(0)

    def run(cfg, label):
        S = cfg["grid_x"] * cfg["grid_y"] * cfg["neurons_per_column"] * cfg["synapses_per_neuron"]
        N = cfg["grid_x"] * cfg["grid_y"] * cfg["neurons_per_column"]
        try:
            dp.footprint_bytes(cfg)
        except dp.DpsnnError as e:
            return {"synapses": S, "skipped": str(e)}
        t0 = time.perf_counter()
        net = dp.Network(cfg, device=0)
        net.sync()
        build_s = time.perf_counter() - t0
        done = 0
        while done < args.paper_warmup:
            k = min(1000, args.paper_warmup - done)
            net.step(k)
            net.sync()
            done += k
            if done % 2000 == 0:
                print(f"[bench] paper {label}: warm-up {done}/{args.paper_warmup}",
                      file=sys.stderr, flush=True)
        s0 = net.stats()
        t0 = time.perf_counter()
        done = 0
        while done < args.paper_steps:
            k = min(500, args.paper_steps - done)
            net.step(k)
            done += k
        net.sync()
        wall = time.perf_counter() - t0
        s1 = net.stats()
        # per-kernel breakdown over the next 200 steps, with the timers on
        net.set_timing(True)
        net.step(200)
        net.sync()
        s2 = net.stats()
        net.close()
        d = {k: s1[k] - s0[k] for k in s1}
        kt = {k: (s2[f"ms_{k}"] - s1[f"ms_{k}"]) / 200.0 for k in KERNELS}
        sim_s = args.paper_steps / 1000.0
        rate = d["spikes"] / N / sim_s
        wps = wall / sim_s
        print(f"[bench] paper {label}: {wps:.4f} wall s per sim s at {rate:.1f} Hz",
              file=sys.stderr, flush=True)
        return {"synapses": S, "neurons": N, "rate_hz": rate, "wall_s_per_sim_s": wps,
                "normalized_s": wps / (rate * S) if rate > 0 else None,
                "events_per_s": d["events"] / wall, "build_s": build_s,
                "kernel_ms_per_step": kt}

    t1 = []
    for k, (gx, gy, rate, wps, norm) in enumerate(W.PAPER_TABLE1):
        r = run(dict(W.paper_table1(k), sum_mode=mode), f"table1 {gx}x{gy}")
        r.update(grid=f"{gx}x{gy}", paper_rate_hz=rate, paper_wall_s_per_sim_s=wps,
                 paper_normalized_s=norm)
        t1.append(r)
    t3 = []
    for k, (M, ncol, gx, gy, rate, rel) in enumerate(W.PAPER_TABLE3):
        r = run(dict(W.paper_table3(k), sum_mode=mode), f"table3 M={M} {ncol}/col {gx}x{gy}")
        r.update(M=M, neurons_per_column=ncol, grid=f"{gx}x{gy}", paper_rate_hz=rate,
                 paper_relative_time=rel)
        t3.append(r)
    base = t3[0].get("normalized_s")
    for r in t3:
        r["relative_time"] = r["normalized_s"] / base if base and r.get("normalized_s") else None
    head = max((r for r in t1 if "events_per_s" in r), key=lambda r: r["synapses"])
    out = {
        "metric": "synaptic events/s",
        "value": head["events_per_s"],
        "unit": "events/s",
        "n_gpus": 1, "steps": args.paper_steps, "warmup": args.paper_warmup,
        "ms_per_step": head["wall_s_per_sim_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if mode != W.SUM_FIXED else "f32+i64acc",
        "data": "synthetic (seeded Philox networks and thalamic input, as in the paper)",
        "config": {
            "workload": (f"paper Table 1 grid {head['grid']} of 1000-neuron columns, M = 200, "
                         f"76/12/8/4 % projection; value is this grid's events/s; the sweep "
                         f"over Table 1 and Table 3 shapes follows"),
            "sum_mode": args.mode,
            "timed_steps": f"{args.paper_warmup}..{args.paper_warmup + args.paper_steps - 1}",
        },
        "paper_table1": t1,
        "paper_table3": t3,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def run_window(net, warmup, steps, label):
    """`warmup` untimed steps, then `steps` steps timed with per-kernel HIP
    event timers; returns the counter differences over the timed steps, the
    wall time and the first timed step."""
    import torch
    done = 0
    while done < warmup:
        n = min(100, warmup - done)
        net.step(n)
        net.sync()
        done += n
    net.set_timing(True)
    first = net.t
    s0 = net.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(100, steps - done)
        net.step(n)
        done += n
        if done % 500 == 0 or done == steps:
            net.sync()
            print(f"[bench] {label}: {done}/{steps} timed steps", file=sys.stderr, flush=True)
    net.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s1 = net.stats()
    net.set_timing(False)
    d = {k: s1[k] - s0[k] for k in s1 if isinstance(s1[k], (int, float))}
    return d, wall, first


def evolve(net, target, label, fuse_after=0xFFFFFFFF):
    """Step the network to `target` completed steps (input preparation, not
    timed).  LTP and delivery run as two kernels here, so that the fused
    kernel's launches in a profile of this run are those of the timed window
    and its warm-up; the results do not depend on the launch shapes."""
    if net.t >= target:
        return
    net.set_tuning(7, 0)
    while net.t < target:
        n = min(1000, target - net.t)
        net.step(n)
        net.sync()
        print(f"[bench] {label}: evolved to step {net.t}", file=sys.stderr, flush=True)
    net.set_tuning(7, fuse_after)


def window_report(cfg, d, wall, steps, first, workload=None, mode=None, measured=False):
    """Throughput, rate and the roofline of the dominant kernel of one timed
    window (the algorithmic bytes per unit above times the window's counted
    work units, divided by the kernel's HIP-event time)."""
    N = cfg["grid_x"] * cfg["grid_y"] * cfg["neurons_per_column"]
    M = cfg["synapses_per_neuron"]
    n_exc_syn = int(cfg["grid_x"] * cfg["grid_y"] *
                    round(cfg["exc_fraction"] * cfg["neurons_per_column"]) * M)
    events, exc_ev = d["events"], d["events_exc"]
    inh_ev = events - exc_ev
    sim_s = steps / 1000.0
    rate_hz = d["spikes"] / N / sim_s
    bytes_k = {
        "deliver": exc_ev * BYTES_EXC_EVENT + inh_ev * BYTES_INH_EVENT,
        "ltp": d["ltp_visits"] * BYTES_LTP_VISIT,
        "neuron": d["n_neuron"] * N * BYTES_NEURON,
        "wupdate": d["n_wupdate"] * n_exc_syn * BYTES_CONSOLIDATION,
    }
    kern = _kernel_table(d, bytes_k)
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    ach = kern[dom]["achieved_GBs"]
    launches = kern[dom]["launches"]
    traffic = None
    if measured:
        traffic = measured_traffic(workload, steps, first, mode, f"k_{dom}")
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4) if ach else None, "traffic": traffic,
            "kernel": f"k_{dom}", "avg_launch_us": kern[dom]["avg_us"],
            "algo_bytes_per_launch": kern[dom]["algo_bytes_per_launch"],
            "units_per_launch": {
                "exc_events": exc_ev / launches if dom in ("deliver", "ltp_deliver") else 0,
                "inh_events": inh_ev / launches if dom in ("deliver", "ltp_deliver") else 0,
                "ltp_visits": d["ltp_visits"] / launches if dom in ("ltp", "ltp_deliver") else 0,
                "neuron_updates": N if dom == "neuron" else 0},
            "bytes_per_unit": {"exc_event": BYTES_EXC_EVENT, "inh_event": BYTES_INH_EVENT,
                               "ltp_visit": BYTES_LTP_VISIT, "neuron": BYTES_NEURON,
                               "consolidation_per_exc_synapse": BYTES_CONSOLIDATION}}
    return {
        "value": events / wall, "ms_per_step": 1000.0 * wall / steps,
        "timed_steps": f"{first}..{first + steps - 1}", "rate_hz": rate_hz,
        "wall_s_per_sim_s": wall / sim_s,
        "wall_s_per_sim_s_per_hz": (wall / sim_s) / rate_hz if rate_hz > 0 else None,
        "events": events, "events_exc": exc_ev, "events_inh": inh_ev,
        "ltp_visits": d["ltp_visits"], "spikes": d["spikes"],
        "kernels": kern, "roofline": roof,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large",
                    choices=["tiny", "mid", "large", "paper128", "batched", "serving", "paper",
                             "consolidation"])
    ap.add_argument("--evolve", type=int, default=None,
                    help="steps the network evolves (untimed) before the warm-up; default 150 "
                         "for large (all-firing from about step 100), 0 otherwise")
    ap.add_argument("--no-startup", action="store_true", help="large: skip the start-up window")
    ap.add_argument("--no-paper-rate", action="store_true",
                    help="large: skip the window on the paper's 128x128 grid at its own rates")
    ap.add_argument("--no-batched", action="store_true",
                    help="large: skip the window on the batched mix of 32 networks")
    ap.add_argument("--no-serving", action="store_true",
                    help="large: skip the job-server window at a load the device carries")
    ap.add_argument("--paper-rate-evolve", type=int, default=8000)
    ap.add_argument("--paper-rate-steps", type=int, default=200)
    ap.add_argument("--nets", type=int, default=32, help="networks in the batched workload")
    ap.add_argument("--requests", type=int, default=400, help="jobs in the serving workload")
    ap.add_argument("--rate", type=float, default=20.0, help="serving arrivals per second")
    ap.add_argument("--budget-gb", type=float, default=240.0, help="serving admission budget")
    ap.add_argument("--quantum", type=int, default=8, help="serving steps per quantum")
    ap.add_argument("--warmup-jobs", type=int, default=4)
    ap.add_argument("--jobs-out", default="", help="serving: write per-job records (JSON) here")
    ap.add_argument("--paper-warmup", type=int, default=8000, help="paper: steps before timing")
    ap.add_argument("--paper-steps", type=int, default=2000, help="paper: timed steps")
    ap.add_argument("--mode", default="fixed", choices=["fixed", "atomic", "ordered"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", default="", help="key=value,... passed to dpsnn_set_tuning")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for scaling HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU halo exchange is a design only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1310_8478_amd import dpsnn as dp
    from paper_1310_8478_amd import workloads as W

    mode = {"fixed": W.SUM_FIXED, "atomic": W.SUM_ATOMIC, "ordered": W.SUM_ORDERED}[args.mode]
    if args.workload == "batched":
        return bench_batched(args, mode)
    if args.workload == "serving":
        return bench_serving(args, mode)
    if args.workload == "paper":
        return bench_paper(args, mode)
    if args.workload == "consolidation":
        return bench_consolidation(args, mode)
    make, _ = W.WORKLOADS[args.workload]
    cfg = make(sum_mode=mode)
    large = args.workload == "large"
    n_evolve = args.evolve if args.evolve is not None else (150 if large else 0)
    torch.cuda.set_device(0)

    tune_kv = [tuple(int(x) for x in kv.split("=")) for kv in filter(None, args.tune.split(","))]
    fuse_after = dict(tune_kv).get(7, 0xFFFFFFFF)

    def tuned(net):
        for k, v in tune_kv:
            net.set_tuning(k, v)
        return net

    t0 = time.perf_counter()
    net = tuned(dp.Network(cfg, device=0))
    net.sync()
    build_s = time.perf_counter() - t0
    print(f"[bench] built {args.workload} in {build_s:.2f} s", file=sys.stderr, flush=True)

    startup = None
    if n_evolve and not args.no_startup:
        # the same network's first steps: the start-up window, from t = 0
        d, wall, first = run_window(net, args.warmup, args.steps, "start-up window")
        startup = window_report(cfg, d, wall, args.steps, first)
        # the step time a caller sees without per-kernel timers (fresh network)
        plain = tuned(dp.Network(cfg, device=0))
        plain.step(args.warmup)
        plain.sync()
        t1 = time.perf_counter()
        plain.step(args.steps)
        plain.sync()
        startup["ms_per_step_without_timers"] = 1000.0 * (time.perf_counter() - t1) / args.steps
        plain.close()
    evolve(net, n_evolve, args.workload, fuse_after)
    d, wall, first = run_window(net, args.warmup, args.steps, "timed window")
    head = window_report(cfg, d, wall, args.steps, first, workload=args.workload, mode=args.mode,
                         measured=True)
    net.close()
    ms_plain = None
    if not n_evolve and head["ms_per_step"] < 2.0:
        net = tuned(dp.Network(cfg, device=0))
        net.step(args.warmup)
        net.sync()
        t1 = time.perf_counter()
        net.step(args.steps)
        net.sync()
        ms_plain = 1000.0 * (time.perf_counter() - t1) / args.steps
        net.close()

    paper_rate = None
    if large and not args.no_paper_rate:
        # the paper's 3.2 G-synapse analogue (Table 1's 128x128 grid of
        # 1000-neuron columns, M = 200, its projection) at its own firing
        # rates, timed after its 8 s warm-up (Sec. 3, measurement protocol)
        pcfg = W.paper_table1(7, sum_mode=mode)
        pnet = tuned(dp.Network(pcfg, device=0))
        evolve(pnet, args.paper_rate_evolve, "paper 128x128", fuse_after)
        pd_, pwall, pfirst = run_window(pnet, args.warmup, args.paper_rate_steps, "paper 128x128")
        paper_rate = window_report(pcfg, pd_, pwall, args.paper_rate_steps, pfirst)
        paper_rate["config"] = {"workload": _describe("paper Table 1 128x128", pcfg),
                                "neurons": pcfg["grid_x"] * pcfg["grid_y"] * 1000,
                                "synapses": pcfg["grid_x"] * pcfg["grid_y"] * 1000 * 200,
                                "evolved_steps": args.paper_rate_evolve}
        pnet.close()

    batched = None
    if large and not args.no_batched:
        # the batched mix: 32 uneven networks in one launch set (41 warm-up
        # steps: 36 of autotuning), against the same networks one at a time
        b = run_batched(32, 41, 200, mode, args.mode)
        b.pop("first_config")
        batched = {k: b[k] for k in ("value", "unit", "ms_per_step", "one_by_one_events_per_s",
                                     "batch_speedup", "rate_hz", "build_s", "roofline", "config")}
    serving = None
    if large and not args.no_serving:
        # the job server at a load it carries: 60 jobs (sides 4..16, 100..500
        # steps) arriving at 4/s, so latency is service time, not queueing
        reqs = W.serving_stream(60, lam=4.0, max_side=16, max_steps=500)
        sv = run_serving(reqs, args.budget_gb, args.quantum, 2, mode, args.mode, label=" (light load)")
        serving = {k: sv[k] for k in ("value", "unit", "serve_p50_s", "serve_p99_s", "serve_max_s",
                                      "queue_wait_mean_s", "build_mean_s", "jobs_per_s", "span_s",
                                      "arrivals_span_s", "peak_running", "config")}
        serving["offered_events_per_s"] = (sv["config"]["events_per_job_mean"] * len(reqs)
                                           / reqs[-1]["arrival"])

    cpu = None
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(cfg, args.cpu_seconds, evolve=n_evolve)

    N = cfg["grid_x"] * cfg["grid_y"] * cfg["neurons_per_column"]
    M = cfg["synapses_per_neuron"]
    regime = None
    if large:
        regime = (f"evolved {n_evolve} steps before the warm-up (the paper times activity after "
                  f"the network has evolved); this workload's constants drive it to fire every "
                  f"neuron every step from about step 100, so that regime is what a 1000 ms job "
                  f"runs in; measured rate {head['rate_hz']:.1f} Hz")
    out = {
        "metric": "synaptic events/s",
        "value": head["value"],
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if mode != W.SUM_FIXED else "f32+i64acc",
        "data": "synthetic (seeded Philox network and thalamic input, as in the paper)",
        "config": {
            "workload": _describe(args.workload, cfg),
            "neurons": N, "synapses": N * M, "sum_mode": args.mode,
            "timed_steps": head["timed_steps"], "evolved_steps": n_evolve,
            "regime": regime,
        },
        "ms_per_step_without_timers": ms_plain,
        "wall_s_per_sim_s_per_hz": head["wall_s_per_sim_s_per_hz"],
        "wall_s_per_sim_s": head["wall_s_per_sim_s"],
        "rate_hz": head["rate_hz"],
        "build_s": build_s,
        "counts": {k: head[k] for k in ("events", "events_exc", "events_inh", "ltp_visits", "spikes")},
        "kernels": head["kernels"],
        "roofline": head["roofline"],
        "startup": startup,
        "paper_rate": paper_rate,
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
