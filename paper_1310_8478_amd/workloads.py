"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds configuration presets and seeded input generators only; it
contains none of the simulation's arithmetic.  The paper's workloads are
themselves synthetic (Sec. 2: a 2-D grid of columns of Izhikevich neurons with
a statistical thalamic input), so nothing here stands in for a dataset.

Field meanings follow the paper: grid CFX x CFY of columns and events per ms
per column (Sec. 2, "Distributed generation of reproducible connections"),
M forward synapses per neuron with delays 1..20 ms (Sec. 2, "Projection of
synapses"), 80 % RS / 20 % FS neurons (Sec. 2, "Spiking neuron model").
"""
from __future__ import annotations

import numpy as np

SUM_ORDERED = 0   # fp32 left fold in canonical order (bit-exact mode)
SUM_ATOMIC = 1    # fp32 atomics, unordered (statistical mode, GPU only)
SUM_FIXED = 2     # fixed-point int64 exact sum (bit-exact and order-free)

CONN_CONFIG = 0   # own_fraction to the own column, rest uniform over 12 neighbours
CONN_PAPER = 1    # 76 % own, 3/2/1 % to each first/second/third neighbour

_BASE = dict(
    grid_x=2, grid_y=2, neurons_per_column=1250, exc_fraction=0.8,
    synapses_per_neuron=100, conn_mode=CONN_CONFIG, own_fraction=0.5,
    max_delay=20, w_exc_init=6.0, w_inh=-5.0, w_max=10.0,
    a_plus=0.1, a_minus=0.12, tau_plus=20.0, tau_minus=20.0,
    weight_update_period=1000, wu_bias=0.01, sd_decay=0.9,
    thalamic_rate=1.0, thalamic_current=20.0, seed=1310,
    sum_mode=SUM_FIXED, raster_steps=0,
)


def make_config(**over) -> dict:
    cfg = dict(_BASE)
    for k, v in over.items():
        if k not in cfg:
            raise KeyError(f"unknown config field {k!r}")
        cfg[k] = v
    return cfg


def _preset(base: dict, over: dict) -> dict:
    cfg = dict(base)
    cfg.update(over)
    return make_config(**cfg)


def tiny(**over) -> dict:
    """2x2 columns x 1250 neurons, M = 100 (0.5 M synapses), 1000 ms."""
    return _preset(dict(grid_x=2, grid_y=2, synapses_per_neuron=100), over)


def mid(**over) -> dict:
    """24x24 columns x 1250 neurons (720 k neurons), M = 200 (144 M synapses)."""
    return _preset(dict(grid_x=24, grid_y=24, synapses_per_neuron=200), over)


def large(**over) -> dict:
    """64x64 columns x 1250 neurons (5.12 M neurons), M = 625 (3.2 G synapses)."""
    return _preset(dict(grid_x=64, grid_y=64, synapses_per_neuron=625), over)


def paper_shaped(grid=(4, 4), M=200, **over) -> dict:
    """The paper's own scaling workload: 1000-neuron columns, M = 200, 76/12/8/4."""
    return _preset(dict(grid_x=grid[0], grid_y=grid[1], neurons_per_column=1000,
                        synapses_per_neuron=M, conn_mode=CONN_PAPER), over)


WORKLOADS = {
    "tiny": (tiny, 1000),
    "mid": (mid, 1000),
    "large": (large, 1000),
}


def batched_mix(n_nets: int = 32, seed: int = 8478) -> list[dict]:
    """Independent networks of uneven size: square grids of side U{2..16},
    M ~ U{100..400}, thalamic rate ~ U[0.5, 2], seeds 2000 + b."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_nets):
        side = int(rng.integers(2, 17))
        M = int(rng.integers(100, 401))
        rate = float(np.float32(rng.uniform(0.5, 2.0)))
        out.append(make_config(grid_x=side, grid_y=side, synapses_per_neuron=M,
                               thalamic_rate=rate, seed=2000 + b))
    return out


def serving_stream(n_req: int = 400, lam: float = 20.0, seed: int = 8479):
    """Poisson request stream: inter-arrival Exp(lam) seconds; square grid side
    U{4..32}; M ~ U{100..625}; duration ~ U{100..2000} steps; seed 3000 + k."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for k in range(n_req):
        t += float(rng.exponential(1.0 / lam))
        side = int(rng.integers(4, 33))
        M = int(rng.integers(100, 626))
        steps = int(rng.integers(100, 2001))
        reqs.append(dict(arrival=t, steps=steps,
                         config=make_config(grid_x=side, grid_y=side,
                                            synapses_per_neuron=M, seed=3000 + k)))
    return reqs


def stimulus_list(n_neurons: int, n_steps: int, count: int, seed: int,
                  mv_range=(5.0, 40.0)):
    """Seeded external stimulus entries (step, neuron, mV), used by tests that
    force spikes at known times."""
    rng = np.random.default_rng(seed)
    t = rng.integers(0, n_steps, size=count).astype(np.uint32)
    ids = rng.integers(0, n_neurons, size=count).astype(np.uint32)
    mv = rng.uniform(*mv_range, size=count).astype(np.float32)
    return t, ids, mv
