"""Data of the paper's single-column observable (Sec. 2, "Production of
observables", Fig. 2-3): a 320 ms raster of one column of 1000 Izhikevich
neurons (80 % RS, 20 % FS) and the membrane-potential traces of individual
neurons, produced on the GPU by the library's state probes.

    python -m paper_1310_8478_amd.figures --out fig23.json

writes the raster (stamps, ids) and the traced v and u as JSON.
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import workloads as W

# two excitatory (RS) neurons, as in the figure, and one inhibitory (FS)
FIG23_PROBES = [117, 512, 903]


def column_trace(warmup_ms: int = 2000, window_ms: int = 320, probes=FIG23_PROBES,
                 device: int = 0, sum_mode: int = W.SUM_FIXED, seed: int = 1310) -> dict:
    """One paper-shaped column (Table 1's 1x1 grid: 1000 neurons, M = 200,
    the paper's projection and drive) stepped warmup_ms steps, then traced for
    window_ms steps: spikes with stamps warmup_ms + 1 .. warmup_ms + window_ms
    and v, u of the probed neurons after each of those steps."""
    from . import dpsnn as dp
    cfg = W.paper_table1(0, sum_mode=sum_mode, seed=seed)
    net = dp.Network(cfg, device=device)
    try:
        net.step(warmup_ms)
        net.set_probes(probes)
        net.step(window_ms)
        net.sync()
        t0, t1 = warmup_ms + 1, warmup_ms + window_ms + 1
        tt, ii = net.read_spikes(t0, t1)
        v, u = net.read_probes(t0, t1)
    finally:
        net.close()
    return dict(config=cfg, warmup_ms=warmup_ms, window_ms=window_ms, probes=list(probes),
                spike_times=tt, spike_ids=ii, v=v, u=u)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--window", type=int, default=320)
    args = ap.parse_args()
    fig = column_trace(args.warmup, args.window)
    rec = {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in fig.items()}
    with open(args.out, "w") as f:
        json.dump(rec, f)
    n = len(fig["spike_times"])
    print(f"{n} spikes in {args.window} ms ({n / 1000 / (args.window / 1000):.1f} Hz); "
          f"traced neurons {fig['probes']}: v range "
          f"{float(fig['v'].min()):.1f} .. {float(fig['v'].max()):.1f} mV")


if __name__ == "__main__":
    main()
