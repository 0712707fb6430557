"""Independent test-side references used to pin the oracle.

* brute_force(): a dense, clock-driven re-derivation of the step for tiny
  networks.  Currents come from dense per-delay weight matrices and a full
  spike matrix (no spike queues, no per-neuron delay lists); fixed-point sums
  use Python's exact integers and its own rounding; STDP pairs are found by
  scanning the spike matrix.
* stdp_posthoc(): recomputes P, D and w from a raster and the connectivity
  alone, with a per-synapse state machine advanced in time order
  (stdp_posthoc_synapses: the same for a chosen set of synapses).

Both follow the paper's definitions (Sec. 2: Izhikevich neuron with two 0.5 ms
sub-steps, delayed injection at t_i + D, STDP dt = t_post - t_pre - d) and the
readings listed with the oracle.
"""
from __future__ import annotations

import math

import numpy as np

F = np.float32


def tables(cfg, n=4096):
    """STDP amplitudes A exp(-dt/tau), evaluated in fp64 with the C library's
    exp (math.exp), rounded to fp32, subnormal results flushed to 0."""
    tp = np.zeros(n, dtype=np.float32)
    tm = np.zeros(n, dtype=np.float32)
    fmin = np.finfo(np.float32).tiny
    for k in range(n):
        a = F(float(F(cfg["a_plus"])) * math.exp(-k / float(F(cfg["tau_plus"]))))
        b = F(float(F(cfg["a_minus"])) * math.exp(-k / float(F(cfg["tau_minus"]))))
        tp[k] = a if abs(a) >= fmin else F(0)
        tm[k] = b if abs(b) >= fmin else F(0)
    return tp, tm


def qfix(x) -> int:
    """x rounded to a multiple of 2^-32 (ties to even), as an integer count."""
    return round(float(F(x)) * 4294967296.0)


def dqfix(a: int):
    """Nearest fp32 to a * 2^-32 (a is exact in fp64 for the sizes used)."""
    return F(float(a) / 4294967296.0)


def _izh(v, u, I, a, b, c, d):
    v, u, I = F(v), F(u), F(I)
    for _ in range(2):
        e = F(F(0.04) * v)
        e = F(e * v)
        e = F(e + F(F(5.0) * v))
        e = F(e + F(140.0))
        e = F(e - u)
        e = F(e + I)
        v = F(v + F(F(0.5) * e))
    u = F(u + F(F(a) * F(F(F(b) * v) - u)))
    fired = bool(v >= F(30.0))
    if fired:
        v = F(c)
        u = F(u + F(d))
    return v, u, fired


def brute_force(orc, cfg, T, stim=None):
    """Returns raster (list of (stamp, id)), w, P, D (canonical) and v, u."""
    Ncol = cfg["neurons_per_column"]
    C = cfg["grid_x"] * cfg["grid_y"]
    N, M, Dmax = C * Ncol, cfg["synapses_per_neuron"], cfg["max_delay"]
    Ne = orc.exc_per_column(cfg)
    tgt = np.zeros((N, M), dtype=np.int64)
    dly = np.zeros((N, M), dtype=np.int64)
    w = np.zeros((N, M), dtype=np.float32)
    for i in range(N):
        for j in range(M):
            tgt[i, j], dly[i, j], w[i, j] = orc.synapse(cfg, i, j)
    exc_src = (np.arange(N) % Ncol) < Ne
    P = np.zeros((N, M), dtype=np.float32)
    D = np.zeros((N, M), dtype=np.float32)
    tp, tm = tables(cfg)
    fixed = cfg["sum_mode"] == 2
    S = np.zeros((T + 2, N), dtype=bool)          # S[s, k]: neuron k stamped s
    params = [(0.02, 0.2, -65.0, 8.0) if (k % Ncol) < Ne else (0.1, 0.2, -65.0, 2.0)
              for k in range(N)]
    v = np.array([F(p[2]) for p in params], dtype=np.float32)
    u = np.array([F(F(p[1]) * F(p[2])) for p in params], dtype=np.float32)
    stim = stim or ([], [], [])

    def latest(k, limit):
        for s in range(min(limit, T + 1), 0, -1):
            if S[s, k]:
                return s
        return None

    for t in range(T):
        # LTP for neurons stamped t
        if t >= 1:
            for k in np.nonzero(S[t])[0]:
                for p in range(N):
                    if not exc_src[p]:
                        continue
                    for j in np.nonzero(tgt[p] == k)[0]:
                        tpre = latest(p, t - dly[p, j])
                        if tpre is not None:
                            P[p, j] = F(P[p, j] + tp[t - dly[p, j] - tpre])
        # currents
        if fixed:
            acc = [0] * N
        else:
            acc = [F(0.0)] * N

        def add(k, x):
            if fixed:
                acc[k] += qfix(x)
            else:
                acc[k] = F(acc[k] + F(x))
        for c in range(C):
            for lk in orc.thalamic(cfg, c, t):
                add(c * Ncol + lk, cfg["thalamic_current"])
        for e in range(len(stim[0])):
            if stim[0][e] == t:
                add(int(stim[1][e]), stim[2][e])
        for d in range(1, Dmax + 1):
            s = t - d + 1
            if s < 1:
                continue
            for i in np.nonzero(S[s])[0]:
                for j in range(M):
                    if dly[i, j] != d:
                        continue
                    k = tgt[i, j]
                    add(k, w[i, j])
                    if exc_src[i]:
                        tq = latest(k, t)
                        if tq is not None:
                            D[i, j] = F(D[i, j] + tm[t + 1 - tq])
        # neurons
        for k in range(N):
            I = dqfix(acc[k]) if fixed else acc[k]
            v[k], u[k], fired = _izh(v[k], u[k], I, *params[k])
            if fired:
                S[t + 1, k] = True
        # consolidation
        Tw = cfg["weight_update_period"]
        if Tw and (t + 1) % Tw == 0:
            for i in range(N):
                if not exc_src[i]:
                    continue
                for j in range(M):
                    sd = F(P[i, j] - D[i, j])
                    x = F(w[i, j] + F(F(cfg["wu_bias"]) + sd))
                    if x < F(0):
                        x = F(0)
                    if x > F(cfg["w_max"]):
                        x = F(cfg["w_max"])
                    w[i, j] = x
                    P[i, j] = F(F(cfg["sd_decay"]) * sd)
                    D[i, j] = F(0)
    raster = [(s, k) for s in range(1, T + 1) for k in np.nonzero(S[s])[0]]
    return raster, w.ravel(), P.ravel(), D.ravel(), v, u


def stdp_posthoc(cfg, N, times, ids, tgt, dly, T):
    """P, D and w of every synapse recomputed from the raster and connectivity.

    Per synapse s = (i -> k, d): arrivals happen at first-effect times a = stamp_i + d
    and are processed in step a - 1; post spikes of k stamped t_k potentiate in
    step t_k.  Within a step the order is LTP, then LTD, then consolidation."""
    M = cfg["synapses_per_neuron"]
    return stdp_posthoc_synapses(cfg, times, ids, np.repeat(np.arange(N), M), tgt, dly, T)


def stdp_posthoc_synapses(cfg, times, ids, src, tgt, dly, T):
    """stdp_posthoc for a chosen set of synapses (source, target, delay
    arrays): only the spike stamps of the neurons they join are used, so it
    serves sampled rows of networks too large for the whole arrays."""
    Ncol = cfg["neurons_per_column"]
    Ne = int(math.floor(float(F(cfg["exc_fraction"])) * Ncol + 0.5))
    tp, tm = tables(cfg)
    src = np.asarray(src, dtype=np.int64)
    tgt = np.asarray(tgt, dtype=np.int64)
    dly = np.asarray(dly, dtype=np.int64)
    exc = (src % Ncol) < Ne
    # the neurons involved, renumbered 0 .. n-1
    inv, code = np.unique(np.concatenate([src, tgt]), return_inverse=True)
    csrc, ctgt = code[:len(src)], code[len(src):]
    nS = len(src)
    w = np.where(exc, F(cfg["w_exc_init"]), F(cfg["w_inh"])).astype(np.float32)
    P = np.zeros(nS, dtype=np.float32)
    D = np.zeros(nS, dtype=np.float32)
    NONE = -(1 << 40)
    last_arr = np.full(nS, NONE, dtype=np.int64)          # latest arrival time <= now
    last_post = np.full(len(inv), NONE, dtype=np.int64)   # latest post stamp <= now
    times = np.asarray(times, dtype=np.int64)
    ids = np.asarray(ids, dtype=np.int64)
    pos = np.searchsorted(inv, ids)
    keep = (pos < len(inv)) & (inv[np.minimum(pos, len(inv) - 1)] == ids) & (times < T + 2)
    fired_at = np.zeros((T + 2, len(inv)), dtype=bool)
    fired_at[times[keep], pos[keep]] = True
    # arrivals per step: synapses whose source fired at stamp t - d + 1
    Tw = cfg["weight_update_period"]
    for t in range(T):
        if t >= 1 and fired_at[t].any():
            last_post[fired_at[t]] = t
            m = exc & fired_at[t][ctgt] & (last_arr != NONE)
            # LTP uses arrivals with first effect <= t (registered in earlier steps)
            P[m] = P[m] + tp[t - last_arr[m]]
        s_src = t - dly + 1
        ok = (s_src >= 1)
        arr = np.zeros(nS, dtype=bool)
        arr[ok] = fired_at[s_src[ok], csrc[ok]]
        m = arr & exc & (last_post[ctgt] != NONE)
        D[m] = D[m] + tm[t + 1 - last_post[ctgt[m]]]
        last_arr[arr] = t + 1
        if Tw and (t + 1) % Tw == 0:
            sd = (P - D).astype(np.float32)
            x = (w + (F(cfg["wu_bias"]) + sd)).astype(np.float32)
            x = np.where(x < F(0), F(0), x)
            x = np.where(x > F(cfg["w_max"]), F(cfg["w_max"]), x).astype(np.float32)
            w = np.where(exc, x, w).astype(np.float32)
            P = np.where(exc, (F(cfg["sd_decay"]) * sd).astype(np.float32), P)
            D = np.where(exc, F(0), D).astype(np.float32)
    return w, P, D


# ---------------------------------------------------------------------------
# Statistical parity of an unordered summation mode.  Once weights are not
# integers, runs that sum the same currents in different (all valid) orders
# diverge chaotically, and single bursts decide a run's mean rate (heavy
# tails): the comparison is over an ensemble of seeds, by the median of the
# per-seed rate deviations and by the pooled weight histogram.
# ---------------------------------------------------------------------------
def ensemble_stats(runs_a, runs_b, exc_mask, bins=100, wmax=10.0):
    """runs_*: lists of (n_spikes, raster pair (tt, ii), w) per seed, same
    seeds in the same order.  Returns the median |rate_a / rate_b - 1|, the
    L1 distance of the pooled excitatory-weight histograms (each normalised),
    and the number of seeds whose rasters differ."""
    dev, ha, hb, differ = [], 0, 0, 0
    for (na, ra, wa), (nb, rb, wb) in zip(runs_a, runs_b):
        dev.append(abs(na / nb - 1.0))
        same = len(ra[0]) == len(rb[0]) and (ra[0] == rb[0]).all() and (ra[1] == rb[1]).all()
        differ += 0 if same else 1
        ha = ha + np.histogram(wa[exc_mask], bins=bins, range=(0.0, wmax))[0]
        hb = hb + np.histogram(wb[exc_mask], bins=bins, range=(0.0, wmax))[0]
    l1 = float(np.abs(ha / ha.sum() - hb / hb.sum()).sum())
    return float(np.median(dev)), l1, differ
