// The 1 ms simulation step (Sec. 2, "Mixed time-driven and event driven
// simulation", loop items 2.1-2.7, and the periodic "long term synaptic
// plasticity" block of Table 2).
//
//   k_ltp      item 2.1: every neuron stamped t potentiates its incoming
//              excitatory synapses; workgroups per target column walk the
//              reverse rows of the column's spiking neurons (contiguous runs);
//              k_ltp_sp is the wavefront-level form for sparse columns.
//   k_deliver  items 2.3-2.6: workgroups per source column deliver the
//              spikes stamped t-d+1 through the column's delay-d synapses,
//              accumulate the currents of the reachable target columns in an
//              LDS window, apply LTD, then flush the window (k_deliver_seq:
//              the ordered-summation form).  k_ltp_deliver runs LTP and
//              delivery as one launch, which is the default.
//   k_neuron   item 2.7 plus the thalamic input: Izhikevich update with two
//              0.5 ms sub-steps, threshold and reset, spike history, and the
//              raster word of each wavefront written with one ballot.
//   k_consolidate  every weight_update_period steps: fold P - D into the
//              weights in one forward-order pass (k_wupdate + k_wupdate_fwd:
//              the two-pass form, for networks without the
//              forward-to-reverse map).
// Every kernel reads its network's step as t = t0 + tstep: t0 from the
// network's descriptor, tstep a launch argument.  k_rebase moves t0 forward,
// which lets one captured graph of G steps be replayed at any step.
#include "net.h"

namespace dpsnn {

namespace {

// entries of the LDS queue of the sparse delivery path (segments or spikes)
constexpr uint32_t kQueue = 1024;

// ---------------------------------------------------------------------------
// LTP (item 2.1).  Synapse (p -> k, delay d), post stamp t: the latest spike
// of p with stamp <= t - d pairs with it, dt = t - d - stamp >= 0 and
// P += A+ exp(-dt / tau+) (Sec. 2, STDP rule).  hist[p] bit b means p was
// stamped t - b, so dt = ctz(hist >> d) when a bit remains; t_old holds the
// latest stamp older than the 32-step window.
// ---------------------------------------------------------------------------
template <int U>
__device__ __forceinline__ void ltp_body(const NetDesc* __restrict__ nds,
                                         const uint2* __restrict__ bmap, uint32_t allow_stage,
                                         uint32_t nparts, uint32_t tstep, uint32_t bid) {
    // workgroup bid: part `part` of the column of map entry bid / nparts
    const uint2 br = bmap[bid / nparts];
    const uint32_t part = bid % nparts;
    const NetDesc& nd = nds[br.x];
    const Dims d = nd.d;
    const uint32_t t = nd.t0 + tstep;
    if (t < 1) return;  // no stamp 0: nothing to potentiate in the first step
    const uint64_t* __restrict__ ring = nd.ring;
    const uint2* __restrict__ hist = nd.hist;
    const uint64_t* __restrict__ rowptr = nd.rowptr;
    const uint32_t* __restrict__ srcmap = nd.srcmap;
    // the target column's reverse rows through pointers offset by their start
    // rounded down to a multiple of 4: 32-bit offsets, aligned quads
    const uint32_t ct = br.y;
    const uint64_t rb = rowptr[(size_t)ct * d.Ncol] & ~3ull;
    const uint32_t* __restrict__ rev_srcd = nd.rev_srcd + rb;
    float* __restrict__ P = nd.Pacc + rb;
    const float* __restrict__ tp = nd.tp;
    const uint32_t tp_len = nd.tp_len;
    DevStats* __restrict__ stats = nd.stats;
    extern __shared__ uint32_t lds[];
    const uint32_t BS = blockDim.x;
    uint32_t* pref = lds;              // [BS + 1]
    uint32_t* x0 = pref + BS + 1;      // [BS]
    uint32_t* sh = x0 + BS;            // [20]
    uint32_t* smap = sh + 20;          // [13]
    float* tph = (float*)(smap + 16);  // [64] first LTP amplitudes
    uint32_t* hwin = smap + 16 + 64;   // [13 * Ncol] when staged
    const uint32_t tid = threadIdx.x;
    const uint64_t* words = ring + ((size_t)(t % d.R) * d.C + ct) * d.W;

    // the column's raster words and the small tables, loaded together
    WordRuns wr{0ull, 0ull, 0ull};
    if (tid < d.W) wr = word_runs(words, d.W, tid, 0u);
    if (tid < kSlots) smap[tid] = srcmap[ct * kSlots + tid];
    if (tid < 64) tph[tid] = tid < tp_len ? tp[tid] : 0.0f;
    const uint32_t cs = (uint32_t)__popcll(wr.starts);
    const uint32_t ce = (uint32_t)__popcll(wr.ends);
    uint32_t nsp;
    (void)block_scan((uint32_t)__popcll(wr.word), sh, nsp);
    if (nsp == 0) return;  // block-uniform
    // the k-th run starts at the k-th start bit and ends at the k-th end bit
    // of the column (runs may span words); starts and ends are counted in one
    // scan (at most 32 of each per word and 1024 words: each half < 2^16)
    uint32_t tot;
    const uint32_t pre = block_scan(cs | (ce << 16), sh, tot);
    uint32_t nruns = tot & 0xFFFFu;
    const uint32_t bs_ = pre & 0xFFFFu, be_ = pre >> 16;
    // stage the 13 source columns' history when the expected visits (spiking
    // targets x about 0.8 M incoming excitatory synapses each) outnumber it
    const bool stage = allow_stage && nparts == 1u &&
                       (uint64_t)nsp * d.M * 4u >= 5ull * kSlots * d.Ncol;
    __syncthreads();
    if (stage) {
        const uint32_t nwin = kSlots * d.Ncol;
        for (uint32_t x = tid; x < nwin; x += BS) {
            const uint32_t q = x / d.Ncol;
            const uint32_t l = x - q * d.Ncol;
            hwin[x] = hist[smap[q] * d.Ncol + l].x;
        }
    }
    unsigned long long visits = 0;
    if (nsp == d.Ncol) {
        // every neuron of the column fired: its reverse rows form one block
        __syncthreads();
        const uint32_t c_lo = (uint32_t)(rowptr[(size_t)ct * d.Ncol] - rb);
        const uint32_t c_hi = (uint32_t)(rowptr[(size_t)(ct + 1) * d.Ncol] - rb);
        const uint32_t x_lo = part_bound4(c_lo, c_hi, part, nparts);
        const uint32_t x_hi = part_bound4(c_lo, c_hi, part + 1u, nparts);
        const uint32_t total = x_hi - x_lo;
        // LTP of one reverse entry: returns the new P
        auto ltp_one = [&](uint32_t sd, float pv) -> float {
            const uint32_t dl = sd & 63u;
            const uint32_t l = (sd >> 6) & 0xFFFFu;
            const uint32_t sl = sd >> 22;
            const uint32_t p = smap[sl] * d.Ncol + l;
            const uint2 ht = stage ? make_uint2(hwin[sl * d.Ncol + l], 0u) : hist[p];
            const uint32_t m = ht.x >> dl;
            uint32_t dt;
            if (m) {
                dt = (uint32_t)__ffs((int)m) - 1u;
            } else {
                const int32_t to = (int32_t)(stage ? hist[p].y : ht.y);
                if (to == kNoSpike) return pv;
                dt = (uint32_t)((int64_t)t - dl - to);
            }
            return pv + (dt < 64u ? tph[dt] : (dt < tp_len ? tp[dt] : 0.0f));
        };
        const uint32_t a0 = min(x_hi, (x_lo + 3u) & ~3u);
        const uint32_t a1 = max(a0, x_hi & ~3u);
        {
            uint32_t x = 0xFFFFFFFFu;
            if (tid < a0 - x_lo) x = x_lo + tid;
            else if (tid >= 64u && tid - 64u < x_hi - a1) x = a1 + (tid - 64u);
            if (x != 0xFFFFFFFFu) P[x] = ltp_one(rev_srcd[x], P[x]);
        }
        constexpr int G = 2;
        struct Grp {
            uint32_t x[G];
            uint4 sd[G];
            float4 pv[G];
            bool ok[G];
        };
        const uint32_t nq = (a1 - a0) >> 2;
        const WaveRange wr_ = wave_range(nq);
        auto load = [&](uint32_t qb, Grp& g) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const uint32_t qi = qb + q * 64u + lane_id();
                g.ok[q] = qi < wr_.end;
                g.x[q] = a0 + 4u * (g.ok[q] ? qi : wr_.begin);
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
                g.sd[q] = g.ok[q] ? *(const uint4*)(rev_srcd + g.x[q]) : make_uint4(0u, 0u, 0u, 0u);
                g.pv[q] = g.ok[q] ? *(const float4*)(P + g.x[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        auto process = [&](Grp& g) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (!g.ok[q]) continue;
                float4 o;
                o.x = ltp_one(g.sd[q].x, g.pv[q].x);
                o.y = ltp_one(g.sd[q].y, g.pv[q].y);
                o.z = ltp_one(g.sd[q].z, g.pv[q].z);
                o.w = ltp_one(g.sd[q].w, g.pv[q].w);
                *(float4*)(P + g.x[q]) = o;
            }
        };
        Grp A, B;
        if (wr_.begin < wr_.end) load(wr_.begin, A);
        for (uint32_t qb = wr_.begin; qb < wr_.end; qb += 2u * 64u * G) {
            const uint32_t nb = qb + 64u * G;
            if (nb < wr_.end) load(nb, B);
            process(A);
            const uint32_t na = nb + 64u * G;
            if (na < wr_.end) load(na, A);
            if (nb < wr_.end) process(B);
        }
        visits = total;
        nruns = 0;  // the run loop below has nothing left to do
    }
    for (uint32_t r0 = 0; r0 < nruns; r0 += BS) {
        {
            unsigned long long m = wr.starts;
            for (uint32_t k = 0; k < cs; ++k) {
                const uint32_t idx = bs_ + k;
                const uint32_t b = (uint32_t)__ffsll((long long)m) - 1u;
                m &= m - 1ull;
                if (idx >= r0 && idx < r0 + BS) x0[idx - r0] = tid * 64u + b;
            }
            m = wr.ends;
            for (uint32_t k = 0; k < ce; ++k) {
                const uint32_t idx = be_ + k;
                const uint32_t b = (uint32_t)__ffsll((long long)m) - 1u;
                m &= m - 1ull;
                if (idx >= r0 && idx < r0 + BS) pref[idx - r0] = tid * 64u + b + 1u;  // exclusive
            }
        }
        __syncthreads();
        const uint32_t nr = min(BS, nruns - r0);
        uint32_t a = 0, len = 0;
        if (tid < nr) {
            const uint32_t le = min(pref[tid], d.Ncol);
            const uint32_t ls = min(x0[tid], le);
            const uint64_t ga = rowptr[(size_t)ct * d.Ncol + ls];
            a = (uint32_t)(ga - rb);
            len = (uint32_t)(rowptr[(size_t)ct * d.Ncol + le] - ga);
        }
        __syncthreads();
        uint32_t E;
        const uint32_t ex = block_scan(len, sh, E);
        if (tid < nr) {
            x0[tid] = a;
            pref[tid] = ex;
        }
        __syncthreads();
        uint32_t plo, phi;
        part_slice(E, part, nparts, plo, phi);
        const WaveRange wr_ = wave_range_in(plo, phi);
        uint32_t cur = wr_.begin < wr_.end ? upper_run(pref, 0u, nr, wr_.begin) : 0u;
        for (uint32_t eb = wr_.begin; eb < wr_.end; eb += 64u * U) {
            uint32_t xs[U], sd[U];
            float pv[U];
            bool ok[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const uint32_t sb = eb + q * 64u;
                const uint32_t e = sb + lane_id();
                ok[q] = e < wr_.end;
                if (sb < wr_.end && cur + 1 < nr && pref[cur + 1] <= sb)
                    cur = upper_run(pref, cur + 1, nr, sb);
                const uint32_t r = ok[q] ? lane_run(pref, cur, nr, e) : 0u;
                xs[q] = ok[q] ? x0[r] + (e - pref[r]) : 0u;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                sd[q] = ok[q] ? rev_srcd[xs[q]] : 0u;
                pv[q] = ok[q] ? P[xs[q]] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                if (!ok[q]) continue;
                const uint32_t dl = sd[q] & 63u;
                const uint32_t l = (sd[q] >> 6) & 0xFFFFu;
                const uint32_t s = sd[q] >> 22;
                const uint32_t p = smap[s] * d.Ncol + l;
                const uint2 ht = stage ? make_uint2(hwin[s * d.Ncol + l], 0u) : hist[p];
                const uint32_t m = ht.x >> dl;
                uint32_t dt;
                if (m) {
                    dt = (uint32_t)__ffs((int)m) - 1u;
                } else {
                    const int32_t to = (int32_t)(stage ? hist[p].y : ht.y);
                    if (to == kNoSpike) continue;
                    dt = (uint32_t)((int64_t)t - dl - to);
                }
                const float a = dt < 64u ? tph[dt] : (dt < tp_len ? tp[dt] : 0.0f);
                P[xs[q]] = pv[q] + a;
            }
        }
        visits += phi - plo;
        __syncthreads();
    }
    if (tid == 0 && visits) atomicAdd(&stats[ct & 63].ltp_visits, visits);
}

template <int U>
__global__ __launch_bounds__(1024) void k_ltp(const NetDesc* __restrict__ nds,
                                              const uint2* __restrict__ bmap, uint32_t allow_stage,
                                              uint32_t nparts, uint32_t tstep) {
    ltp_body<U>(nds, bmap, allow_stage, nparts, tstep, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Delivery, current injection and LTD (items 2.3-2.6).  A spike stamped s
// reaches the synapses of delay d in step s + d - 1 (its current first moves
// the target at s + d, "inject W at t_i + D", Sec. 2).  All spiking sources
// of the column that share a delay occupy contiguous runs of the forward
// array, so each run is one contiguous stretch of (tgt, w, D).  LTD: the
// target's latest stamp t_q <= t precedes the arrival at t + 1, dt = t + 1 -
// t_q, D += A- exp(-dt / tau-).
// ---------------------------------------------------------------------------
// WIN: 0 no LDS window (global atomics), 1 window over all 13 reachable
// columns, 2 window over the own column only (targets in the neighbour
// columns take global atomics; small LDS, several workgroups per CU).
template <bool FIXED, int WIN, typename TgtT, int U>
__device__ __forceinline__ void deliver_body(const NetDesc* __restrict__ nds,
                                             const uint2* __restrict__ bmap,
                                             uint32_t allow_age, uint32_t nparts, uint32_t nsplit,
                                             uint32_t wslots,
                                             unsigned long long* __restrict__ set_events,
                                             uint32_t tstep, uint32_t bid) {
    // workgroup bid: part `part` (a slice of the events) and window share sp
    // of the column of map entry bid / (nparts * nsplit)
    const uint32_t per = nparts * nsplit;
    const uint2 br = bmap[bid / per];
    const uint32_t part = (bid % per) % nparts;
    const uint32_t sp = (bid % per) / nparts;
    const NetDesc& nd = nds[br.x];
    const Dims d = nd.d;
    const uint32_t t = nd.t0 + tstep;
    if (t < 1) return;  // no spike has been stamped yet
    const uint64_t* __restrict__ ring = nd.ring;
    const uint64_t* __restrict__ seg_off = nd.seg_off;
    // the source column's forward block through pointers offset by its start
    // rounded down to a multiple of 4: 32-bit offsets, aligned quads
    const uint64_t fb = ((uint64_t)br.y * d.Ncol * d.M) & ~3ull;
    const TgtT* __restrict__ tgt = (const TgtT*)nd.tgt + fb;
    const float* __restrict__ w = nd.w + fb;
    float* __restrict__ Dacc = nd.Dacc + fb;
    const int32_t* __restrict__ t_last = nd.t_last;
    const uint32_t* __restrict__ colmap = nd.colmap;
    const float* __restrict__ tm = nd.tm;
    const uint32_t tm_len = nd.tm_len;
    void* __restrict__ acc_v = nd.acc;
    DevStats* __restrict__ stats = nd.stats;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ unsigned long long red64[16];
    const uint32_t BS = blockDim.x;
    const uint32_t nwin = kSlots * d.Ncol;
    constexpr bool WINDOW = WIN != 0;
    // with the full window the column's targets may be shared out over nsplit
    // workgroups by slot: this one owns window indices [wlo, wlo + wspan),
    // reads every event of its slice and delivers (and depresses) only the
    // ones whose target it owns
    const uint32_t s_lo = WIN == 1 ? (sp * kSlots) / nsplit : 0u;
    const uint32_t s_hi = WIN == 1 ? ((sp + 1u) * kSlots) / nsplit : (uint32_t)kSlots;
    const uint32_t wlo = s_lo * d.Ncol;
    const uint32_t wspan = (s_hi - s_lo) * d.Ncol;
    auto own = [&](uint32_t wi) { return wi - wlo < wspan; };
    // the partial window (WIN 2) covers the first wslots slots: the own
    // column, then the nearest neighbour rings
    const uint32_t nlds = WIN == 1 ? wspan : (WIN == 2 ? wslots * d.Ncol : 0u);  // window entries
    // the window sums in fixed point in both modes: integer LDS atomics are
    // several times faster than fp32 LDS atomics on this GPU; the unordered
    // fp32 mode rounds each column's exact partial sum to fp32 once, at the
    // flush, and adds it to the target with a float atomic
    const size_t win_bytes = (((size_t)nlds * 8) + 15) & ~(size_t)15;
    // age window: steps since each reachable target's latest spike, saturated
    // at 255 (255 also means "never" or "look it up"); staged when the
    // workgroup has enough events to reuse it
    uint8_t* age = lds_raw + win_bytes;
    // the age window covers the LDS current window's slots with the partial
    // window (WIN 2), else every slot this workgroup owns
    const uint32_t aspan = WIN == 2 ? nlds : wspan;
    const size_t age_bytes = allow_age ? (((size_t)aspan + 15) & ~(size_t)15) : 0;
    uint32_t* pref = (uint32_t*)(lds_raw + win_bytes + age_bytes);  // [BS + 1]
    uint32_t* pos0 = pref + BS + 1;                      // [BS]
    uint32_t* excf = pos0 + BS;                          // [BS]
    uint32_t* sh = excf + BS;                            // [20]
    uint32_t* cmap = sh + 20;                            // [13]
    float* tmh = (float*)(cmap + 16);                    // [64] first LTD amplitudes
    const uint32_t tid = threadIdx.x;
    const uint32_t c = br.y;
    long long* win64 = (long long*)lds_raw;
    long long* acc64 = (long long*)acc_v;
    float* acc32 = (float*)acc_v;

    if (WINDOW) {
        for (uint32_t x = tid; x < nlds; x += BS) {
            win64[x] = 0;
        }
    }
    if (tid < kSlots) cmap[tid] = colmap[c * kSlots + tid];
    if (tid < 64) tmh[tid] = tid < tm_len ? tm[tid] : 0.0f;

    const long long q_inh = to_fixed(d.w_inh);
    const uint32_t split = (d.Ne > 0 && d.Ne < d.Ncol) ? d.Ne : 0u;
    // tasks (delay, raster word) are taken a whole number of delays at a time
    // (the host keeps W <= BS), so that no run is split between two chunks;
    // this thread's word of the first chunk is loaded here, together with the
    // tables above, and serves both the all-firing test and the run decoding
    const uint32_t dpc = max(1u, BS / d.W);
    const uint32_t nd0 = min(dpc, d.Dmax);
    const int64_t s0 = (int64_t)t - (int64_t)(1u + tid / d.W) + 1;
    const bool live0 = tid < nd0 * d.W && s0 >= 1;
    WordRuns wr0{0ull, 0ull, 0ull};
    if (live0)
        wr0 = word_runs(ring + ((size_t)((uint64_t)s0 % d.R) * d.C + c) * d.W, d.W,
                        tid - (tid / d.W) * d.W, split);
    unsigned long long ev_local = 0, exc_events = 0;  // this thread's deliveries
    bool staged = false;
    // the column's inhibitory synapses (all of delay 1) form one forward range
    const size_t s1 = (size_t)c * d.segs;
    const uint32_t inh_lo = d.Ne < d.Ncol ? (uint32_t)(seg_off[s1 + d.Ne] - fb) : 0u;
    const uint32_t inh_hi = d.Ne < d.Ncol ? (uint32_t)(seg_off[s1 + d.Ncol] - fb) : 0u;
    auto is_exc = [&](uint32_t p) { return !(p >= inh_lo && p < inh_hi); };
    auto global_id = [&](uint32_t wi) {
        const uint32_t sl = sizeof(TgtT) == 2 ? div_ncol(d, wi) : wi / d.Ncol;
        return cmap[sl] * d.Ncol + (wi - sl * d.Ncol);
    };
    // one delivery to window index wi with weight wv (excitatory: ex), and
    // its LTD added to dv
    auto deliver_one = [&](bool ex, uint32_t wi, float wv, float& dv) {
        if (!own(wi)) return;
        ++ev_local;
        exc_events += ex ? 1u : 0u;
        if (WIN == 1 || (WIN == 2 && wi < nlds)) {
            atomicAdd((unsigned long long*)&win64[wi - wlo],
                      (unsigned long long)(ex ? to_fixed(wv) : q_inh));
        } else {
            if (FIXED) {
                atomicAdd((unsigned long long*)&acc64[global_id(wi)],
                          (unsigned long long)(ex ? to_fixed(wv) : q_inh));
            } else {
                atomicAdd(&acc32[global_id(wi)], ex ? wv : d.w_inh);
            }
        }
        if (ex) {
            const uint32_t ag = (staged && wi - wlo < aspan) ? age[wi - wlo] : 255u;
            uint32_t dt = 0xFFFFFFFFu;
            if (ag < 255u) {
                dt = ag + 1u;
            } else {
                const int32_t tq = t_last[global_id(wi)];
                if (tq != kNoSpike) dt = (uint32_t)((int64_t)t + 1 - tq);
            }
            if (dt != 0xFFFFFFFFu)
                dv = dv + (dt < 64u ? tmh[dt] : (dt < tm_len ? tm[dt] : 0.0f));
        }
    };

    // Dense case: every neuron of the column fired in each of the last Dmax
    // steps, so every synapse of the column delivers and the events are the
    // column's whole contiguous block of the forward arrays.
    int full = (t >= d.Dmax) ? 1 : 0;
    if (full) {
        const uint32_t tail = d.Ncol - (d.W - 1u) * 64u;
        const unsigned long long last = tail >= 64u ? ~0ull : ((1ull << tail) - 1ull);
        for (uint32_t x = tid; x < d.Dmax * d.W; x += BS) {
            const uint32_t dd = x / d.W + 1u, wd = x - (dd - 1u) * d.W;
            const uint64_t word = (x == tid && live0)
                                      ? wr0.word
                                      : ring[((size_t)((t - dd + 1u) % d.R) * d.C + c) * d.W + wd];
            if (word != (wd + 1u == d.W ? last : ~0ull)) full = 0;
        }
    }
    __syncthreads();
    full = __syncthreads_and(full);
    if (full) {
        const uint32_t c0 = (uint32_t)((uint64_t)c * d.Ncol * d.M - fb);
        const uint32_t cb = part_bound4(c0, c0 + d.Ncol * d.M, part, nparts);
        const uint32_t total = part_bound4(c0, c0 + d.Ncol * d.M, part + 1u, nparts) - cb;
        if (allow_age && total >= aspan) {  // block-uniform
            for (uint32_t x = tid; x < aspan; x += BS) {
                const uint32_t xw = x + wlo;
                const uint32_t sl = sizeof(TgtT) == 2 ? div_ncol(d, xw) : xw / d.Ncol;
                const int32_t tq = t_last[cmap[sl] * d.Ncol + (xw - sl * d.Ncol)];
                const int64_t ag = (tq == kNoSpike) ? 255 : (int64_t)t - tq;
                age[x] = (uint8_t)(ag < 255 ? ag : 255);
            }
            staged = true;
        }
        __syncthreads();
        // unaligned head and tail (at most 3 positions each), one lane each
        const uint32_t fin = cb + total;
        const uint32_t a0 = min(fin, (cb + 3u) & ~3u);
        const uint32_t a1 = max(a0, fin & ~3u);
        {
            uint32_t p = 0xFFFFFFFFu;
            if (tid < a0 - cb) p = cb + tid;
            else if (tid >= 64u && tid - 64u < fin - a1) p = a1 + (tid - 64u);
            if (p != 0xFFFFFFFFu) {
                const bool ex = is_exc(p);
                const uint32_t wi = (uint32_t)tgt[p];
                float dv = ex ? Dacc[p] : 0.0f;
                deliver_one(ex, wi, ex ? w[p] : d.w_inh, dv);
                if (ex && own(wi)) Dacc[p] = dv;
            }
        }
        // aligned body: four consecutive positions per lane, vector loads
        constexpr int G = 2;
        struct Grp {
            uint32_t p[G];
            uint2 ti[G];
            float4 wv[G], dv[G];
            bool ok[G];
            uint32_t exm[G];  // bit k: position p + k is excitatory
        };
        const uint32_t nq = (a1 - a0) >> 2;
        const WaveRange wr_ = wave_range(nq);
        auto load = [&](uint32_t qb, Grp& g) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                const uint32_t qi = qb + q * 64u + lane_id();
                g.ok[q] = qi < wr_.end;
                g.p[q] = a0 + 4u * (g.ok[q] ? qi : wr_.begin);
                uint32_t m = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) m |= (is_exc(g.p[q] + k) ? 1u : 0u) << k;
                g.exm[q] = g.ok[q] ? m : 0u;
            }
#pragma unroll
            for (int q = 0; q < G; ++q) {
                g.ti[q] = g.ok[q] ? *(const uint2*)(tgt + g.p[q]) : make_uint2(0u, 0u);
                g.wv[q] = g.exm[q] ? *(const float4*)(w + g.p[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
                g.dv[q] = g.exm[q] ? *(const float4*)(Dacc + g.p[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        };
        auto process = [&](Grp& g) {
#pragma unroll
            for (int q = 0; q < G; ++q) {
                if (!g.ok[q]) continue;
                const uint32_t m = g.exm[q];
                uint32_t wi[4];
                if (sizeof(TgtT) == 2) {
                    wi[0] = g.ti[q].x & 0xFFFFu; wi[1] = g.ti[q].x >> 16;
                    wi[2] = g.ti[q].y & 0xFFFFu; wi[3] = g.ti[q].y >> 16;
                } else {
                    const uint32_t* tp32 = (const uint32_t*)tgt;
                    wi[0] = tp32[g.p[q]]; wi[1] = tp32[g.p[q] + 1];
                    wi[2] = tp32[g.p[q] + 2]; wi[3] = tp32[g.p[q] + 3];
                }
                deliver_one(m & 1u, wi[0], g.wv[q].x, g.dv[q].x);
                deliver_one(m & 2u, wi[1], g.wv[q].y, g.dv[q].y);
                deliver_one(m & 4u, wi[2], g.wv[q].z, g.dv[q].z);
                deliver_one(m & 8u, wi[3], g.wv[q].w, g.dv[q].w);
                // D of the excitatory positions whose target this workgroup owns
                const uint32_t sm = m & ((own(wi[0]) ? 1u : 0u) | (own(wi[1]) ? 2u : 0u) |
                                         (own(wi[2]) ? 4u : 0u) | (own(wi[3]) ? 8u : 0u));
                if (sm == 0xFu) {
                    *(float4*)(Dacc + g.p[q]) = g.dv[q];
                } else if (sm) {
                    if (sm & 1u) Dacc[g.p[q]] = g.dv[q].x;
                    if (sm & 2u) Dacc[g.p[q] + 1] = g.dv[q].y;
                    if (sm & 4u) Dacc[g.p[q] + 2] = g.dv[q].z;
                    if (sm & 8u) Dacc[g.p[q] + 3] = g.dv[q].w;
                }
            }
        };
        Grp A, B;
        if (wr_.begin < wr_.end) load(wr_.begin, A);
        for (uint32_t qb = wr_.begin; qb < wr_.end; qb += 2u * 64u * G) {
            const uint32_t nb = qb + 64u * G;
            if (nb < wr_.end) load(nb, B);
            process(A);
            const uint32_t na = nb + 64u * G;
            if (na < wr_.end) load(na, A);
            if (nb < wr_.end) process(B);
        }
    } else {
        // not all firing: decode the spiking runs, a chunk of delays at a time
        const uint32_t wd = tid - (tid / d.W) * d.W;
        WordRuns wr = wr0;  // this thread's word of the current chunk
        for (uint32_t d0 = 1; d0 <= d.Dmax; d0 += dpc) {
            const uint32_t dd = d0 + tid / d.W;
            // starts and ends counted in one scan: at most 32 of each per word
            // and at most 1024 words, so neither half reaches 2^16
            const uint32_t cs = (uint32_t)__popcll(wr.starts);
            const uint32_t ce = (uint32_t)__popcll(wr.ends);
            uint32_t tot;
            const uint32_t pre = block_scan(cs | (ce << 16), sh, tot);
            const uint32_t nruns = tot & 0xFFFFu;
            const uint32_t bs_ = pre & 0xFFFFu, be_ = pre >> 16;
            for (uint32_t r0 = 0; r0 < nruns; r0 += BS) {
                // k-th start / k-th end of the chunk form run k (runs never cross a delay)
                {
                    unsigned long long m = wr.starts;
                    for (uint32_t k = 0; k < cs; ++k) {
                        const uint32_t idx = bs_ + k;
                        const uint32_t b = (uint32_t)__ffsll((long long)m) - 1u;
                        m &= m - 1ull;
                        if (idx >= r0 && idx < r0 + BS) {
                            pos0[idx - r0] = wd * 64u + b;
                            excf[idx - r0] = dd;
                        }
                    }
                    m = wr.ends;
                    for (uint32_t k = 0; k < ce; ++k) {
                        const uint32_t idx = be_ + k;
                        const uint32_t b = (uint32_t)__ffsll((long long)m) - 1u;
                        m &= m - 1ull;
                        if (idx >= r0 && idx < r0 + BS) pref[idx - r0] = wd * 64u + b + 1u;
                    }
                }
                __syncthreads();
                const uint32_t nr = min(BS, nruns - r0);
                // run -> its forward range [a, e) and the aligned quads over it
                uint32_t a = 0, e = 0, nq = 0;
                if (tid < nr) {
                    const uint32_t le = min(pref[tid], d.Ncol);
                    const uint32_t ls = min(pos0[tid], le);
                    const uint32_t rd = min(max(excf[tid], 1u), d.Dmax);
                    const size_t sb = (size_t)c * d.segs + (size_t)(rd - 1u) * d.Ncol;
                    a = (uint32_t)(seg_off[sb + ls] - fb);
                    e = max(a, (uint32_t)(seg_off[sb + le] - fb));
                    nq = e > a ? ((e + 3u) >> 2) - (a >> 2) : 0u;
                }
                __syncthreads();
                uint32_t Q;
                const uint32_t qx = block_scan(nq, sh, Q);
                if (tid < nr) {
                    pos0[tid] = a;
                    excf[tid] = e;
                    pref[tid] = qx;
                }
                uint32_t qlo, qhi;
                part_slice(Q, part, nparts, qlo, qhi);
                if (allow_age && !staged && 4u * (qhi - qlo) >= aspan) {  // block-uniform
                    for (uint32_t x = tid; x < aspan; x += BS) {
                        const uint32_t xw = x + wlo;
                        const uint32_t sl = sizeof(TgtT) == 2 ? div_ncol(d, xw) : xw / d.Ncol;
                        const int32_t tq = t_last[cmap[sl] * d.Ncol + (xw - sl * d.Ncol)];
                        const int64_t ag = (tq == kNoSpike) ? 255 : (int64_t)t - tq;
                        age[x] = (uint8_t)(ag < 255 ? ag : 255);
                    }
                    staged = true;
                }
                __syncthreads();
                // each lane takes one quad of positions p .. p+3 of a run at a time
                // (vector loads; bit j of the mask: p + j lies in the run)
                constexpr int QU = U >= 2 ? U / 2 : 1;
                const WaveRange wr_ = wave_range_in(qlo, qhi);
                uint32_t cur = wr_.begin < wr_.end ? upper_run(pref, 0u, nr, wr_.begin) : 0u;
                for (uint32_t kb = wr_.begin; kb < wr_.end; kb += 64u * QU) {
                    uint32_t p4[QU], m4[QU], ti[QU][4];
                    bool ex4[QU];
                    float4 wv[QU], dv[QU];
    #pragma unroll
                    for (int q = 0; q < QU; ++q) {
                        const uint32_t sb = kb + q * 64u;
                        const uint32_t k = sb + lane_id();
                        const bool ok = k < wr_.end;
                        if (sb < wr_.end && cur + 1 < nr && pref[cur + 1] <= sb)
                            cur = upper_run(pref, cur + 1, nr, sb);
                        const uint32_t r = ok ? lane_run(pref, cur, nr, k) : 0u;
                        const uint32_t ra = pos0[r], re = excf[r];
                        const uint32_t p = ok ? ((ra >> 2) + (k - pref[r])) << 2 : 0u;
                        uint32_t m = 0;
    #pragma unroll
                        for (uint32_t j = 0; j < 4; ++j) m |= (ok && p + j >= ra && p + j < re) ? (1u << j) : 0u;
                        p4[q] = p;
                        m4[q] = m;
                        ex4[q] = m && is_exc(ra);
                    }
    #pragma unroll
                    for (int q = 0; q < QU; ++q) {
                        if (sizeof(TgtT) == 2) {
                            const uint2 tv = m4[q] ? *(const uint2*)(tgt + p4[q]) : make_uint2(0u, 0u);
                            ti[q][0] = tv.x & 0xFFFFu; ti[q][1] = tv.x >> 16;
                            ti[q][2] = tv.y & 0xFFFFu; ti[q][3] = tv.y >> 16;
                        } else {
                            const uint4 tv = m4[q] ? *(const uint4*)((const uint32_t*)tgt + p4[q])
                                                   : make_uint4(0u, 0u, 0u, 0u);
                            ti[q][0] = tv.x; ti[q][1] = tv.y; ti[q][2] = tv.z; ti[q][3] = tv.w;
                        }
                        wv[q] = ex4[q] ? *(const float4*)(w + p4[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
                        dv[q] = ex4[q] ? *(const float4*)(Dacc + p4[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
                    }
    #pragma unroll
                    for (int q = 0; q < QU; ++q) {
                        const uint32_t m = m4[q];
                        if (!m) continue;
                        const bool ex = ex4[q];
                        if (m & 1u) deliver_one(ex, ti[q][0], wv[q].x, dv[q].x);
                        if (m & 2u) deliver_one(ex, ti[q][1], wv[q].y, dv[q].y);
                        if (m & 4u) deliver_one(ex, ti[q][2], wv[q].z, dv[q].z);
                        if (m & 8u) deliver_one(ex, ti[q][3], wv[q].w, dv[q].w);
                        if (ex) {
                            // a partial quad may share positions with another
                            // run; only owned targets' D is written
                            const uint32_t sm =
                                m & ((own(ti[q][0]) ? 1u : 0u) | (own(ti[q][1]) ? 2u : 0u) |
                                     (own(ti[q][2]) ? 4u : 0u) | (own(ti[q][3]) ? 8u : 0u));
                            if (sm == 0xFu) {
                                *(float4*)(Dacc + p4[q]) = dv[q];
                            } else {
                                if (sm & 1u) Dacc[p4[q]] = dv[q].x;
                                if (sm & 2u) Dacc[p4[q] + 1] = dv[q].y;
                                if (sm & 4u) Dacc[p4[q] + 2] = dv[q].z;
                                if (sm & 8u) Dacc[p4[q] + 3] = dv[q].w;
                            }
                        }
                    }
                }
                __syncthreads();
            }
            // the next chunk's word
            const uint32_t d1 = d0 + dpc;
            if (d1 <= d.Dmax) {
                const int64_t s1 = (int64_t)t - (int64_t)(d1 + tid / d.W) + 1;
                wr = WordRuns{0ull, 0ull, 0ull};
                if (tid < min(dpc, d.Dmax - d1 + 1u) * d.W && s1 >= 1)
                    wr = word_runs(ring + ((size_t)((uint64_t)s1 % d.R) * d.C + c) * d.W, d.W, wd, split);
            }
        }
    }
    if (WINDOW) {
        __syncthreads();
        for (uint32_t x = tid; x < nlds; x += BS) {
            const uint32_t xw = x + wlo;
            const uint32_t sl = sizeof(TgtT) == 2 ? div_ncol(d, xw) : xw / d.Ncol;
            const uint32_t kg = cmap[sl] * d.Ncol + (xw - sl * d.Ncol);
            const long long val = win64[x];
            if (val != 0) {
                if (FIXED) atomicAdd((unsigned long long*)&acc64[kg], (unsigned long long)val);
                else atomicAdd(&acc32[kg], from_fixed(val));
            }
        }
    }
    __syncthreads();
    const unsigned long long events = block_sum64(ev_local, red64);
    const unsigned long long exc_total = block_sum64(exc_events, red64);
    if (tid == 0 && events) {
        atomicAdd(&stats[c & 63].events, events);
        atomicAdd(&stats[c & 63].events_exc, exc_total);
        atomicAdd(set_events, events);
    }
}

template <bool FIXED, int WIN, typename TgtT, int U>
__global__ __launch_bounds__(1024) void k_deliver(const NetDesc* __restrict__ nds,
                                                  const uint2* __restrict__ bmap,
                                                  uint32_t allow_age, uint32_t nparts,
                                                  uint32_t nsplit, uint32_t wslots,
                                                  unsigned long long* __restrict__ set_events,
                                                  uint32_t tstep) {
    deliver_body<FIXED, WIN, TgtT, U>(nds, bmap, allow_age, nparts, nsplit, wslots, set_events,
                                      tstep, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Sparse columns: LTP and delivery organised by wavefront.  At the paper's
// rates a column has a few spiking neurons per stamp, so block-wide run
// decoding, scans and per-event run searches cost more instructions than the
// memory traffic they organise.  These paths decode raster words inside one
// wavefront (no barrier per task) and give every lane a whole piece of work:
// LTP streams the reverse rows of up to four spiking neurons at once, one
// aligned quad of entries per lane; delivery queues the excitatory (source,
// delay) segments of the column in LDS and gives each lane one segment, and
// streams each inhibitory spike (all of whose synapses have delay 1 and form
// one range of M synapses) with one wavefront.  The arithmetic and the order
// in which each synapse's state is updated are those of the dense paths.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_uniform(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// Row of lane x in a wavefront's batch: the largest lane r with exq[r] <= x
// (exq: exclusive prefix of the rows' work, ascending over the lanes).
__device__ __forceinline__ uint32_t wave_find_row(uint32_t exq, uint32_t x) {
    uint32_t r = 0;
#pragma unroll
    for (uint32_t step = 32; step > 0; step >>= 1) {
        const uint32_t v = (uint32_t)__shfl((int)exq, (int)(r + step), 64);
        if (v <= x) r += step;
    }
    return r;
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)v, o, 64);
        if (lane >= (uint32_t)o) v += y;
    }
    return v;
}

// Sparse LTP.  Each wavefront collects the spiking neurons of its raster
// words into its lanes (up to 64 at a time), loads their row bounds at once,
// and spreads the rows' aligned quads of reverse entries over the lanes, four
// quads per lane in flight.  A workgroup takes `cpw` target columns of one
// network (map entries bid, bid + nwg, ...: with nwg a multiple of 8 they sit
// on the workgroup's XCD), or with cpw = 1 one part of one column of any
// network of the set; its latency is that of its longest chain of loads, not
// of its column count, so fewer, fuller workgroups finish sooner.  With
// allow_stage and cpw = 1 the own column's spike history (the source of most
// incoming synapses) is first copied to LDS when the column's spiking
// neurons will read it more often than the copy costs.
constexpr uint32_t kMaxCpw = 8;

__device__ __forceinline__ void ltp_sparse_body(const NetDesc* __restrict__ nds,
                                                const uint2* __restrict__ bmap, uint32_t nparts,
                                                uint32_t allow_stage, uint32_t cpw, uint32_t nwg,
                                                uint32_t n_entries, uint32_t tstep,
                                                uint32_t bid) {
    const uint32_t part = cpw == 1u ? bid % nparts : 0u;
    const uint32_t e0 = cpw == 1u ? bid / nparts : bid;
    if (e0 >= n_entries) return;  // a workgroup beyond the columns (nwg is rounded up)
    const NetDesc& nd = nds[bmap[e0].x];  // cpw > 1: one network
    const Dims d = nd.d;
    const uint32_t t = nd.t0 + tstep;
    if (t < 1) return;
    const uint2* __restrict__ hist = nd.hist;
    const uint64_t* __restrict__ rowptr = nd.rowptr;
    const uint32_t* __restrict__ rev_srcd = nd.rev_srcd;
    float* __restrict__ P = nd.Pacc;
    const float* __restrict__ tp = nd.tp;
    const uint32_t tp_len = nd.tp_len;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    uint2* hown = (uint2*)lds_raw;  // [Ncol] the own column's spike history (cpw = 1)
    __shared__ uint32_t smap[kMaxCpw * kSlots];
    __shared__ uint32_t ccol[kMaxCpw];
    __shared__ float tph[64];
    __shared__ uint32_t nsp_sh;
    __shared__ unsigned long long red64[16];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t nw = blockDim.x >> 6;
    // this workgroup's columns: entries e0 + k * nwg below n_entries (cpw = 1: e0)
    const uint32_t ncols = cpw == 1u ? 1u : min(cpw, (n_entries - e0 + nwg - 1u) / nwg);
    if (tid < ncols) ccol[tid] = bmap[e0 + tid * nwg].y;
    if (tid < 64) tph[tid] = tid < tp_len ? tp[tid] : 0.0f;
    if (tid == 0) nsp_sh = 0;
    __syncthreads();
    for (uint32_t x = tid; x < ncols * kSlots; x += blockDim.x)
        smap[x] = nd.srcmap[ccol[x / kSlots] * kSlots + (x % kSlots)];
    const uint64_t* __restrict__ ring = nd.ring + (size_t)(t % d.R) * d.C * d.W;
    const uint32_t nwords = ncols * d.W;
    uint32_t cnt_own = 0;
    for (uint32_t x = tid; x < nwords; x += blockDim.x)
        cnt_own += (uint32_t)__popcll(ring[(size_t)ccol[x / d.W] * d.W + (x % d.W)]);
    if (cnt_own) atomicAdd(&nsp_sh, cnt_own);
    __syncthreads();
    const uint32_t nsp = nsp_sh;
    if (nsp == 0) return;  // block-uniform
    // copying Ncol entries pays when the expected own-column visits (about
    // M x 0.8 x 0.5 per spiking neuron) outnumber them
    const bool staged = cpw == 1u && allow_stage && (uint64_t)nsp * d.M * 2u >= 5ull * d.Ncol;
    if (staged) {
        for (uint32_t x = tid; x < d.Ncol; x += blockDim.x) hown[x] = hist[(size_t)ccol[0] * d.Ncol + x];
        __syncthreads();
    }
    // LTP of one reverse entry of a target in the workgroup's column k
    auto ltp_one = [&](uint32_t k, uint32_t sd, float pv) -> float {
        const uint32_t dl = sd & 63u;
        const uint32_t sl = sd >> 22;
        const uint32_t l = (sd >> 6) & 0xFFFFu;
        const uint2 ht = (staged && sl == 0u) ? hown[l] : hist[smap[k * kSlots + sl] * d.Ncol + l];
        const uint32_t m = ht.x >> dl;
        uint32_t dt;
        if (m) {
            dt = (uint32_t)__ffs((int)m) - 1u;
        } else {
            const int32_t to = (int32_t)ht.y;
            if (to == kNoSpike) return pv;
            dt = (uint32_t)((int64_t)t - dl - to);
        }
        return pv + (dt < 64u ? tph[dt] : (dt < tp_len ? tp[dt] : 0.0f));
    };
    const uint32_t gw = wave_uniform(part * nw + (tid >> 6));
    const uint32_t gstride = nparts * nw;
    unsigned long long visits = 0;
    uint32_t g = gw, gk = 0, gbase = 0;
    unsigned long long m = 0;
    for (;;) {
        // up to 64 spiking neurons of this wavefront's words, one per lane
        uint32_t cnt = 0, myid = 0, myk = 0;
        while (cnt < 64u) {
            if (!m) {
                if (g >= nwords) break;
                gk = g / d.W;
                const uint32_t wd = g - gk * d.W;
                m = ring[(size_t)ccol[gk] * d.W + wd];
                gbase = ccol[gk] * d.Ncol + wd * 64u;
                g += gstride;
                continue;
            }
            const uint32_t b = (uint32_t)__ffsll((long long)m) - 1u;
            m &= m - 1ull;
            if (lane == cnt) {
                myid = gbase + b;
                myk = gk;
            }
            ++cnt;
        }
        if (cnt == 0u) break;
        uint64_t a = 0, e = 0;
        if (lane < cnt) {
            a = rowptr[myid];
            e = rowptr[myid + 1];
            visits += e - a;
        }
        const uint32_t nq = e > a ? (uint32_t)(((e + 3u) >> 2) - (a >> 2)) : 0u;
        const uint32_t inc = wave_incl_scan(nq);
        const uint32_t exq = inc - nq;
        const uint32_t Q = (uint32_t)__shfl((int)inc, 63, 64);
        for (uint32_t base = 0; base < Q; base += 256u) {
            uint64_t p[4], ra[4], re[4];
            uint32_t rk[4];
            uint4 sdv[4];
            float4 pv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t x = base + (uint32_t)u * 64u + lane;
                const uint32_t r = wave_find_row(exq, x);
                ra[u] = (uint64_t)__shfl((long long)a, (int)r, 64);
                re[u] = (uint64_t)__shfl((long long)e, (int)r, 64);
                rk[u] = (uint32_t)__shfl((int)myk, (int)r, 64);
                const uint32_t rx = (uint32_t)__shfl((int)exq, (int)r, 64);
                p[u] = ((ra[u] >> 2) + (x - rx)) << 2;
                if (x >= Q) re[u] = 0u;  // no entry of this quad is in a row
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool any = re[u] != 0u;
                sdv[u] = any ? *(const uint4*)(rev_srcd + p[u]) : make_uint4(0u, 0u, 0u, 0u);
                pv[u] = any ? *(const float4*)(P + p[u]) : make_float4(0.f, 0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint64_t q = p[u];
                const bool in0 = q >= ra[u] && q < re[u], in1 = q + 1u >= ra[u] && q + 1u < re[u];
                const bool in2 = q + 2u >= ra[u] && q + 2u < re[u], in3 = q + 3u >= ra[u] && q + 3u < re[u];
                float4 o = pv[u];
                if (in0) o.x = ltp_one(rk[u], sdv[u].x, pv[u].x);
                if (in1) o.y = ltp_one(rk[u], sdv[u].y, pv[u].y);
                if (in2) o.z = ltp_one(rk[u], sdv[u].z, pv[u].z);
                if (in3) o.w = ltp_one(rk[u], sdv[u].w, pv[u].w);
                // a quad shared with another neuron's row keeps that row's entries
                if (in0 && in1 && in2 && in3) {
                    *(float4*)(P + q) = o;
                } else {
                    if (in0) P[q] = o.x;
                    if (in1) P[q + 1] = o.y;
                    if (in2) P[q + 2] = o.z;
                    if (in3) P[q + 3] = o.w;
                }
            }
        }
        if (cnt < 64u) break;  // every word of this wavefront has been read
    }
    const unsigned long long v = block_sum64(visits, red64);
    // the stats slot of the first column (counters are only summed)
    if (tid == 0 && v) atomicAdd(&nd.stats[ccol[0] & 63].ltp_visits, v);
}

// Sparse delivery.  One pass over the column's (delay, raster word) tasks
// (two per thread) finds the spiking sources; one block scan gives every
// excitatory (source, delay) segment and every inhibitory spike a queue slot.
// Each lane then delivers whole segments, eight synapses (two aligned quads)
// at a time with all their loads in flight; each wavefront delivers two
// inhibitory spikes at a time (an inhibitory neuron's M synapses all have
// delay 1 and lie in one range of the column's delay-1 block).  Currents of
// the first wslots slots are summed in an LDS window, the rest go to global
// atomics; LTD reads the own column's spike ages from an LDS copy.
template <bool FIXED, typename TgtT>
__device__ __forceinline__ void deliver_sparse_body(const NetDesc* __restrict__ nds,
                                                    const uint2* __restrict__ bmap,
                                                    uint32_t nparts, uint32_t wslots,
                                                    unsigned long long* __restrict__ set_events,
                                                    uint32_t tstep, uint32_t bid) {
    const uint2 br = bmap[bid / nparts];
    const uint32_t part = bid % nparts;
    const NetDesc& nd = nds[br.x];
    const Dims d = nd.d;
    const uint32_t t = nd.t0 + tstep;
    if (t < 1) return;
    const uint32_t c = br.y;
    const uint64_t* __restrict__ ring = nd.ring;
    const uint64_t* __restrict__ seg_off = nd.seg_off;
    const uint64_t fb = ((uint64_t)c * d.Ncol * d.M) & ~3ull;
    const TgtT* __restrict__ tgt = (const TgtT*)nd.tgt + fb;
    const float* __restrict__ w = nd.w + fb;
    float* __restrict__ Dacc = nd.Dacc + fb;
    const int32_t* __restrict__ t_last = nd.t_last;
    const float* __restrict__ tm = nd.tm;
    const uint32_t tm_len = nd.tm_len;
    long long* __restrict__ acc64 = (long long*)nd.acc;
    float* __restrict__ acc32 = (float*)nd.acc;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ uint32_t cmap[kSlots];
    __shared__ float tmh[64];
    __shared__ uint32_t sh[20];
    __shared__ unsigned long long red64[16];
    const uint32_t BS = blockDim.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t nw = BS >> 6;
    const uint32_t nlds = wslots * d.Ncol;  // LDS window: the first wslots slots
    long long* win64 = (long long*)lds_raw;
    uint8_t* age = lds_raw + (((size_t)nlds * 8 + 15) & ~(size_t)15);         // [Ncol]
    uint32_t* qa = (uint32_t*)(age + (((size_t)d.Ncol + 15) & ~(size_t)15));  // [kQueue]
    uint32_t* qe = qa + kQueue;                                                // [kQueue]
    uint32_t* qi = qe + kQueue;                                                // [kQueue]
    for (uint32_t x = tid; x < nlds; x += BS) win64[x] = 0;
    // steps since each own-column neuron's latest spike, 255 = none or older
    for (uint32_t x = tid; x < d.Ncol; x += BS) {
        const int32_t tq = t_last[(size_t)c * d.Ncol + x];
        const int64_t ag = (tq == kNoSpike) ? 255 : (int64_t)t - tq;
        age[x] = (uint8_t)(ag < 255 ? ag : 255);
    }
    if (tid < kSlots) cmap[tid] = nd.colmap[c * kSlots + tid];
    if (tid < 64) tmh[tid] = tid < tm_len ? tm[tid] : 0.0f;
    const long long q_inh = to_fixed(d.w_inh);
    const size_t s1 = (size_t)c * d.segs;
    const uint32_t inh_lo = d.Ne < d.Ncol ? (uint32_t)(seg_off[s1 + d.Ne] - fb) : 0u;
    unsigned long long ev_local = 0, exc_events = 0;
    auto global_id = [&](uint32_t wi) {
        const uint32_t sl = sizeof(TgtT) == 2 ? div_ncol(d, wi) : wi / d.Ncol;
        return cmap[sl] * d.Ncol + (wi - sl * d.Ncol);
    };
    auto add_current = [&](uint32_t wi, long long q, float f) {
        if (wi < nlds) {
            atomicAdd((unsigned long long*)&win64[wi], (unsigned long long)q);
        } else if (FIXED) {
            atomicAdd((unsigned long long*)&acc64[global_id(wi)], (unsigned long long)q);
        } else {
            atomicAdd(&acc32[global_id(wi)], f);
        }
    };
    // steps dt from the target's latest spike to the arrival (t + 1), or
    // 0xFFFFFFFF if it never fired; own-column targets from the LDS ages
    auto arrival_dt = [&](uint32_t wi) -> uint32_t {
        if (wi < d.Ncol) {
            const uint32_t ag = age[wi];
            if (ag < 255u) return ag + 1u;
        }
        const int32_t tq = t_last[global_id(wi)];
        return tq == kNoSpike ? 0xFFFFFFFFu : (uint32_t)((int64_t)t + 1 - tq);
    };
    auto ltd_add = [&](uint32_t dt, float dv) -> float {
        if (dt == 0xFFFFFFFFu) return dv;
        return dv + (dt < 64u ? tmh[dt] : (dt < tm_len ? tm[dt] : 0.0f));
    };
    __syncthreads();
    // this part's tasks: task index x = part + nparts * k; a round hands two
    // tasks to each thread
    const uint32_t ntask = d.Dmax * d.W;
    const uint32_t nmine = ntask > part ? (ntask - part + nparts - 1u) / nparts : 0u;
    for (uint32_t k0 = 0; k0 < nmine; k0 += 2u * BS) {
        unsigned long long mex[2] = {0ull, 0ull}, mih[2] = {0ull, 0ull};
        uint32_t dd[2] = {1u, 1u}, wd[2] = {0u, 0u};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t k = k0 + (uint32_t)h * BS + tid;
            if (k >= nmine) continue;
            const uint32_t x = part + nparts * k;
            dd[h] = x / d.W + 1u;
            wd[h] = x - (dd[h] - 1u) * d.W;
            const int64_t st = (int64_t)t - (int64_t)dd[h] + 1;
            if (st < 1) continue;
            const unsigned long long m = ring[((size_t)((uint64_t)st % d.R) * d.C + c) * d.W + wd[h]];
            // local ids below Ne are excitatory; inhibitory synapses all have delay 1
            const uint32_t lo = wd[h] * 64u;
            const unsigned long long em = d.Ne <= lo ? 0ull
                                         : (d.Ne >= lo + 64u ? ~0ull : ((1ull << (d.Ne - lo)) - 1ull));
            mex[h] = m & em;
            mih[h] = dd[h] == 1u ? (m & ~em) : 0ull;
        }
        const uint32_t nex = (uint32_t)(__popcll(mex[0]) + __popcll(mex[1]));
        const uint32_t nih = (uint32_t)(__popcll(mih[0]) + __popcll(mih[1]));
        uint32_t tot;
        // at most 2 x 64 bits per thread and 256 threads: each half < 2^16
        const uint32_t pre = block_scan(nex | (nih << 16), sh, tot);
        const uint32_t tex = tot & 0xFFFFu, tih = tot >> 16;
        for (uint32_t r0 = 0; r0 < max(tex, tih); r0 += kQueue) {
            // queue slots [r0, r0 + kQueue) of both kinds
            uint32_t ie = pre & 0xFFFFu, ii = pre >> 16;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                unsigned long long me = mex[h], mi = mih[h];
                while (me) {
                    const uint32_t b = (uint32_t)__ffsll((long long)me) - 1u;
                    me &= me - 1ull;
                    if (ie >= r0 && ie < r0 + kQueue) {
                        const size_t sg = s1 + (size_t)(dd[h] - 1u) * d.Ncol + wd[h] * 64u + b;
                        qa[ie - r0] = (uint32_t)(seg_off[sg] - fb);
                        qe[ie - r0] = (uint32_t)(seg_off[sg + 1] - fb);
                    }
                    ++ie;
                }
                while (mi) {
                    const uint32_t b = (uint32_t)__ffsll((long long)mi) - 1u;
                    mi &= mi - 1ull;
                    if (ii >= r0 && ii < r0 + kQueue) qi[ii - r0] = wd[h] * 64u + b;
                    ++ii;
                }
            }
            __syncthreads();
            const uint32_t ne = tex > r0 ? min(kQueue, tex - r0) : 0u;
            const uint32_t ni = tih > r0 ? min(kQueue, tih - r0) : 0u;
            // excitatory segments: one per lane, two aligned quads at a time
            for (uint32_t sgi = tid; sgi < ne; sgi += BS) {
                const uint32_t a = qa[sgi], e = qe[sgi];
                for (uint32_t p0 = a & ~3u; p0 < e; p0 += 8u) {
                    uint32_t wi[8];
                    float wv[8], dv[8];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const uint32_t q = p0 + 4u * (uint32_t)u;
                        const bool ok = q < e;
                        if (sizeof(TgtT) == 2) {
                            const uint2 tv = ok ? *(const uint2*)(tgt + q) : make_uint2(0u, 0u);
                            wi[4 * u + 0] = tv.x & 0xFFFFu; wi[4 * u + 1] = tv.x >> 16;
                            wi[4 * u + 2] = tv.y & 0xFFFFu; wi[4 * u + 3] = tv.y >> 16;
                        } else {
                            const uint4 tv = ok ? *(const uint4*)((const uint32_t*)tgt + q)
                                                : make_uint4(0u, 0u, 0u, 0u);
                            wi[4 * u + 0] = tv.x; wi[4 * u + 1] = tv.y;
                            wi[4 * u + 2] = tv.z; wi[4 * u + 3] = tv.w;
                        }
                        const float4 w4 = ok ? *(const float4*)(w + q) : make_float4(0.f, 0.f, 0.f, 0.f);
                        const float4 d4 = ok ? *(const float4*)(Dacc + q) : make_float4(0.f, 0.f, 0.f, 0.f);
                        wv[4 * u + 0] = w4.x; wv[4 * u + 1] = w4.y; wv[4 * u + 2] = w4.z; wv[4 * u + 3] = w4.w;
                        dv[4 * u + 0] = d4.x; dv[4 * u + 1] = d4.y; dv[4 * u + 2] = d4.z; dv[4 * u + 3] = d4.w;
                    }
                    uint32_t dts[8];
                    bool in[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const uint32_t pj = p0 + (uint32_t)j;
                        in[j] = pj >= a && pj < e;
                        dts[j] = in[j] ? arrival_dt(wi[j]) : 0xFFFFFFFFu;
                    }
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        if (!in[j]) continue;
                        add_current(wi[j], to_fixed(wv[j]), wv[j]);
                        dv[j] = ltd_add(dts[j], dv[j]);
                    }
                    // a quad shared with another segment keeps that segment's D
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const uint32_t q = p0 + 4u * (uint32_t)u;
                        if (in[4 * u] && in[4 * u + 1] && in[4 * u + 2] && in[4 * u + 3]) {
                            *(float4*)(Dacc + q) = make_float4(dv[4 * u], dv[4 * u + 1], dv[4 * u + 2], dv[4 * u + 3]);
                        } else {
#pragma unroll
                            for (int j = 0; j < 4; ++j)
                                if (in[4 * u + j]) Dacc[q + j] = dv[4 * u + j];
                        }
                    }
                }
                ev_local += e - a;
                exc_events += e - a;
            }
            // inhibitory spikes: two per wavefront at a time, one quad per lane each
            for (uint32_t sp = tid >> 6; sp < ni; sp += 2u * nw) {
                const uint32_t sp2 = sp + nw;
                const uint32_t a1 = inh_lo + (qi[sp] - d.Ne) * d.M;
                const uint32_t a2 = sp2 < ni ? inh_lo + (qi[sp2] - d.Ne) * d.M : a1;
                const uint32_t n2 = sp2 < ni ? d.M : 0u;
                for (uint32_t off = 4u * lane; off < d.M + 3u; off += 256u) {
                    uint32_t wi[8];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const uint32_t q = ((u == 0 ? a1 : a2) & ~3u) + off;
                        const bool ok = q < (u == 0 ? a1 + d.M : a2 + n2);
                        if (sizeof(TgtT) == 2) {
                            const uint2 tv = ok ? *(const uint2*)(tgt + q) : make_uint2(0u, 0u);
                            wi[4 * u + 0] = tv.x & 0xFFFFu; wi[4 * u + 1] = tv.x >> 16;
                            wi[4 * u + 2] = tv.y & 0xFFFFu; wi[4 * u + 3] = tv.y >> 16;
                        } else {
                            const uint4 tv = ok ? *(const uint4*)((const uint32_t*)tgt + q)
                                                : make_uint4(0u, 0u, 0u, 0u);
                            wi[4 * u + 0] = tv.x; wi[4 * u + 1] = tv.y;
                            wi[4 * u + 2] = tv.z; wi[4 * u + 3] = tv.w;
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const uint32_t sa = u == 0 ? a1 : a2, se = u == 0 ? a1 + d.M : a2 + n2;
                        const uint32_t q = (sa & ~3u) + off;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (q + (uint32_t)j >= sa && q + (uint32_t)j < se)
                                add_current(wi[4 * u + j], q_inh, d.w_inh);
                    }
                }
                if (lane == 0) ev_local += d.M + n2;
            }
            __syncthreads();  // the queues are refilled
        }
    }
    // flush the window: one global atomic per target that received current
    for (uint32_t x = tid; x < nlds; x += BS) {
        const long long val = win64[x];
        if (val != 0) {
            const uint32_t kg = global_id(x);
            if (FIXED) atomicAdd((unsigned long long*)&acc64[kg], (unsigned long long)val);
            else atomicAdd(&acc32[kg], from_fixed(val));
        }
    }
    const unsigned long long events = block_sum64(ev_local, red64);
    const unsigned long long exc_total = block_sum64(exc_events, red64);
    if (tid == 0 && events) {
        atomicAdd(&nd.stats[c & 63].events, events);
        atomicAdd(&nd.stats[c & 63].events_exc, exc_total);
        atomicAdd(set_events, events);
    }
}

__global__ __launch_bounds__(256) void k_ltp_sp(const NetDesc* __restrict__ nds,
                                                const uint2* __restrict__ bmap, uint32_t nparts,
                                                uint32_t allow_stage, uint32_t cpw, uint32_t nwg,
                                                uint32_t n_entries, uint32_t tstep) {
    ltp_sparse_body(nds, bmap, nparts, allow_stage, cpw, nwg, n_entries, tstep, blockIdx.x);
}

template <bool FIXED, typename TgtT>
__global__ __launch_bounds__(256) void k_deliver_sp(const NetDesc* __restrict__ nds,
                                                    const uint2* __restrict__ bmap,
                                                    uint32_t nparts, uint32_t wslots,
                                                    unsigned long long* __restrict__ set_events,
                                                    uint32_t tstep) {
    deliver_sparse_body<FIXED, TgtT>(nds, bmap, nparts, wslots, set_events, tstep, blockIdx.x);
}

// LTP and delivery of one step in a single launch, for launches small enough
// that kernel boundaries dominate: the first n_ltp workgroups run LTP, the
// rest delivery.  The two write disjoint state (P; currents and D) and read
// nothing the other writes, so they may run concurrently.
template <bool FIXED, int WIN, typename TgtT, int U>
__global__ __launch_bounds__(1024) void k_ltp_deliver(const NetDesc* __restrict__ nds,
                                                      const uint2* __restrict__ bmap,
                                                      uint32_t allow_stage, uint32_t allow_age,
                                                      uint32_t nparts, uint32_t nsplit,
                                                      uint32_t wslots,
                                                      unsigned long long* __restrict__ set_events,
                                                      uint32_t tstep, uint32_t n_ltp,
                                                      uint32_t ltp_sparse, uint32_t cpw,
                                                      uint32_t n_entries) {
    if (blockIdx.x < n_ltp && ltp_sparse)
        ltp_sparse_body(nds, bmap, nparts, allow_stage, cpw, n_ltp, n_entries, tstep, blockIdx.x);
    else if (blockIdx.x < n_ltp)
        ltp_body<4>(nds, bmap, allow_stage, nparts, tstep, blockIdx.x);
    else
        deliver_body<FIXED, WIN, TgtT, U>(nds, bmap, allow_age, nparts, nsplit, wslots, set_events,
                                          tstep, blockIdx.x - n_ltp);
}

// Both sparse paths in one launch: the first n_ltp workgroups do LTP.
template <bool FIXED, typename TgtT>
__global__ __launch_bounds__(256) void k_ltp_deliver_sp(const NetDesc* __restrict__ nds,
                                                        const uint2* __restrict__ bmap,
                                                        uint32_t nparts, uint32_t wslots,
                                                        uint32_t allow_stage,
                                                        unsigned long long* __restrict__ set_events,
                                                        uint32_t tstep, uint32_t n_ltp) {
    if (blockIdx.x < n_ltp)
        ltp_sparse_body(nds, bmap, nparts, allow_stage, 1u, n_ltp, n_ltp, tstep, blockIdx.x);
    else
        deliver_sparse_body<FIXED, TgtT>(nds, bmap, nparts, wslots, set_events, tstep,
                                         blockIdx.x - n_ltp);
}

// ---------------------------------------------------------------------------
// ORDERED mode: the same deliveries, recorded per target with their canonical
// key (delay, source id, rank within the source's delay-d synapses, which is
// ascending j), then folded in key order by the neuron kernel.  PASS 0 counts
// events per target, PASS 1 writes them and applies LTD.
// ---------------------------------------------------------------------------
template <int PASS, typename TgtT>
__global__ __launch_bounds__(256) void k_deliver_seq(const NetDesc* __restrict__ nds,
                                                     const uint2* __restrict__ bmap,
                                                     uint32_t tstep) {
    const uint2 br = bmap[blockIdx.x];
    const NetDesc& nd = nds[br.x];
    const Dims d = nd.d;
    const uint32_t t = nd.t0 + tstep;
    if (t < 1) return;
    const uint64_t* __restrict__ ring = nd.ring;
    const uint64_t* __restrict__ seg_off = nd.seg_off;  // below 2^32 in this mode
    const TgtT* __restrict__ tgt = (const TgtT*)nd.tgt;
    const float* __restrict__ w = nd.w;
    float* __restrict__ Dacc = nd.Dacc;
    const int32_t* __restrict__ t_last = nd.t_last;
    const uint32_t* __restrict__ colmap = nd.colmap;
    const float* __restrict__ tm = nd.tm;
    const uint32_t tm_len = nd.tm_len;
    uint32_t* __restrict__ ev_cnt = nd.ev_cnt;
    const uint32_t* __restrict__ ev_start = nd.ev_start;
    uint32_t* __restrict__ cursor = nd.cursor;
    unsigned long long* __restrict__ ev_key = nd.ev_key;
    float* __restrict__ ev_w = nd.ev_w;
    DevStats* __restrict__ stats = nd.stats;
    const uint32_t c = br.y;
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t nwave = blockDim.x >> 6;
    const uint32_t ntasks = d.Dmax * d.W;
    unsigned long long events = 0, exc_events = 0;
    for (uint32_t task = wave; task < ntasks; task += nwave) {
        const uint32_t dd = task / d.W + 1u;
        const uint32_t wd = task - (dd - 1u) * d.W;
        const int64_t s = (int64_t)t - (int64_t)dd + 1;
        if (s < 1) continue;
        unsigned long long m = ring[((size_t)((uint64_t)s % d.R) * d.C + c) * d.W + wd];
        while (m) {
            const uint32_t l = wd * 64u + (uint32_t)__ffsll((long long)m) - 1u;
            m &= m - 1ull;
            const uint32_t i = c * d.Ncol + l;
            const bool exc = l < d.Ne;
            const size_t sg = (size_t)c * d.segs + (size_t)(dd - 1u) * d.Ncol + l;
            const uint32_t p0 = (uint32_t)seg_off[sg], p1 = (uint32_t)seg_off[sg + 1];
            for (uint32_t pos = p0 + lane; pos < p1; pos += 64) {
                const uint32_t wi = (uint32_t)tgt[pos];
                const uint32_t sl = wi / d.Ncol;
                const uint32_t kg = colmap[c * kSlots + sl] * d.Ncol + (wi - sl * d.Ncol);
                if (PASS == 0) {
                    atomicAdd(&ev_cnt[kg], 1u);
                } else {
                    const uint32_t slot = ev_start[kg] + atomicAdd(&cursor[kg], 1u);
                    ev_key[slot] = ((unsigned long long)dd << 42) |
                                   ((unsigned long long)i << 16) |
                                   (unsigned long long)(pos - p0);
                    ev_w[slot] = exc ? w[pos] : d.w_inh;
                    if (exc) {
                        const int32_t tq = t_last[kg];
                        if (tq != kNoSpike) {
                            const uint32_t dt = (uint32_t)((int64_t)t + 1 - tq);
                            Dacc[pos] = Dacc[pos] + (dt < tm_len ? tm[dt] : 0.0f);
                        }
                    }
                }
            }
            if (PASS == 1) {
                events += p1 - p0;
                if (exc) exc_events += p1 - p0;
            }
        }
    }
    if (PASS == 1 && lane == 0 && events) {
        atomicAdd(&stats[c & 63].events, events);
        atomicAdd(&stats[c & 63].events_exc, exc_events);
    }
}

// ---------------------------------------------------------------------------
// Neuron update (item 2.7) with the thalamic input (Sec. 2, reproducible
// stimulus: a prescribed number of events per ms per column).  The recovery
// equation is read as u' = a (b v - u) (the printed a (b v - c) has no rest
// state); v takes two 0.5 ms sub-steps and u one 1 ms step (Sec. 3).
// One thread per neuron; each wavefront covers one 64-neuron raster word.
// ---------------------------------------------------------------------------
// Events per target up to which the ordered fold selects keys one by one
// (O(n^2) reads, no writes); above it the target's events are sorted first:
// by the whole wavefront in LDS up to kLdsSort events (and folded there),
// else in place by the target's own thread.
constexpr uint32_t kSelectFold = 32;
constexpr uint32_t kLdsSort = 1024;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort of one target's events by the 64 lanes of a wavefront, in
// two helpers that a host test also runs (lane by lane, which is the same
// computation: the pairs of one stage are disjoint):
// wave_sort_load: the n events into sk / sw, padded to P (a power of two,
// at least 64) with keys above every real key; bitonic_stage: the
// compare-exchange stage (k, j) for the elements lane, lane + 64, ... .
__device__ __forceinline__ uint32_t wave_sort_load(const unsigned long long* __restrict__ key,
                                                   const float* __restrict__ wt, uint32_t n,
                                                   unsigned long long* __restrict__ sk,
                                                   float* __restrict__ sw, uint32_t lane) {
    uint32_t P = 64u;
    while (P < n) P <<= 1;
    for (uint32_t x = lane; x < P; x += 64u) {
        sk[x] = x < n ? key[x] : ~0ull;
        sw[x] = x < n ? wt[x] : 0.0f;
    }
    return P;
}

__device__ __forceinline__ void bitonic_stage(unsigned long long* __restrict__ sk,
                                              float* __restrict__ sw, uint32_t P, uint32_t k,
                                              uint32_t j, uint32_t lane) {
    for (uint32_t x = lane; x < P; x += 64u) {
        const uint32_t y = x ^ j;
        if (y > x) {
            const unsigned long long a = sk[x], b = sk[y];
            if ((a > b) == ((x & k) == 0u)) {
                sk[x] = b;
                sk[y] = a;
                const float wa = sw[x];
                sw[x] = sw[y];
                sw[y] = wa;
            }
        }
    }
}

// One target's n (kSelectFold < n <= kLdsSort) events sorted by key by all 64
// lanes of a wavefront in the wavefront's LDS arrays sk / sw.  Called with
// the whole wavefront active; the sorted events stay in LDS.
__device__ __forceinline__ void wave_sort_events(const unsigned long long* __restrict__ key,
                                                 const float* __restrict__ wt, uint32_t n,
                                                 unsigned long long* __restrict__ sk,
                                                 float* __restrict__ sw) {
    const uint32_t lane = lane_id();
    const uint32_t P = wave_sort_load(key, wt, n, sk, sw, lane);
    wave_sync();
    for (uint32_t k = 2u; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0u; j >>= 1) {
            bitonic_stage(sk, sw, P, k, j, lane);
            wave_sync();
        }
    }
}

// The fp32 fold of a neuron's external input of the step, onto a: its
// thalamic hits, then its stimulus entries in list order.
__device__ __forceinline__ float fold_external(float a, uint32_t hits, float thal_mv, uint32_t sb,
                                               uint32_t se, const uint32_t* __restrict__ stim_id,
                                               const float* __restrict__ stim_mv, uint32_t k) {
    for (uint32_t h = 0; h < hits; ++h) a = a + thal_mv;
    for (uint32_t e = sb; e < se; ++e)
        if (stim_id[e] == k) a = a + stim_mv[e];
    return a;
}

// One target's n events of a step, sorted in place by key (weights move
// with their keys): heapsort, O(n log n) in the target's own slot range.
__device__ __forceinline__ void sift_events(unsigned long long* __restrict__ key,
                                            float* __restrict__ wt, uint32_t r, uint32_t end) {
    const unsigned long long rk = key[r];
    const float rw = wt[r];
    for (;;) {
        uint32_t ch = 2u * r + 1u;
        if (ch >= end) break;
        unsigned long long ck = key[ch];
        if (ch + 1u < end) {
            const unsigned long long k2 = key[ch + 1u];
            if (k2 > ck) {
                ch += 1u;
                ck = k2;
            }
        }
        if (ck <= rk) break;
        key[r] = ck;
        wt[r] = wt[ch];
        r = ch;
    }
    key[r] = rk;
    wt[r] = rw;
}

__device__ __forceinline__ void sort_events(unsigned long long* __restrict__ key,
                                            float* __restrict__ wt, uint32_t n) {
    for (uint32_t s = n / 2u; s-- > 0u;) sift_events(key, wt, s, n);
    for (uint32_t end = n; end > 1u; --end) {
        const unsigned long long k0 = key[0];
        const float w0 = wt[0];
        key[0] = key[end - 1u];
        wt[0] = wt[end - 1u];
        key[end - 1u] = k0;
        wt[end - 1u] = w0;
        sift_events(key, wt, 0u, end - 1u);
    }
}

template <uint32_t MODE>
__global__ __launch_bounds__(256) void k_neuron(const NetDesc* __restrict__ nds,
                                                const uint2* __restrict__ bmap, uint32_t tstep) {
    const uint2 br = bmap[blockIdx.x];
    const NetDesc& nd = nds[br.x];
    const Dims d = nd.d;
    const uint32_t t = nd.t0 + tstep;
    float* __restrict__ v = nd.v;
    float* __restrict__ u = nd.u;
    void* __restrict__ acc_v = nd.acc;
    uint32_t* __restrict__ hist32 = (uint32_t*)nd.hist;  // x, y interleaved
    int32_t* __restrict__ t_last = nd.t_last;
    uint64_t* __restrict__ ring = nd.ring;
    const uint32_t thal_whole = nd.thal_whole, thal_thr = nd.thal_thr;
    const float thal_mv = nd.thal_mv;
    const uint32_t* __restrict__ stim_id = nd.stim_id;
    const float* __restrict__ stim_mv = nd.stim_mv;
    uint32_t* __restrict__ ev_cnt = nd.ev_cnt;
    const uint32_t* __restrict__ ev_start = nd.ev_start;
    unsigned long long* __restrict__ ev_key = nd.ev_key;
    float* __restrict__ ev_w = nd.ev_w;
    uint32_t* __restrict__ cursor = nd.cursor;
    DevStats* __restrict__ stats = nd.stats;
    // stimulus entries of step t: [sb, se) of the step-sorted list
    uint32_t sb = 0, se = 0;
    if (nd.stim_n) {
        uint32_t lo = 0, hi = nd.stim_n;
        while (lo < hi) { const uint32_t m = (lo + hi) >> 1; if (nd.stim_t[m] < t) lo = m + 1; else hi = m; }
        sb = lo;
        hi = nd.stim_n;
        while (lo < hi) { const uint32_t m = (lo + hi) >> 1; if (nd.stim_t[m] <= t) lo = m + 1; else hi = m; }
        se = lo;
    }
    __shared__ uint32_t wsum[4];
    const uint32_t wi = br.y + (threadIdx.x >> 6);
    const uint32_t lane = lane_id();
    const bool wave_ok = wi < d.C * d.W;
    const uint32_t c = wave_ok ? wi / d.W : 0u;
    const uint32_t wd = wi - c * d.W;
    const uint32_t l = wd * 64u + lane;
    const bool valid = wave_ok && l < d.Ncol;
    bool fired = false;
    // Thalamic picks of column c in step t: pick p is word 1 + p % 3 of
    // generator call p / 3, and word 0 of call 0 decides the fractional
    // count.  The 64 lanes of a wavefront draw the calls in parallel and
    // count the hits on their own 64 neurons in LDS.
    __shared__ uint32_t thc[4][64];
    const uint32_t wv = threadIdx.x >> 6;
    thc[wv][lane] = 0u;
    __syncthreads();
    if (wave_ok && (thal_whole | thal_thr)) {  // wavefront-uniform
        uint32_t n = 0;
        for (uint32_t call0 = 0;; call0 += 64u) {
            const uint32_t call = call0 + lane;
            uint32_t z[4] = {c, t, kTagThal, call};
            philox10(z, d.key0, d.key1);
            if (call0 == 0) n = thal_whole + (__shfl(z[0], 0, 64) < thal_thr ? 1u : 0u);
#pragma unroll
            for (uint32_t q = 0; q < 3; ++q) {
                if (3u * call + q < n) {
                    const uint32_t rel = pick(z[1 + q], d.Ncol) - wd * 64u;
                    if (rel < 64u) atomicAdd(&thc[wv][rel], 1u);
                }
            }
            if (n <= 3u * (call0 + 64u)) break;
        }
    }
    __syncthreads();
    // ORDERED: targets with many events this step are sorted by the whole
    // wavefront in LDS, and each such target's lane folds them there, after
    // its external input (the same sums as the per-neuron path below)
    float lds_fold = 0.0f;
    if constexpr (MODE == DPSNN_SUM_ORDERED) {
        __shared__ unsigned long long ssk[4][kLdsSort];
        __shared__ float ssw[4][kLdsSort];
        const uint32_t kk = valid ? c * d.Ncol + l : 0u;
        const uint32_t ne = valid ? ev_cnt[kk] : 0u;
        const uint32_t b0 = valid ? ev_start[kk] : 0u;
        const bool mine = valid && ne > kSelectFold && ne <= kLdsSort;
        if (mine) lds_fold = fold_external(0.0f, thc[wv][lane], thal_mv, sb, se, stim_id, stim_mv, kk);
        unsigned long long big = __ballot(mine);
        while (big) {
            const uint32_t src = (uint32_t)__ffsll((long long)big) - 1u;
            big &= big - 1ull;
            const uint32_t nb = __shfl(ne, (int)src, 64);
            const uint32_t bb = __shfl(b0, (int)src, 64);
            wave_sort_events(ev_key + bb, ev_w + bb, nb, ssk[wv], ssw[wv]);
            if (lane == src)
                for (uint32_t x = 0; x < nb; ++x) lds_fold = lds_fold + ssw[wv][x];
            wave_sync();  // the next target reuses the LDS arrays
        }
    }
    if (valid) {
        const uint32_t k = c * d.Ncol + l;
        // external input: this neuron's thalamic hits, then the stimulus
        const uint32_t hits = thc[wv][lane];
        long long a64 = 0;
        float a32 = 0.0f;
        if (MODE == DPSNN_SUM_FIXED) a64 = ((long long*)acc_v)[k];
        if (MODE == DPSNN_SUM_ATOMIC) a32 = ((float*)acc_v)[k];
        if (MODE == DPSNN_SUM_FIXED) {
            a64 += (long long)hits * to_fixed(thal_mv);
            for (uint32_t e = sb; e < se; ++e)
                if (stim_id[e] == k) a64 += to_fixed(stim_mv[e]);
        } else {
            a32 = fold_external(a32, hits, thal_mv, sb, se, stim_id, stim_mv, k);
        }
        if (MODE == DPSNN_SUM_ORDERED) {
            // canonical-order fold of this step's deliveries (keys are
            // distinct): few events are taken by repeated selection of the
            // next key (reads only); many are first sorted in place
            const uint32_t b0 = ev_start[k];
            const uint32_t ne = ev_cnt[k];
            if (ne <= kSelectFold) {
                unsigned long long prev = 0ull;
                for (uint32_t r = 0; r < ne; ++r) {
                    unsigned long long best = ~0ull;
                    float bw = 0.0f;
                    for (uint32_t x = 0; x < ne; ++x) {
                        const unsigned long long kk = ev_key[b0 + x];
                        if (kk > prev && kk < best) { best = kk; bw = ev_w[b0 + x]; }
                    }
                    a32 = a32 + bw;
                    prev = best;
                }
            } else if (ne <= kLdsSort) {
                a32 = lds_fold;  // folded from LDS above, external input first
            } else {
                sort_events(ev_key + b0, ev_w + b0, ne);
                for (uint32_t x = 0; x < ne; ++x) a32 = a32 + ev_w[b0 + x];
            }
            ev_cnt[k] = 0u;
            cursor[k] = 0u;
        }
        const float I = (MODE == DPSNN_SUM_FIXED) ? from_fixed(a64) : a32;
        const bool rs = l < d.Ne;
        const float pa = rs ? 0.02f : 0.1f;
        const float pb = 0.2f;
        const float pc = -65.0f;
        const float pd = rs ? 8.0f : 2.0f;
        float vv = v[k], uu = u[k];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float e = 0.04f * vv;
            e = e * vv;
            e = e + 5.0f * vv;
            e = e + 140.0f;
            e = e - uu;
            e = e + I;
            vv = vv + 0.5f * e;
        }
        const float bv = pb * vv;
        uu = uu + pa * (bv - uu);
        if (vv >= 30.0f) {
            vv = pc;
            uu = uu + pd;
            fired = true;
        }
        v[k] = vv;
        u[k] = uu;
        // history: bit b <-> stamp (t + 1) - b after the shift
        const uint32_t h = hist32[2 * (size_t)k];
        if (h >> 31) hist32[2 * (size_t)k + 1] = (uint32_t)((int32_t)t - 31);
        hist32[2 * (size_t)k] = (h << 1) | (fired ? 1u : 0u);
        if (fired) t_last[k] = (int32_t)t + 1;
        if (MODE == DPSNN_SUM_FIXED) ((long long*)acc_v)[k] = 0;
        else ((float*)acc_v)[k] = 0.0f;
    }
    const unsigned long long mask = __ballot(fired);
    if (lane == 0) {
        if (wave_ok) ring[((size_t)((t + 1u) % d.R) * d.C + c) * d.W + wd] = mask;
        wsum[wv] = (uint32_t)__popcll(mask);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t x = 0; x < (blockDim.x >> 6); ++x) s += wsum[x];
        if (s) atomicAdd(&stats[(br.y >> 2) & 63].spikes, (unsigned long long)s);
    }
}

// Consolidation: for every excitatory synapse (reverse entry x, forward
// position f): sd = P - D; w <- clamp(w + (bias + sd), 0, w_max);
// P <- decay * sd; D <- 0.
// Done in two passes so that only one array is touched out of order:
//   k_wupdate     (reverse order): sd = P - D[f]; D[f] <- sd; P <- decay * sd;
//   k_wupdate_fwd (forward order, coalesced): w <- clamp(w + (bias + D)); D <- 0
// for the excitatory positions (the inhibitory synapses of a column are one
// delay-1 range of its forward block, which the second pass skips).
// Workgroup (target column ct, chunk q) of the map: entries of ct's reverse
// rows; an entry's forward position is the block start of the column that
// reaches ct through its slot plus rev_fwd.
__global__ __launch_bounds__(256) void k_wupdate(const NetDesc* __restrict__ nds,
                                                 const uint2* __restrict__ bmap) {
    __shared__ uint32_t smap[kSlots];
    const uint2 br = bmap[blockIdx.x];
    const NetDesc& nd = *nds;
    const Dims d = nd.d;
    const uint32_t* __restrict__ rev_srcd = nd.rev_srcd;
    const uint32_t* __restrict__ rev_fwd = nd.rev_fwd;
    float* __restrict__ P = nd.Pacc;
    float* __restrict__ Dacc = nd.Dacc;
    const float decay = nd.sd_decay;
    const uint32_t ct = br.x;
    if (threadIdx.x < kSlots) smap[threadIdx.x] = nd.srcmap[ct * kSlots + threadIdx.x];
    __syncthreads();
    const uint64_t colsz = (uint64_t)d.Ncol * d.M;
    const uint64_t chunk = (uint64_t)blockDim.x * kWupdateItems;
    const uint64_t x0 = nd.rowptr[(size_t)ct * d.Ncol] + (uint64_t)br.y * chunk;
    const uint64_t x1 = min(x0 + chunk, nd.rowptr[(size_t)(ct + 1) * d.Ncol]);
    for (uint64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
        const uint64_t f = (uint64_t)smap[rev_srcd[x] >> 22] * colsz + rev_fwd[x];
        const float sd = P[x] - Dacc[f];
        Dacc[f] = sd;
        P[x] = decay * sd;
    }
}

// Consolidation in one pass over the forward order, for networks that keep
// fwd_rev: for excitatory position f of column c with fwd_rev[f] = slot << 28
// | o, the reverse entry is x = (first reverse position of the column
// reached from c through slot) + o, and
//   sd = P[x] - D[f]; w[f] <- clamp(w[f] + (bias + sd)); D[f] <- 0;
//   P[x] <- decay * sd,
// the same operations, in the same precision, as the two passes above.
// Workgroup (column c, group q) takes the excitatory source neurons
// [q*G, q*G + G) of c: their synapses of every delay, Dmax contiguous
// ranges of the forward order, so w, D and fwd_rev stream (non-temporal
// accesses: they are touched once and should not push P out of L2).  The
// reverse rows are sorted by (slot, source, delay), so the P entries of a
// run of source neurons are one short stretch of each target row's run for
// that slot, and the few hundred source neurons in flight on an XCD (two
// 1024-thread workgroups per CU) touch P lines that stay in its L2 until the
// next neurons reuse them.  Work maps (`order`): with 1 and 2 all groups of
// a column run on one XCD (the hardware hands workgroup b to XCD b mod 8);
// for k = b / 8, step s = k / Q takes group k mod Q of
//   1: column 8 s + b mod 8 (the eight XCDs on consecutive columns),
//   2: column (x, y) = (8 (s / GY) + b mod 8, s mod GY): the XCDs walk the
//      grid in strips of 8 columns, top to bottom, so the columns that share
//      target columns run close together in time (grids with GX a multiple
//      of 8);
//   0: column b / Q, group b mod Q (fewer than 64 columns).
constexpr uint32_t kConsUnroll = 4;      // forward positions in flight per thread
constexpr uint32_t kConsSynapses = 2048; // synapses per workgroup (sets G)

template <uint32_t U>
__global__ __launch_bounds__(1024) void k_consolidate(const NetDesc* __restrict__ nds, uint32_t G,
                                                      uint32_t Q, uint32_t order) {
    __shared__ uint64_t base[16];  // first reverse position of the column in each slot
    __shared__ uint64_t s0[32];    // first forward position of each delay's range
    __shared__ uint32_t pre[33];   // prefix sums of the ranges' lengths
    const NetDesc& nd = *nds;
    const Dims d = nd.d;
    uint32_t c, q;
    if (order == 2u) {
        const uint32_t k = blockIdx.x >> 3;
        const uint32_t st = k / Q;
        const uint32_t cx = (st / d.GY) * 8u + (blockIdx.x & 7u);
        if (cx >= d.GX) return;
        c = (st % d.GY) * d.GX + cx;
        q = k % Q;
    } else if (order == 1u) {
        const uint32_t k = blockIdx.x >> 3;
        c = (k / Q) * 8u + (blockIdx.x & 7u);
        q = k % Q;
    } else {
        c = blockIdx.x / Q;
        q = blockIdx.x % Q;
    }
    if (c >= d.C) return;
    const uint32_t l0 = q * G;
    const uint32_t l1 = min(l0 + G, d.Ne);
    if (threadIdx.x < kSlots)
        base[threadIdx.x] = nd.rowptr[(size_t)nd.colmap[c * kSlots + threadIdx.x] * d.Ncol];
    if (threadIdx.x < 64u) {
        // segment (delay k+1, neuron l) of column c starts at
        // seg_off[c*segs + k*Ncol + l]; index k*Ncol + Ncol is the next
        // delay's first segment (or the next column's, or the sentinel)
        const uint32_t k = threadIdx.x;
        uint32_t len = 0;
        if (k < d.Dmax) {
            const uint64_t* so = nd.seg_off + (size_t)c * d.segs + (size_t)k * d.Ncol;
            const uint64_t a = so[l0];
            s0[k] = a;
            len = (uint32_t)(so[l1] - a);
        }
        uint32_t inc = len;
#pragma unroll
        for (int o = 1; o < 32; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (k >= (uint32_t)o) inc += y;
        }
        if (k < 32u) pre[k + 1] = inc;
        if (k == 0u) pre[0] = 0u;
    }
    __syncthreads();
    const uint32_t* __restrict__ fwd_rev = nd.fwd_rev;
    float* __restrict__ P = nd.Pacc;
    float* __restrict__ Dacc = nd.Dacc;
    float* __restrict__ w = (float*)nd.w;
    const float bias = nd.wu_bias, wmax = nd.w_max, decay = nd.sd_decay;
    const uint32_t total = pre[d.Dmax];
    for (uint32_t i0 = threadIdx.x; i0 < total; i0 += U * blockDim.x) {
        // U positions per thread: every load issued before the first store
        uint64_t f[U], x[U];
        float dv[U], wv[U], pv[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * blockDim.x;
            f[u] = ~0ull;
            if (i < total) {
                // the last range k with pre[k] <= i (empty ranges are skipped)
                uint32_t lo = 0, hi = d.Dmax;
                while (hi - lo > 1u) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (pre[mid] <= i) lo = mid;
                    else hi = mid;
                }
                f[u] = s0[lo] + (i - pre[lo]);
                const uint32_t code = __builtin_nontemporal_load(&fwd_rev[f[u]]);
                x[u] = base[code >> 28] + (code & 0x0FFFFFFFu);
                dv[u] = __builtin_nontemporal_load(&Dacc[f[u]]);
                wv[u] = __builtin_nontemporal_load(&w[f[u]]);
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u)
            if (f[u] != ~0ull) pv[u] = P[x[u]];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            if (f[u] == ~0ull) continue;
            const float sd = pv[u] - dv[u];
            float nw = wv[u] + (bias + sd);
            if (nw < 0.0f) nw = 0.0f;
            if (nw > wmax) nw = wmax;
            __builtin_nontemporal_store(nw, &w[f[u]]);
            __builtin_nontemporal_store(0.0f, &Dacc[f[u]]);
            P[x[u]] = decay * sd;
        }
    }
}

// State probes (Sec. 2, "Production of observables": the trace of the
// membrane potential and other state variables of individual neurons): after
// the neuron update of step t, v and u of each probed neuron into row
// (t + 1) % R of the network's probe ring.  Workgroups (chunk x, member y).
__global__ __launch_bounds__(256) void k_probe(const NetDesc* __restrict__ nds, uint32_t tstep) {
    const NetDesc& nd = nds[blockIdx.y];
    const uint32_t n = nd.probe_n;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const uint32_t t = nd.t0 + tstep;
    float* row = nd.probe_buf + (size_t)((t + 1u) % nd.d.R) * 2u * n;
    const uint32_t k = nd.probe_id[p];
    row[p] = nd.v[k];
    row[n + p] = nd.u[k];
}

// t0 += delta for each of the K descriptors of a launch set
__global__ __launch_bounds__(64) void k_rebase(NetDesc* __restrict__ nds, uint32_t K, uint32_t delta) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < K) nds[k].t0 += delta;
}

__global__ __launch_bounds__(256) void k_wupdate_fwd(const NetDesc* __restrict__ nds) {
    const NetDesc& nd = *nds;
    const Dims d = nd.d;
    const uint64_t* __restrict__ seg_off = nd.seg_off;
    float* __restrict__ Dacc = nd.Dacc;
    float* __restrict__ w = (float*)nd.w;
    const float bias = nd.wu_bias, wmax = nd.w_max;
    const uint64_t S = (uint64_t)d.N * d.M;
    const uint64_t colsz = (uint64_t)d.Ncol * d.M;
    const uint64_t chunk = (uint64_t)blockDim.x * kWupdateItems;
    const uint64_t f0 = (uint64_t)blockIdx.x * chunk;
    const uint64_t f1 = min(f0 + chunk, S);
    uint32_t cur = 0xFFFFFFFFu;
    uint64_t lo = 0, hi = 0;  // inhibitory range of column cur
    for (uint64_t f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
        const uint32_t c = (uint32_t)(f / colsz);
        if (c != cur) {
            cur = c;
            const size_t s1 = (size_t)c * d.segs;
            lo = d.Ne < d.Ncol ? seg_off[s1 + d.Ne] : 0ull;
            hi = d.Ne < d.Ncol ? seg_off[s1 + d.Ncol] : 0ull;
        }
        if (f >= lo && f < hi) continue;
        float nw = w[f] + (bias + Dacc[f]);
        if (nw < 0.0f) nw = 0.0f;
        if (nw > wmax) nw = wmax;
        w[f] = nw;
        Dacc[f] = 0.0f;
    }
}

template <typename K>
void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536)
        (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)bytes);
}

// Workgroups per column for delivery and LTP: sets with fewer columns than
// a few per compute unit split every column into equal parts, each part at
// least about 8 K synapses of the smallest column.  The results do not
// depend on the split.
uint32_t column_parts(const LaunchSet& L, const Tuning& tune) {
    if (L.sum_mode == DPSNN_SUM_ORDERED || L.n_col == 0) return 1u;
    if (tune.parts) return tune.parts;
    const uint32_t target = 512u;  // two workgroups per compute unit
    if (L.n_col >= target) return 1u;
    const uint64_t want = (target + L.n_col - 1u) / L.n_col;
    const uint64_t cap = std::max<uint64_t>(1u, L.min_col_syn / 8192u);
    return (uint32_t)std::min<uint64_t>(std::min<uint64_t>(want, cap), 1024u);
}

// LTP launch parameters handed to launch_deliver when the two are fused.
struct FusedLtp {
    bool on = false;
    uint32_t allow_stage = 0;
    size_t lds = 0;
    uint32_t sparse = 0;   // LTP by the wavefront-level sparse body
    uint32_t cpw = 1;      // sparse LTP: target columns per workgroup
    uint32_t nwg = 0;      // sparse LTP workgroups when cpw > 1 (a multiple of 8)
};

template <typename TgtT>
hipError_t launch_deliver(LaunchSet& L, const Tuning& tune, hipStream_t stream, Net* const* members,
                          uint32_t nparts, uint32_t tstep, const FusedLtp& fl) {
    if (L.sum_mode == DPSNN_SUM_ORDERED) {
        // one network only (checked when the set is made)
        Net& n = *members[0];
        hipLaunchKernelGGL((k_deliver_seq<0, TgtT>), dim3(L.n_col), dim3(256), 0, stream, L.descs,
                           L.bmap_col, tstep);
        if (n.t >= 1) {
            hipError_t e = scan_u32(n, stream, n.ev_cnt, n.ev_start, n.d.N);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_deliver_seq<1, TgtT>), dim3(L.n_col), dim3(256), 0, stream, L.descs,
                           L.bmap_col, tstep);
        return hipGetLastError();
    }
    const bool fixed = L.sum_mode == DPSNN_SUM_FIXED;
    // one thread per raster word of a column and delay chunk
    const uint32_t BS = std::max<uint32_t>(tune.deliver_block, ((L.max_w + 63) / 64) * 64);
    const size_t esz = 8;  // fixed-point window entries in every mode
    // the full window may be shared out by slot over nsplit workgroups
    const uint32_t split_req = std::min<uint32_t>(std::max<uint32_t>(tune.split, 1u), (uint32_t)kSlots);
    const uint32_t share = (kSlots + split_req - 1u) / split_req;  // most slots of one share
    const size_t win_full = (((size_t)share * L.max_ncol * esz) + 15) & ~(size_t)15;
    const uint32_t wslots = std::min<uint32_t>(std::max<uint32_t>(tune.own_slots, 1u), (uint32_t)kSlots);
    const size_t win_own = (((size_t)wslots * L.max_ncol * esz) + 15) & ~(size_t)15;
    const size_t base = ((size_t)3 * BS + 1 + 20 + 16 + 64) * sizeof(uint32_t);
    // window mode: the requested one if it fits, else the own-column window
    // if that fits, else none
    int wmode = 0;
    if (tune.window == 1 && win_full + base + 256 <= tune.max_lds) wmode = 1;
    else if (tune.window >= 1 && win_own + base + 256 <= tune.max_lds) wmode = 2;
    const uint32_t nsplit = wmode == 1 ? split_req : 1u;
    const size_t agew = (((size_t)(wmode == 1 ? share : (wmode == 2 ? wslots : (uint32_t)kSlots)) *
                          L.max_ncol) + 15) & ~(size_t)15;
    const size_t lds0 = (wmode == 1 ? win_full : (wmode == 2 ? win_own : 0)) + base;
    const uint32_t allow_age = (tune.age && lds0 + agew + 256 <= tune.max_lds) ? 1u : 0u;
    const size_t lds = lds0 + (allow_age ? agew : 0);
    const uint32_t n_ltp = L.n_col * nparts;
    const uint32_t nblk = n_ltp * nsplit;
    // LTP workgroups of the fused launch (fewer when one takes several columns)
    const uint32_t n_ltpw = fl.cpw > 1u ? fl.nwg : n_ltp;
#define DPSNN_DELIVER(FX, WN, UU)                                                              \
    do {                                                                                       \
        if (fl.on) {                                                                           \
            const size_t lf = std::max(lds, fl.lds);                                           \
            allow_lds(k_ltp_deliver<FX, WN, TgtT, UU>, lf);                                    \
            hipLaunchKernelGGL((k_ltp_deliver<FX, WN, TgtT, UU>), dim3(n_ltpw + nblk), dim3(BS), \
                               lf, stream, L.descs, L.bmap_col, fl.allow_stage, allow_age,     \
                               nparts, nsplit, wslots, L.ev_count, tstep, n_ltpw, fl.sparse,   \
                               fl.cpw, L.n_col);                                               \
        } else {                                                                               \
            allow_lds(k_deliver<FX, WN, TgtT, UU>, lds);                                       \
            hipLaunchKernelGGL((k_deliver<FX, WN, TgtT, UU>), dim3(nblk), dim3(BS), lds,       \
                               stream, L.descs, L.bmap_col, allow_age, nparts, nsplit, wslots, \
                               L.ev_count, tstep);                                             \
        }                                                                                      \
    } while (0)
#define DPSNN_DELIVER_W(FX, UU)                                                                \
    do {                                                                                       \
        if (wmode == 1) DPSNN_DELIVER(FX, 1, UU);                                              \
        else if (wmode == 2) DPSNN_DELIVER(FX, 2, UU);                                         \
        else DPSNN_DELIVER(FX, 0, UU);                                                         \
    } while (0)
    if (tune.unroll == 1) {
        if (fixed) DPSNN_DELIVER_W(true, 1); else DPSNN_DELIVER_W(false, 1);
    } else if (tune.unroll == 2) {
        if (fixed) DPSNN_DELIVER_W(true, 2); else DPSNN_DELIVER_W(false, 2);
    } else if (tune.unroll == 4) {
        if (fixed) DPSNN_DELIVER_W(true, 4); else DPSNN_DELIVER_W(false, 4);
    } else {
        if (fixed) DPSNN_DELIVER_W(true, 8); else DPSNN_DELIVER_W(false, 8);
    }
#undef DPSNN_DELIVER_W
#undef DPSNN_DELIVER
    return hipGetLastError();
}

// The wavefront-level sparse paths (LTP and delivery; FIXED or ATOMIC
// summation), fused into one launch when the fuse rule allows.
template <typename TgtT>
hipError_t launch_sparse(LaunchSet& L, const Tuning& tune, Timers& tm, hipStream_t stream,
                         uint32_t nparts, uint32_t tstep) {
    const bool fixed = L.sum_mode == DPSNN_SUM_FIXED;
    auto pad16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
    // delivery: the LDS window over the first wslots slots (fewer if it does
    // not fit), the own column's spike ages and three queues
    uint32_t wslots = std::min<uint32_t>(std::max<uint32_t>(tune.own_slots, 1u), (uint32_t)kSlots);
    auto lds_for = [&](uint32_t ws) {
        return pad16((size_t)ws * L.max_ncol * 8) + pad16(L.max_ncol) + 3 * sizeof(uint32_t) * kQueue;
    };
    while (wslots > 0 && lds_for(wslots) + 2048 > tune.max_lds) --wslots;
    const size_t lds_d = lds_for(wslots);
    // LTP: the own column's spike history (8 bytes per neuron) when it fits
    const size_t hist_b = (size_t)L.max_ncol * 8;
    const uint32_t allow_stage = (tune.ltp_stage && hist_b <= 32768 && hist_b + 2048 <= tune.max_lds) ? 1u : 0u;
    const size_t lds_l = allow_stage ? hist_b : 0;
    const uint32_t n = L.n_col * nparts;
    if ((uint64_t)n <= tune.fuse) {
        const size_t lds = std::max(lds_d, lds_l);
        tm.begin(1, stream);
        if (fixed) {
            allow_lds(k_ltp_deliver_sp<true, TgtT>, lds);
            hipLaunchKernelGGL((k_ltp_deliver_sp<true, TgtT>), dim3(2 * n), dim3(256), lds, stream,
                               L.descs, L.bmap_col, nparts, wslots, allow_stage, L.ev_count, tstep, n);
        } else {
            allow_lds(k_ltp_deliver_sp<false, TgtT>, lds);
            hipLaunchKernelGGL((k_ltp_deliver_sp<false, TgtT>), dim3(2 * n), dim3(256), lds, stream,
                               L.descs, L.bmap_col, nparts, wslots, allow_stage, L.ev_count, tstep, n);
        }
        tm.end(stream);
        return hipGetLastError();
    }
    tm.begin(0, stream);
    hipLaunchKernelGGL(k_ltp_sp, dim3(n), dim3(256), lds_l, stream, L.descs, L.bmap_col, nparts,
                       allow_stage, 1u, n, n, tstep);
    tm.end(stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    tm.begin(1, stream);
    if (fixed) {
        allow_lds(k_deliver_sp<true, TgtT>, lds_d);
        hipLaunchKernelGGL((k_deliver_sp<true, TgtT>), dim3(n), dim3(256), lds_d, stream, L.descs,
                           L.bmap_col, nparts, wslots, L.ev_count, tstep);
    } else {
        allow_lds(k_deliver_sp<false, TgtT>, lds_d);
        hipLaunchKernelGGL((k_deliver_sp<false, TgtT>), dim3(n), dim3(256), lds_d, stream, L.descs,
                           L.bmap_col, nparts, wslots, L.ev_count, tstep);
    }
    tm.end(stream);
    return hipGetLastError();
}

}  // namespace

void Timers::begin(int kind, hipStream_t s) {
    if (!on) return;
    Timed tt;
    tt.kind = kind;
    if (pool.size() >= 2) {
        tt.a = pool.back(); pool.pop_back();
        tt.b = pool.back(); pool.pop_back();
    } else {
        (void)hipEventCreate(&tt.a);
        (void)hipEventCreate(&tt.b);
    }
    (void)hipEventRecord(tt.a, s);
    pending.push_back(tt);
}

void Timers::end(hipStream_t s) {
    if (!on) return;
    (void)hipEventRecord(pending.back().b, s);
}

void Timers::collect() {
    for (auto& tt : pending) {
        float x = 0.0f;
        if (hipEventElapsedTime(&x, tt.a, tt.b) == hipSuccess) {
            ms[tt.kind] += x;
            n[tt.kind] += 1;
        }
        pool.push_back(tt.a);
        pool.push_back(tt.b);
    }
    pending.clear();
}

void Timers::release() {
    for (auto& tt : pending) {
        (void)hipEventDestroy(tt.a);
        (void)hipEventDestroy(tt.b);
    }
    pending.clear();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

// Regime estimate of the set: fold in the last counter copy once it has
// landed, and start a new copy every 8 steps.  A copy still in flight 16
// steps after it was enqueued is waited for, which keeps the host at most
// about 16 steps ahead of the device and the estimate at most that stale.
void sample_regime(LaunchSet& L, hipStream_t stream, Net* const* members) {
    // sets under 64 columns always take the dense shapes: nothing to measure
    if (!L.ev_host || !L.ev_copied || L.n_col < 64u) return;
    bool landed = false;
    if (L.copy_pending) {
        hipError_t q = hipEventQuery(L.ev_copied);
        if (q == hipErrorNotReady && L.steps - L.copy_steps >= 16u) q = hipEventSynchronize(L.ev_copied);
        landed = q == hipSuccess;
    }
    if (landed) {
        const unsigned long long v = *(volatile unsigned long long*)L.ev_host;
        if (L.copy_steps > L.base_steps && L.n_col) {
            L.per_col = (double)(v - L.base_count) / (double)(L.copy_steps - L.base_steps) /
                        (double)L.n_col;
            for (uint32_t k = 0; k < L.K; ++k) members[k]->per_col = L.per_col;
            if (L.sparse && L.per_col > L.avg_nwin) L.sparse = false;
            else if (!L.sparse && L.per_col < 0.8 * L.avg_nwin) L.sparse = true;
        }
        L.base_count = v;
        L.base_steps = L.copy_steps;
        L.copy_pending = false;
    }
    if (!L.copy_pending && L.steps - L.copy_steps >= 8u) {
        if (hipMemcpyAsync(L.ev_host, L.ev_count, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           stream) == hipSuccess &&
            hipEventRecord(L.ev_copied, stream) == hipSuccess) {
            L.copy_pending = true;
            L.copy_steps = L.steps;
        }
    }
}

// The launch shapes for this step: explicit knobs as set, automatic ones by
// the set's regime.  Sparse shapes (small LDS, 256-thread workgroups, several
// per CU) pay off when each source column delivers fewer events than its
// current window has entries and there are enough workgroups (at least 512
// column parts, from at least 64 columns) to fill the chip; otherwise the
// full window and 1024-thread workgroups are faster.
Tuning effective_tuning(const LaunchSet& L, const Tuning& tune) {
    Tuning t = tune;
    const uint64_t wgs = (uint64_t)L.n_col * column_parts(L, tune);
    const bool many = L.n_col >= 2048u || (L.n_col >= 64u && wgs >= 512u);
    const bool sparse = many && L.sparse;
    // sparse shapes split the columns of sets of 512 .. 1023 columns in two
    // (smaller sets keep the parts above: measured best)
    if (sparse && !t.parts && L.sum_mode != DPSNN_SUM_ORDERED && L.n_col >= 512u &&
        L.n_col < 1024u) {
        const uint64_t want = (1024u + L.n_col - 1u) / L.n_col;
        const uint64_t cap = std::max<uint64_t>(1u, L.min_col_syn / 8192u);
        t.parts = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(want, cap), 1024u);
    }
    if (!t.deliver_block) t.deliver_block = sparse ? 256u : 1024u;
    if (!t.ltp_block) t.ltp_block = sparse ? 256u : 1024u;
    if (t.window == 3u) t.window = sparse ? 2u : 1u;
    if (t.age == 2u) t.age = sparse ? 0u : 1u;
    if (t.ltp_stage == 2u) t.ltp_stage = sparse ? 0u : 1u;
    // the partial window: the own column alone on grids below 2048 columns,
    // the own column and two neighbour slots on larger ones (measured)
    if (t.own_slots == 0u) t.own_slots = (sparse && L.n_col >= 2048u) ? 3u : 1u;
    if (t.sparse_ltp == 2u) t.sparse_ltp = sparse ? 1u : 0u;
    if (t.ltp_cols == 0u) t.ltp_cols = 1u;
    if (t.sparse_deliver == 2u) t.sparse_deliver = 0u;  // measured slower than the run path
    return t;
}

namespace {

bool same_shapes(const Tuning& a, const Tuning& b) {
    return a.deliver_block == b.deliver_block && a.ltp_block == b.ltp_block && a.window == b.window &&
           a.unroll == b.unroll && a.age == b.age && a.parts == b.parts && a.ltp_stage == b.ltp_stage &&
           a.fuse == b.fuse && a.split == b.split && a.own_slots == b.own_slots &&
           a.sparse_ltp == b.sparse_ltp && a.sparse_deliver == b.sparse_deliver &&
           a.ltp_cols == b.ltp_cols && a.consolidate == b.consolidate &&
           a.max_lds == b.max_lds;
}

// The kernels of one step of every network of the set at t = t0 + tstep, in
// the paper's loop order: LTP, delivery (+ currents and LTD), neuron update,
// and consolidation for the members flagged in `wu`.  `spikes`: some member
// is past its first step.  Changes no host state except the timers.  Timer
// kinds: 0 LTP, 1 delivery, 2 neuron, 3 consolidation.
hipError_t enqueue_step(LaunchSet& L, const Tuning& tune, Timers& tm, hipStream_t stream,
                        Net* const* members, uint32_t tstep, bool any_spikes, const uint8_t* wu) {
    hipError_t e;
    if (any_spikes && tune.sparse_deliver && L.sum_mode != DPSNN_SUM_ORDERED) {
        const uint32_t nparts = column_parts(L, tune);
        e = L.tgt16 ? launch_sparse<uint16_t>(L, tune, tm, stream, nparts, tstep)
                    : launch_sparse<uint32_t>(L, tune, tm, stream, nparts, tstep);
        if (e != hipSuccess) return e;
    } else if (any_spikes) {
        const uint32_t BSd = std::max<uint32_t>(tune.deliver_block, ((L.max_w + 63) / 64) * 64);
        const bool ltp_sp = tune.sparse_ltp != 0u;
        const uint32_t BS = ltp_sp ? BSd : std::max<uint32_t>(tune.ltp_block, ((L.max_w + 63) / 64) * 64);
        size_t lds;
        uint32_t allow;
        if (ltp_sp) {
            // the sparse LTP body stages the own column's spike history
            const size_t hist_b = (size_t)L.max_ncol * 8;
            allow = (tune.ltp_stage && hist_b <= 32768 && hist_b + 2048 <= tune.max_lds) ? 1u : 0u;
            lds = allow ? hist_b : 0;
        } else {
            const size_t base = ((size_t)2 * BS + 1 + 20 + 16 + 64) * sizeof(uint32_t);
            const size_t hw = (size_t)kSlots * L.max_ncol * sizeof(uint32_t);
            allow = (tune.ltp_stage && base + hw <= tune.max_lds) ? 1u : 0u;
            lds = base + (allow ? hw : 0);
        }
        const uint32_t nparts = column_parts(L, tune);
        // small launches run LTP and delivery as one kernel (same workgroup size)
        FusedLtp fl;
        fl.on = L.sum_mode != DPSNN_SUM_ORDERED && BSd == BS &&
                (uint64_t)L.n_col * nparts <= tune.fuse;
        fl.allow_stage = allow;
        fl.lds = lds;
        fl.sparse = ltp_sp ? 1u : 0u;
        // several columns per sparse LTP workgroup: one network, unsplit columns
        fl.cpw = (ltp_sp && L.K == 1 && nparts == 1u) ? std::max<uint32_t>(1u, tune.ltp_cols) : 1u;
        if (fl.cpw > 1u) {
            fl.nwg = ((L.n_col + fl.cpw - 1u) / fl.cpw + kXcds - 1u) / kXcds * kXcds;
            fl.allow_stage = 0u;
        }
        if (!fl.on && ltp_sp) {
            const uint32_t nl = fl.cpw > 1u ? fl.nwg : L.n_col * nparts;
            tm.begin(0, stream);
            hipLaunchKernelGGL(k_ltp_sp, dim3(nl), dim3(256), lds, stream, L.descs,
                               L.bmap_col, nparts, fl.allow_stage, fl.cpw, nl, L.n_col, tstep);
            tm.end(stream);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        } else if (!fl.on) {
            allow_lds(k_ltp<4>, lds);
            tm.begin(0, stream);
            hipLaunchKernelGGL(k_ltp<4>, dim3(L.n_col * nparts), dim3(BS), lds, stream, L.descs,
                               L.bmap_col, allow, nparts, tstep);
            tm.end(stream);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        tm.begin(1, stream);
        e = L.tgt16 ? launch_deliver<uint16_t>(L, tune, stream, members, nparts, tstep, fl)
                    : launch_deliver<uint32_t>(L, tune, stream, members, nparts, tstep, fl);
        tm.end(stream);
        if (e != hipSuccess) return e;
    }
    tm.begin(2, stream);
    if (L.sum_mode == DPSNN_SUM_FIXED)
        hipLaunchKernelGGL(k_neuron<DPSNN_SUM_FIXED>, dim3(L.n_neu), dim3(256), 0, stream, L.descs, L.bmap_neu, tstep);
    else if (L.sum_mode == DPSNN_SUM_ATOMIC)
        hipLaunchKernelGGL(k_neuron<DPSNN_SUM_ATOMIC>, dim3(L.n_neu), dim3(256), 0, stream, L.descs, L.bmap_neu, tstep);
    else
        hipLaunchKernelGGL(k_neuron<DPSNN_SUM_ORDERED>, dim3(L.n_neu), dim3(256), 0, stream, L.descs, L.bmap_neu, tstep);
    tm.end(stream);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (L.max_probes) {
        hipLaunchKernelGGL(k_probe, dim3((L.max_probes + 255u) / 256u, L.K), dim3(256), 0, stream,
                           L.descs, tstep);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    for (uint32_t k = 0; wu && k < L.K; ++k) {
        if (!wu[k]) continue;
        const Net& n = *members[k];
        tm.begin(3, stream);
        if (n.fwd_rev && tune.consolidate) {
            const uint32_t G = std::max<uint32_t>(1u, (kConsSynapses + n.d.M - 1u) / n.d.M);
            const uint32_t Q = (n.d.Ne + G - 1u) / G;
            const uint32_t order = n.d.C < 64u ? 0u : (n.d.GX % 8u == 0u ? 2u : 1u);
            const uint64_t nwg = order == 2u ? 8ull * Q * (n.d.GX / 8u) * n.d.GY
                                 : order == 1u ? 8ull * Q * ((n.d.C + 7u) / 8u)
                                               : (uint64_t)Q * n.d.C;
            hipLaunchKernelGGL(k_consolidate<kConsUnroll>, dim3((uint32_t)nwg), dim3(1024), 0, stream,
                               L.descs + k, G, Q, order);
        } else {
            hipLaunchKernelGGL(k_wupdate, dim3(L.n_wu[k]), dim3(256), 0, stream, L.descs + k, L.bmap_wu[k]);
            const uint64_t nfwd = ((uint64_t)n.S + 256ull * kWupdateItems - 1) / (256ull * kWupdateItems);
            hipLaunchKernelGGL(k_wupdate_fwd, dim3((uint32_t)nfwd), dim3(256), 0, stream, L.descs + k);
        }
        tm.end(stream);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Steps until member n's next consolidation (0: due in its current step).
uint32_t steps_to_consolidation(const LaunchSet& L, const Net& n, uint32_t k) {
    const uint32_t Tw = n.cfg.weight_update_period;
    if (!Tw || !n.S_exc || !L.n_wu[k]) return 0xFFFFFFFFu;
    const uint32_t r = (n.t + 1u) % Tw;
    return r == 0 ? 0u : Tw - r;
}

// Step offset common to the members (t - t0); false if they disagree.
bool set_tstep(const LaunchSet& L, Net* const* members, uint32_t& tstep) {
    tstep = members[0]->t - L.host_descs[0].t0;
    for (uint32_t k = 1; k < L.K; ++k)
        if (members[k]->t - L.host_descs[k].t0 != tstep) return false;
    return true;
}

// Steps [t, t + G) of every member as one captured graph, replayed on
// `stream`.  The graph holds the G steps' kernels at tstep 0 .. G-1 followed
// by k_rebase(G), so it starts from descriptors with t0 = t: a set whose
// offset is not 0 is rebased first.  It is captured again when G or the
// launch shapes change.  Only steps without consolidation and past the first
// are graphed; there are no memory-set nodes.
hipError_t launch_graph(LaunchSet& L, const Tuning& tune, hipStream_t stream, Net* const* members,
                        uint32_t G) {
    hipError_t e;
    uint32_t tstep;
    if (!set_tstep(L, members, tstep)) return hipErrorInvalidValue;
    if (L.graph && (L.graph_steps != G || !same_shapes(L.graph_tune, tune) ||
                    L.graph_probes != L.max_probes)) {
        (void)hipGraphExecDestroy(L.graph);
        L.graph = nullptr;
    }
    if (tstep) {
        hipLaunchKernelGGL(k_rebase, dim3((L.K + 63u) / 64u), dim3(64), 0, stream, L.descs, L.K, tstep);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        for (uint32_t k = 0; k < L.K; ++k) L.host_descs[k].t0 += tstep;
    }
    if (!L.graph) {
        if (!L.cap_stream && (e = hipStreamCreateWithFlags(&L.cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return e;
        if ((e = hipStreamBeginCapture(L.cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
        Timers off;
        hipError_t ce = hipSuccess;
        for (uint32_t j = 0; j < G && ce == hipSuccess; ++j)
            ce = enqueue_step(L, tune, off, L.cap_stream, members, j, true, nullptr);
        if (ce == hipSuccess) {
            hipLaunchKernelGGL(k_rebase, dim3((L.K + 63u) / 64u), dim3(64), 0, L.cap_stream, L.descs, L.K, G);
            ce = hipGetLastError();
        }
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(L.cap_stream, &g);  // always ends the capture
        if (ce == hipSuccess) ce = e;
        if (ce == hipSuccess) ce = hipGraphInstantiate(&L.graph, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (ce != hipSuccess) {
            L.graph = nullptr;
            return ce;
        }
        L.graph_steps = G;
        L.graph_tune = tune;
        L.graph_probes = L.max_probes;
    }
    if ((e = hipGraphLaunch(L.graph, stream)) != hipSuccess) return e;
    for (uint32_t k = 0; k < L.K; ++k) {
        L.host_descs[k].t0 += G;
        members[k]->t += G;
        members[k]->graph_steps += G;
    }
    L.steps += G;
    sample_regime(L, stream, members);
    return hipSuccess;
}

}  // namespace

// One step, launched directly (see enqueue_step), and the host bookkeeping:
// regime sample, consolidation count, clock.
hipError_t launch_step_set(LaunchSet& L, const Tuning& tune_in, Timers& tm, hipStream_t stream,
                           Net* const* members) {
    if (L.K == 0) return hipSuccess;
    const Tuning tune = effective_tuning(L, tune_in);
    // every member has advanced by the same number of steps since its
    // descriptor's t0 was set; the kernels read t = t0 + tstep
    uint32_t tstep;
    if (!set_tstep(L, members, tstep)) return hipErrorInvalidValue;
    bool any_spikes = false;
    for (uint32_t k = 0; k < L.K; ++k) any_spikes |= members[k]->t >= 1;
    std::vector<uint8_t> wu(L.K);
    for (uint32_t k = 0; k < L.K; ++k) wu[k] = steps_to_consolidation(L, *members[k], k) == 0;
    hipError_t e = enqueue_step(L, tune, tm, stream, members, tstep, any_spikes, wu.data());
    if (e != hipSuccess) return e;
    if (any_spikes) {
        L.steps++;
        sample_regime(L, stream, members);
    }
    for (uint32_t k = 0; k < L.K; ++k) {
        if (wu[k]) members[k]->consolidations++;
        members[k]->t += 1;
    }
    return hipSuccess;
}

// n_steps steps: runs of tune.graph steps that need no consolidation, no
// timers and no first step are replayed as captured graphs, the rest are
// launched one by one.  The results are the same either way.
hipError_t launch_steps(LaunchSet& L, const Tuning& tune_in, Timers& tm, hipStream_t stream,
                        Net* const* members, uint32_t n_steps) {
    const uint32_t G = tune_in.graph;
    uint32_t s = 0;
    while (s < n_steps) {
        bool graphed = G && n_steps - s >= G && !tm.on && L.K && L.sum_mode != DPSNN_SUM_ORDERED;
        for (uint32_t k = 0; graphed && k < L.K; ++k)
            graphed = members[k]->t >= 1 && steps_to_consolidation(L, *members[k], k) >= G;
        const Tuning eff = effective_tuning(L, tune_in);
        // a capture costs about as much as several steps of a small network:
        // capture only when this call replays the graph at least 4 times, or
        // reuse one captured before with the same run length and shapes
        if (graphed && n_steps - s < 4u * G)
            graphed = L.graph && L.graph_steps == G && same_shapes(L.graph_tune, eff) &&
                      L.graph_probes == L.max_probes;
        hipError_t e;
        if (graphed) {
            e = launch_graph(L, eff, stream, members, G);
            s += G;
        } else {
            e = launch_step_set(L, tune_in, tm, stream, members);
            s += 1;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dpsnn
