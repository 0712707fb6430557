// Device-side definitions shared by the HIP kernels of libdpsnn.
//
// Network generation follows Sec. 2 of Paolucci et al. (arXiv 1310.8478):
// every neuron projects M forward synapses with an individual delay, weight
// and target; inhibitory neurons target excitatory neurons of their own
// column with the minimum delay; excitatory neurons target their own column
// and its first, second and third neighbours on a periodic grid; the draws
// are keyed by global ids so the network is independent of the launch shape
// ("Distributed generation of reproducible connections").
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpsnn {

constexpr int kSlots = 13;                 // own column + 12 neighbour columns
constexpr uint32_t kTagSyn = 0x53594E00u;  // counter word 2 of synapse draws
constexpr uint32_t kTagThal = 0x5448414Cu; // counter word 2 of thalamic draws
constexpr int32_t kNoSpike = INT32_MIN;
constexpr uint32_t kHistBits = 32;         // spike-history window in steps
constexpr uint32_t kWupdateItems = 16;     // reverse entries per thread in consolidation

// Network dimensions and generation constants, passed by value to kernels.
struct Dims {
    uint32_t N, C, Ncol, Ne, M, Dmax, GX, GY;
    uint32_t W;            // 64-bit raster words per column (Ncol padded to 64)
    uint32_t R;            // raster ring slots (>= Dmax + 1)
    uint32_t conn_mode, M_own;
    uint32_t paper_end[kSlots];  // cumulative synapse-index ends of the paper blocks
    uint32_t key0, key1;
    float w_exc, w_inh;
    uint32_t segs;         // Dmax * Ncol (source neuron, delay) segments per column
    uint32_t ncol_magic;   // ceil(2^32 / Ncol): exact quotient for operands < 2^16
};

// Device counters of one network, spread over 64 slots to avoid contention.
struct DevStats {
    unsigned long long spikes, events, ltp_visits, events_exc;
};

// Everything a kernel needs to know about one network: its dimensions and
// device arrays.  Kept in device memory; a launch covering several networks
// maps each workgroup to (network, column or word) through a block table.
struct NetDesc {
    Dims d;
    uint32_t t0;                     // steps completed when the launch set was made
    const uint32_t* colmap;          // [C*13]
    const uint32_t* srcmap;          // [C*13]
    const uint64_t* seg_off;         // [C*segs + 1] forward positions
    const void* tgt;                 // uint16_t or uint32_t [S]
    const float* w;                  // [S]
    float* Dacc;                     // [S]
    const uint64_t* rowptr;          // [N+1] reverse positions
    const uint32_t* rev_srcd;        // [S_exc]
    const uint32_t* rev_fwd;         // [S_exc] forward position - c*Ncol*M of the source column c
    float* Pacc;                     // [S_exc]
    const uint32_t* fwd_rev;         // [S] slot << 28 | reverse entry - target column start, or null
    float* v;
    float* u;
    void* acc;                       // long long or float [N]
    uint2* hist;                     // [N] x: spike history bits, y: t_old (int32)
    int32_t* t_last;
    uint64_t* ring;
    const float* tp;
    const float* tm;
    uint32_t tp_len, tm_len;
    DevStats* stats;                 // [64]
    uint32_t thal_whole, thal_thr;
    float thal_mv;
    const uint32_t* stim_t;          // sorted steps of the stimulus entries
    const uint32_t* stim_id;
    const float* stim_mv;
    uint32_t stim_n;
    uint32_t weight_update_period;
    float wu_bias, sd_decay, w_max;
    unsigned long long S_exc;
    // ORDERED mode buffers (null otherwise)
    uint32_t* ev_cnt;
    const uint32_t* ev_start;
    unsigned long long* ev_key;
    float* ev_w;
    uint32_t* cursor;
    // state probes (null / 0 when none): v and u of probe_n chosen neurons
    // after each step, in a ring of R rows laid out [slot][v | u][probe]
    const uint32_t* probe_id;
    float* probe_buf;
    uint32_t probe_n;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, multipliers
// 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0];
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// floor(x * n / 2^32): a uniform word mapped to [0, n).
__device__ __forceinline__ uint32_t pick(uint32_t x, uint32_t n) { return __umulhi(x, n); }

// Quotient by Ncol for operands below 2^16 (window indices).
__device__ __forceinline__ uint32_t div_ncol(const Dims& d, uint32_t x) {
    return __umulhi(x, d.ncol_magic);
}

struct Syn {
    uint32_t slot;   // target column slot: 0 = own, 1..12 = ring offset slot-1
    uint32_t lt;     // local index of the target in its column
    uint32_t delay;  // ms
    bool exc;
};

// Synapse (i, j): target slot and neuron, delay.  colmap[c*13 + q] is the
// column reached from column c through slot q (periodic wrap).
__device__ __forceinline__ Syn draw_synapse(const Dims& d, const uint32_t* __restrict__ colmap,
                                            uint32_t i, uint32_t j) {
    const uint32_t c = i / d.Ncol;
    const uint32_t l = i - c * d.Ncol;
    uint32_t x[4] = {i, j, kTagSyn, 0u};
    philox10(x, d.key0, d.key1);
    Syn s;
    if (l >= d.Ne) {
        s.slot = 0;
        s.lt = pick(x[1], d.Ne);
        s.delay = 1;
        s.exc = false;
        return s;
    }
    uint32_t q;
    if (d.conn_mode == 1u) {
        q = kSlots - 1;
        for (int k = 0; k < kSlots; ++k) {
            if (j < d.paper_end[k]) { q = (uint32_t)k; break; }
        }
    } else {
        q = (j < d.M_own) ? 0u : 1u + pick(x[0], 12u);
    }
    const uint32_t tc = colmap[c * kSlots + q];
    uint32_t lt;
    if (tc == c) {
        const uint32_t r = pick(x[1], d.Ncol - 1u);
        lt = r + (r >= l ? 1u : 0u);
    } else {
        lt = pick(x[1], d.Ncol);
    }
    s.slot = q;
    s.lt = lt;
    s.delay = 1u + pick(x[2], d.Dmax);
    s.exc = true;
    return s;
}

// Fixed-point current unit: x * 2^32 rounded to the nearest integer, ties to even.
__device__ __forceinline__ long long to_fixed(float x) {
    return __float2ll_rn(x * 4294967296.0f);
}

__device__ __forceinline__ float from_fixed(long long a) {
    return (float)a * (1.0f / 4294967296.0f);
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ unsigned long long lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

// Exclusive scan of one value per thread over the whole block; returns the
// thread's prefix and the block total.  sh must hold blockDim.x/64 + 1 words.
// Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (wid == 0) {
        const uint32_t s = lane < nw ? sh[lane] : 0u;
        uint32_t inc = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o) inc += y;
        }
        if (lane < nw) sh[lane] = inc - s;
        if (lane == nw - 1) sh[nw] = inc;
    }
    __syncthreads();
    const uint32_t res = sh[wid] + x - v;
    total = sh[nw];
    __syncthreads();
    return res;
}

// Block-wide sum reduction of a 64-bit value; result valid in every thread.
__device__ __forceinline__ unsigned long long block_sum64(unsigned long long v, unsigned long long* sh) {
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    unsigned long long t = 0;
    for (uint32_t w = 0; w < nw; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Runs of consecutive spiking neurons in one 64-bit raster word.  Bits of the
// neighbouring words decide whether a run continues across the word edge;
// `split` (0 < split < Ncol) forces a run boundary between split-1 and split.
struct WordRuns {
    unsigned long long starts, ends, word;
};

__device__ __forceinline__ WordRuns word_runs(const uint64_t* __restrict__ words, uint32_t W,
                                              uint32_t w, uint32_t split) {
    const unsigned long long m = words[w];
    const unsigned long long prev_top = (w > 0) ? (words[w - 1] >> 63) : 0ull;
    const unsigned long long next_low = (w + 1 < W) ? (words[w + 1] & 1ull) : 0ull;
    WordRuns r;
    r.word = m;
    r.starts = m & ~((m << 1) | prev_top);
    r.ends = m & ~((m >> 1) | (next_low << 63));
    if (split > 0) {
        if (split / 64 == w) r.starts |= m & (1ull << (split % 64));
        if ((split - 1) / 64 == w) r.ends |= m & (1ull << ((split - 1) % 64));
    }
    return r;
}

// Position of the k-th set bit (k counted from 0) of m.
__device__ __forceinline__ uint32_t nth_bit(unsigned long long m, uint32_t k) {
    for (uint32_t s = 0; s < k; ++s) m &= m - 1ull;
    return (uint32_t)__ffsll((long long)m) - 1u;
}

// Largest r in [lo, n) with pref[r] <= e, given pref[lo] <= e (pref ascending).
__device__ __forceinline__ uint32_t upper_run(const uint32_t* pref, uint32_t lo, uint32_t n,
                                              uint32_t e) {
    uint32_t hi = n;  // invariant: pref[lo] <= e, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pref[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// Event ranges of one wavefront: the block's events [0, E) are cut into one
// contiguous range per wavefront (a multiple of 64), so each wavefront streams
// its own stretch of the synapse arrays and follows the runs with a cursor.
struct WaveRange {
    uint32_t begin, end;
};

__device__ __forceinline__ WaveRange wave_range(uint32_t E) {
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t per = ((E + nw * 64u - 1u) / (nw * 64u)) * 64u;
    WaveRange w;
    w.begin = min(E, wave * per);
    w.end = min(E, w.begin + per);
    return w;
}

// Part p of P of the items [0, E): equal shares, in order.
__device__ __forceinline__ void part_slice(uint32_t E, uint32_t p, uint32_t P, uint32_t& lo,
                                           uint32_t& hi) {
    lo = (uint32_t)(((uint64_t)E * p) / P);
    hi = (uint32_t)(((uint64_t)E * (p + 1u)) / P);
}

// Boundary p of P of the positions [lo, hi), inner boundaries rounded up to a
// multiple of 4 (non-decreasing in p; boundary 0 is lo and boundary P is hi).
__device__ __forceinline__ uint32_t part_bound4(uint32_t lo, uint32_t hi, uint32_t p, uint32_t P) {
    if (p == 0) return lo;
    if (p >= P) return hi;
    const uint32_t x = lo + (uint32_t)(((uint64_t)(hi - lo) * p) / P);
    return min(hi, (x + 3u) & ~3u);
}

// wave_range over the items [lo, hi).
__device__ __forceinline__ WaveRange wave_range_in(uint32_t lo, uint32_t hi) {
    WaveRange w = wave_range(hi - lo);
    w.begin += lo;
    w.end += lo;
    return w;
}

// Run of event e for a lane, starting from the wavefront's cursor r (the run
// of the slice base): the common case is one comparison.
__device__ __forceinline__ uint32_t lane_run(const uint32_t* pref, uint32_t r, uint32_t nr,
                                             uint32_t e) {
    if (r + 1 < nr && pref[r + 1] <= e) return upper_run(pref, r + 1, nr, e);
    return r;
}


}  // namespace dpsnn
