// Network construction on the device (Sec. 2, "Initial construction of the
// connectivity infrastructure"; "Distributed generation of reproducible
// connections").  The paper builds, per process, a database of incoming
// synapses split into sets by delay, with two all-to-all exchanges; on one
// GPU the same structure is a local counting sort:
//   1. k_count_rows: one wavefront per source neuron draws its M synapses and
//      counts them per delay (segment lengths) and per excitatory target
//      (in-degrees of the reverse index);
//   2. k_col_scan / scan_u32: prefix sums give segment and reverse-row offsets;
//   3. k_fill_rows: the same draws, ranked stably by delay with wave ballots,
//      are written to their forward positions and reverse slots;
//   4. k_sort_rows / k_sort_long_rows: each reverse row sorted by (source
//      slot, source neuron, delay, forward position), so a source column's
//      entries in a row are one contiguous run;
//   5. k_fwd_rev: for each excitatory forward position, its source slot and
//      reverse entry (consolidation walks the forward order with it).
#include "net.h"

namespace dpsnn {

namespace {

// Mask of the active lanes whose delay equals x, from the five delay-bit
// ballots (delays are below 32).
__device__ __forceinline__ unsigned long long same_delay(unsigned long long act,
                                                         const unsigned long long bb[5],
                                                         uint32_t x) {
    unsigned long long m = act;
#pragma unroll
    for (int b = 0; b < 5; ++b) m &= ((x >> b) & 1u) ? bb[b] : ~bb[b];
    return m;
}

__global__ __launch_bounds__(256) void k_count_rows(Dims d, const uint32_t* __restrict__ colmap,
                                                    uint64_t* __restrict__ seg_off,
                                                    uint32_t* __restrict__ indeg) {
    const uint32_t row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= d.N) return;  // uniform per wavefront
    const uint32_t lane = lane_id();
    const uint32_t c = row / d.Ncol;
    const uint32_t l = row - c * d.Ncol;
    uint32_t cnt = 0;  // lane L counts synapses of delay L + 1
    for (uint32_t base = 0; base < d.M; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < d.M;
        Syn s{0, 0, 0, false};
        if (valid) s = draw_synapse(d, colmap, row, j);
        const unsigned long long act = __ballot(valid);
        unsigned long long bb[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) bb[b] = __ballot(valid && ((s.delay >> b) & 1u));
        cnt += (uint32_t)__popcll(same_delay(act, bb, lane + 1));
        if (valid && s.exc) {
            const uint32_t kg = colmap[c * kSlots + s.slot] * d.Ncol + s.lt;
            atomicAdd(&indeg[kg], 1u);
        }
    }
    if (lane < d.Dmax) seg_off[(size_t)c * d.segs + lane * d.Ncol + l] = cnt;
}

// Per column: exclusive prefix over its (delay, neuron) segment lengths plus
// the column's base position c * Ncol * M (64-bit; a column's own offsets fit
// 32 bits).
__global__ __launch_bounds__(1024) void k_col_scan(Dims d, uint64_t* __restrict__ seg_off) {
    __shared__ uint32_t sh[20];
    const uint32_t c = blockIdx.x;
    uint64_t* p = seg_off + (size_t)c * d.segs;
    const uint64_t base = (uint64_t)c * d.Ncol * d.M;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < d.segs; b0 += blockDim.x) {
        const uint32_t idx = b0 + threadIdx.x;
        const uint32_t v = idx < d.segs ? (uint32_t)p[idx] : 0u;
        uint32_t tot;
        const uint32_t ex = block_scan(v, sh, tot);
        if (idx < d.segs) p[idx] = base + carry + ex;
        carry += tot;
    }
    if (c == d.C - 1 && threadIdx.x == 0) seg_off[(size_t)d.C * d.segs] = (uint64_t)d.N * d.M;
}

template <typename TgtT>
__global__ __launch_bounds__(256) void k_fill_rows(Dims d, const uint32_t* __restrict__ colmap,
                                                   const uint64_t* __restrict__ seg_off,
                                                   TgtT* __restrict__ tgt, float* __restrict__ w,
                                                   const uint64_t* __restrict__ rowptr,
                                                   uint32_t* __restrict__ cursor,
                                                   uint32_t* __restrict__ rev_srcd,
                                                   uint32_t* __restrict__ rev_fwd) {
    const uint32_t row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= d.N) return;
    const uint32_t lane = lane_id();
    const uint32_t c = row / d.Ncol;
    const uint32_t l = row - c * d.Ncol;
    const uint64_t cbase = (uint64_t)c * d.Ncol * d.M;
    uint32_t placed = 0;  // lane L: synapses of delay L + 1 already placed
    for (uint32_t base = 0; base < d.M; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < d.M;
        Syn s{0, 0, 1, false};
        if (valid) s = draw_synapse(d, colmap, row, j);
        const unsigned long long act = __ballot(valid);
        unsigned long long bb[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) bb[b] = __ballot(valid && ((s.delay >> b) & 1u));
        const unsigned long long mine = same_delay(act, bb, s.delay);
        const uint32_t rank = (uint32_t)__popcll(mine & lanemask_lt());
        const uint32_t before = __shfl(placed, (int)(s.delay - 1u), 64);
        if (valid) {
            const uint64_t pos =
                seg_off[(size_t)c * d.segs + (s.delay - 1u) * d.Ncol + l] + before + rank;
            tgt[pos] = (TgtT)(s.slot * d.Ncol + s.lt);
            w[pos] = s.exc ? d.w_exc : d.w_inh;
            if (s.exc) {
                const uint32_t kg = colmap[c * kSlots + s.slot] * d.Ncol + s.lt;
                const uint64_t x = rowptr[kg] + atomicAdd(&cursor[kg], 1u);
                rev_srcd[x] = (s.slot << 22) | (l << 6) | s.delay;
                rev_fwd[x] = (uint32_t)(pos - cbase);
            }
        }
        placed += (uint32_t)__popcll(same_delay(act, bb, lane + 1));
    }
}

// Reverse rows sorted by the 64-bit key rev_srcd << 32 | rev_fwd (distinct
// within a row).  The fill above claims row slots with atomics, so without
// this the order inside a row depends on timing; sorted, the entries that
// one source column sends to a row form one contiguous run (slot-major key).
// No result depends on the order: rows longer than kSortLong stay as filled.
constexpr uint32_t kSortShort = 1024;  // one wavefront per row, in LDS
constexpr uint32_t kSortLong = 8192;   // one 1024-thread workgroup per row

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic network over sk[0 .. P) (P a power of two), `lanes` threads from
// `tid`, synchronised by `sync` after every stage.
template <typename Sync>
__device__ __forceinline__ void bitonic(unsigned long long* sk, uint32_t P, uint32_t tid,
                                        uint32_t lanes, Sync sync) {
    for (uint32_t k = 2u; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0u; j >>= 1) {
            for (uint32_t x = tid; x < P; x += lanes) {
                const uint32_t y = x ^ j;
                if (y > x) {
                    const unsigned long long a = sk[x], b = sk[y];
                    if ((a > b) == ((x & k) == 0u)) {
                        sk[x] = b;
                        sk[y] = a;
                    }
                }
            }
            sync();
        }
    }
}

// Rows of 2 .. kSortShort entries: four rows per 256-thread workgroup, one
// wavefront each.
__global__ __launch_bounds__(256) void k_sort_rows(Dims d, const uint64_t* __restrict__ rowptr,
                                                   uint32_t* __restrict__ rev_srcd,
                                                   uint32_t* __restrict__ rev_fwd) {
    __shared__ unsigned long long sk_all[4][kSortShort];
    const uint32_t row = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (row >= d.N) return;
    const uint64_t x0 = rowptr[row];
    const uint64_t len = rowptr[row + 1] - x0;
    if (len < 2u || len > kSortShort) return;
    const uint32_t n = (uint32_t)len;
    unsigned long long* sk = sk_all[threadIdx.x >> 6];
    const uint32_t lane = lane_id();
    uint32_t P = 2u;
    while (P < n) P <<= 1;
    for (uint32_t x = lane; x < P; x += 64u)
        sk[x] = x < n ? ((unsigned long long)rev_srcd[x0 + x] << 32 | rev_fwd[x0 + x]) : ~0ull;
    wave_fence();
    bitonic(sk, P, lane, 64u, wave_fence);
    for (uint32_t x = lane; x < n; x += 64u) {
        const unsigned long long k = sk[x];
        rev_srcd[x0 + x] = (uint32_t)(k >> 32);
        rev_fwd[x0 + x] = (uint32_t)k;
    }
}

// Rows of kSortShort + 1 .. kSortLong entries: a 1024-thread workgroup per
// row, the workgroups striding over all rows (the length test is uniform
// across a workgroup, so every thread reaches every barrier).
__global__ __launch_bounds__(1024) void k_sort_long_rows(Dims d, const uint64_t* __restrict__ rowptr,
                                                         uint32_t* __restrict__ rev_srcd,
                                                         uint32_t* __restrict__ rev_fwd) {
    __shared__ unsigned long long sk[kSortLong];
    for (uint32_t row = blockIdx.x; row < d.N; row += gridDim.x) {
        const uint64_t x0 = rowptr[row];
        const uint64_t len = rowptr[row + 1] - x0;
        if (len <= kSortShort || len > kSortLong) continue;
        const uint32_t n = (uint32_t)len;
        uint32_t P = 2u;
        while (P < n) P <<= 1;
        for (uint32_t x = threadIdx.x; x < P; x += blockDim.x)
            sk[x] = x < n ? ((unsigned long long)rev_srcd[x0 + x] << 32 | rev_fwd[x0 + x]) : ~0ull;
        __syncthreads();
        bitonic(sk, P, threadIdx.x, blockDim.x, [] { __syncthreads(); });
        for (uint32_t x = threadIdx.x; x < n; x += blockDim.x) {
            const unsigned long long k = sk[x];
            rev_srcd[x0 + x] = (uint32_t)(k >> 32);
            rev_fwd[x0 + x] = (uint32_t)k;
        }
        __syncthreads();  // sk is reused by the next row
    }
}

// fwd_rev[f] = slot << 28 | (x - rowptr[ct * Ncol]) for the reverse entry x
// (target column ct) of excitatory forward position f; positions of
// inhibitory synapses keep 0xFFFFFFFF (slot 15) from the fill before.
// Workgroups (target column, stripe); stripes walk the column's rows.
__global__ __launch_bounds__(256) void k_fwd_rev(Dims d, const uint32_t* __restrict__ srcmap,
                                                 const uint64_t* __restrict__ rowptr,
                                                 const uint32_t* __restrict__ rev_srcd,
                                                 const uint32_t* __restrict__ rev_fwd,
                                                 uint32_t* __restrict__ fwd_rev) {
    const uint32_t ct = blockIdx.x;
    const uint64_t x0 = rowptr[(size_t)ct * d.Ncol];
    const uint64_t x1 = rowptr[(size_t)(ct + 1) * d.Ncol];
    const uint64_t colsz = (uint64_t)d.Ncol * d.M;
    for (uint64_t x = x0 + (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; x < x1;
         x += (uint64_t)gridDim.y * blockDim.x) {
        const uint32_t slot = rev_srcd[x] >> 22;
        const uint64_t f = (uint64_t)srcmap[ct * kSlots + slot] * colsz + rev_fwd[x];
        fwd_rev[f] = slot << 28 | (uint32_t)(x - x0);
    }
}

__global__ void k_init_state(Dims d, float* __restrict__ v, float* __restrict__ u,
                             uint2* __restrict__ hist,
                             int32_t* __restrict__ t_last) {
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d.N) return;
    const uint32_t l = k % d.Ncol;
    const float b = 0.2f, c = -65.0f;
    (void)l;
    v[k] = c;
    u[k] = b * c;
    hist[k] = make_uint2(0u, (uint32_t)kNoSpike);
    t_last[k] = kNoSpike;
}

// Device-wide exclusive scan of 32-bit values into OutT (32- or 64-bit):
// tiles of blockDim elements (a tile's sum must fit 32 bits), then the tile
// offsets in OutT.
template <typename OutT>
__global__ __launch_bounds__(1024) void k_scan_tiles(const uint32_t* __restrict__ in,
                                                     OutT* __restrict__ out,
                                                     OutT* __restrict__ sums, uint32_t n) {
    __shared__ uint32_t sh[20];
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t v = idx < n ? in[idx] : 0u;
    uint32_t tot;
    const uint32_t ex = block_scan(v, sh, tot);
    if (idx < n) out[idx] = ex;
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// out[c] = rowptr[c * Ncol] for c = 0 .. C: where each target column's
// reverse rows start.
__global__ __launch_bounds__(256) void k_col_starts(Dims d, const uint64_t* __restrict__ rowptr,
                                                    uint64_t* __restrict__ out) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c <= d.C) out[c] = rowptr[(size_t)c * d.Ncol];
}

// Exclusive block scan of 64-bit values (same scheme as block_scan).
__device__ __forceinline__ uint64_t block_scan_u64(uint64_t v, uint64_t* sh, uint64_t& total) {
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= (uint32_t)o) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    if (wid == 0) {
        const uint64_t s = lane < nw ? sh[lane] : 0ull;
        uint64_t inc = s;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, 64);
            if (lane >= (uint32_t)o) inc += y;
        }
        if (lane < nw) sh[lane] = inc - s;
        if (lane == nw - 1) sh[nw] = inc;
    }
    __syncthreads();
    const uint64_t res = sh[wid] + x - v;
    total = sh[nw];
    __syncthreads();
    return res;
}

template <typename OutT>
__global__ __launch_bounds__(1024) void k_scan_sums(OutT* __restrict__ sums, uint32_t nb,
                                                    OutT* __restrict__ out, uint32_t n) {
    __shared__ uint64_t sh[20];
    uint64_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        const uint32_t idx = b0 + threadIdx.x;
        const uint64_t v = idx < nb ? (uint64_t)sums[idx] : 0ull;
        uint64_t tot;
        const uint64_t ex = block_scan_u64(v, sh, tot);
        if (idx < nb) sums[idx] = (OutT)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = (OutT)carry;
}

template <typename OutT>
__global__ __launch_bounds__(1024) void k_scan_add(OutT* __restrict__ out,
                                                   const OutT* __restrict__ sums, uint32_t n) {
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) out[idx] += sums[blockIdx.x];
}

template <typename OutT>
hipError_t scan_into(Net& n, hipStream_t stream, const uint32_t* in, OutT* out, uint32_t count) {
    const uint32_t bs = 1024;
    const uint32_t nb = (count + bs - 1) / bs;
    if (nb == 0) {
        return hipMemsetAsync(out, 0, sizeof(OutT), stream);
    }
    OutT* sums = (OutT*)n.scan_tmp;
    hipLaunchKernelGGL(k_scan_tiles<OutT>, dim3(nb), dim3(bs), 0, stream, in, out, sums, count);
    hipLaunchKernelGGL(k_scan_sums<OutT>, dim3(1), dim3(bs), 0, stream, sums, nb, out, count);
    hipLaunchKernelGGL(k_scan_add<OutT>, dim3(nb), dim3(bs), 0, stream, out, sums, count);
    return hipGetLastError();
}

}  // namespace

// out[0..count) = exclusive prefix of in, out[count] = total, on `stream`.
hipError_t scan_u32(Net& n, hipStream_t stream, const uint32_t* in, uint32_t* out, uint32_t count) {
    return scan_into<uint32_t>(n, stream, in, out, count);
}

hipError_t scan_u32_u64(Net& n, hipStream_t stream, const uint32_t* in, uint64_t* out, uint32_t count) {
    return scan_into<uint64_t>(n, stream, in, out, count);
}

hipError_t launch_build(Net& n) {
    const Dims& d = n.d;
    hipError_t e;
    const uint32_t rows_per_block = 4;  // 256 threads, one wavefront per row
    const uint32_t gb = (d.N + rows_per_block - 1) / rows_per_block;
    if ((e = hipMemsetAsync(n.cursor, 0, sizeof(uint32_t) * d.N, n.stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_count_rows, dim3(gb), dim3(256), 0, n.stream, d, n.colmap, n.seg_off,
                       n.cursor);
    hipLaunchKernelGGL(k_col_scan, dim3(d.C), dim3(1024), 0, n.stream, d, n.seg_off);
    if ((e = scan_u32_u64(n, n.stream, n.cursor, n.rowptr, d.N)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(n.cursor, 0, sizeof(uint32_t) * d.N, n.stream)) != hipSuccess) return e;
    // every entry is written below; zeroing keeps stray reads in bounds if not
    if ((e = hipMemsetAsync(n.tgt, 0, (n.tgt16 ? 2 : 4) * (size_t)n.S, n.stream)) != hipSuccess) return e;
    if (n.S_exc) {
        if ((e = hipMemsetAsync(n.rev_srcd, 0, 4 * (size_t)n.S_exc, n.stream)) != hipSuccess) return e;
        if ((e = hipMemsetAsync(n.rev_fwd, 0, 4 * (size_t)n.S_exc, n.stream)) != hipSuccess) return e;
    }
    if (n.tgt16) {
        hipLaunchKernelGGL(k_fill_rows<uint16_t>, dim3(gb), dim3(256), 0, n.stream, d, n.colmap,
                           n.seg_off, (uint16_t*)n.tgt, n.w, n.rowptr, n.cursor, n.rev_srcd,
                           n.rev_fwd);
    } else {
        hipLaunchKernelGGL(k_fill_rows<uint32_t>, dim3(gb), dim3(256), 0, n.stream, d, n.colmap,
                           n.seg_off, (uint32_t*)n.tgt, n.w, n.rowptr, n.cursor, n.rev_srcd,
                           n.rev_fwd);
    }
    if (n.S_exc) {
        hipLaunchKernelGGL(k_sort_rows, dim3((d.N + 3) / 4), dim3(256), 0, n.stream, d, n.rowptr,
                           n.rev_srcd, n.rev_fwd);
        // rows above kSortShort entries need in-degrees near M or above
        if (d.M > kSortShort / 2)
            hipLaunchKernelGGL(k_sort_long_rows, dim3(std::min<uint32_t>(d.N, 2048u)), dim3(1024), 0,
                               n.stream, d, n.rowptr, n.rev_srcd, n.rev_fwd);
    }
    if (n.fwd_rev) {
        if ((e = hipMemsetAsync(n.fwd_rev, 0xFF, 4 * (size_t)n.S, n.stream)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_fwd_rev, dim3(d.C, 64), dim3(256), 0, n.stream, d, n.srcmap, n.rowptr,
                           n.rev_srcd, n.rev_fwd, n.fwd_rev);
    }
    hipLaunchKernelGGL(k_init_state, dim3((d.N + 255) / 256), dim3(256), 0, n.stream, d, n.v, n.u,
                       n.hist, n.t_last);
    hipLaunchKernelGGL(k_col_starts, dim3((d.C + 1 + 255) / 256), dim3(256), 0, n.stream, d,
                       n.rowptr, n.col_rev_dev);
    return hipGetLastError();
}

}  // namespace dpsnn
