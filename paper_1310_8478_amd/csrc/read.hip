// Read-back in canonical synapse order (id * M + j), independent of the
// device layout: each source row is redrawn and ranked exactly as the build
// placed it, which locates every synapse's forward position.
#include "net.h"

#include <algorithm>

namespace dpsnn {

namespace {

__device__ __forceinline__ unsigned long long same_delay_r(unsigned long long act,
                                                           const unsigned long long bb[5],
                                                           uint32_t x) {
    unsigned long long m = act;
#pragma unroll
    for (int b = 0; b < 5; ++b) m &= ((x >> b) & 1u) ? bb[b] : ~bb[b];
    return m;
}

// Rows [i0, i1); only canonical synapses g in [g_lo, g_hi) are written, at
// g - g_lo.  Pg holds P of whole source columns in the forward layout, its
// first entry being forward position pg_base (the excitatory positions of
// the rows' columns are all present; inhibitory synapses have P = 0).
template <typename TgtT>
__global__ __launch_bounds__(256) void k_read_rows(Dims d, const uint32_t* __restrict__ colmap,
                                                   const uint64_t* __restrict__ seg_off,
                                                   const TgtT* __restrict__ tgt,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ Dacc,
                                                   const float* __restrict__ Pg, uint64_t pg_base,
                                                   uint32_t i0, uint32_t i1, uint64_t g_lo,
                                                   uint64_t g_hi, uint32_t* __restrict__ o_tgt,
                                                   uint8_t* __restrict__ o_dly,
                                                   float* __restrict__ o_w, float* __restrict__ o_P,
                                                   float* __restrict__ o_D) {
    const uint32_t row = i0 + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= i1) return;
    const uint32_t lane = lane_id();
    const uint32_t c = row / d.Ncol;
    const uint32_t l = row - c * d.Ncol;
    uint32_t placed = 0;
    for (uint32_t base = 0; base < d.M; base += 64) {
        const uint32_t j = base + lane;
        const bool valid = j < d.M;
        Syn s{0, 0, 1, false};
        if (valid) s = draw_synapse(d, colmap, row, j);
        const unsigned long long act = __ballot(valid);
        unsigned long long bb[5];
#pragma unroll
        for (int b = 0; b < 5; ++b) bb[b] = __ballot(valid && ((s.delay >> b) & 1u));
        const unsigned long long mine = same_delay_r(act, bb, s.delay);
        const uint32_t rank = (uint32_t)__popcll(mine & lanemask_lt());
        const uint32_t before = __shfl(placed, (int)(s.delay - 1u), 64);
        const uint64_t g = (uint64_t)row * d.M + j;
        if (valid && g >= g_lo && g < g_hi) {
            const uint64_t pos =
                seg_off[(size_t)c * d.segs + (s.delay - 1u) * d.Ncol + l] + before + rank;
            const size_t o = (size_t)(g - g_lo);
            const uint32_t wi = (uint32_t)tgt[pos];
            const uint32_t sl = wi / d.Ncol;
            if (o_tgt) o_tgt[o] = colmap[c * kSlots + sl] * d.Ncol + (wi - sl * d.Ncol);
            if (o_dly) o_dly[o] = (uint8_t)s.delay;
            if (o_w) o_w[o] = w[pos];
            if (o_D) o_D[o] = Dacc[pos];
            if (o_P) o_P[o] = s.exc ? Pg[pos - pg_base] : 0.0f;
        }
        placed += (uint32_t)__popcll(same_delay_r(act, bb, lane + 1));
    }
}

// P between the reverse order and the forward layout, for the source columns
// [c0, c1) only.  Pg holds those columns' forward blocks back to back (entry
// (c - c0) * Ncol * M + offset in the block).  Workgroups (target column ct,
// slice y): a reverse entry's source column is the column that reaches ct
// through the entry's slot, its forward offset in that column's block is
// rev_fwd; target columns that no column of the range reaches return at once.
template <bool TO_FWD>
__global__ __launch_bounds__(256) void k_move_P(Dims d, const uint32_t* __restrict__ srcmap,
                                                const uint64_t* __restrict__ rowptr,
                                                const uint32_t* __restrict__ rev_srcd,
                                                const uint32_t* __restrict__ rev_fwd,
                                                float* __restrict__ P, float* __restrict__ Pg,
                                                uint32_t c0, uint32_t c1) {
    __shared__ uint32_t smap[kSlots];
    const uint32_t ct = blockIdx.x;
    if (threadIdx.x < kSlots) smap[threadIdx.x] = srcmap[ct * kSlots + threadIdx.x];
    __syncthreads();
    const uint32_t span = c1 - c0;
    bool reached = false;
#pragma unroll
    for (int q = 0; q < kSlots; ++q) reached |= smap[q] - c0 < span;
    if (!reached) return;  // workgroup-uniform
    const uint64_t colsz = (uint64_t)d.Ncol * d.M;
    const uint64_t x0 = rowptr[(size_t)ct * d.Ncol], x1 = rowptr[(size_t)(ct + 1) * d.Ncol];
    const uint64_t stride = (uint64_t)gridDim.y * blockDim.x;
    for (uint64_t x = x0 + (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; x < x1; x += stride) {
        const uint32_t rel = smap[rev_srcd[x] >> 22] - c0;
        if (rel >= span) continue;
        float* pf = Pg + (uint64_t)rel * colsz + rev_fwd[x];
        if (TO_FWD) *pf = P[x];
        else P[x] = *pf;
    }
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) p[x] = 0.0f;
}

}  // namespace

hipError_t launch_P_to_forward(Net& n, float* Pg, uint32_t c0, uint32_t c1, bool zero_first) {
    if (c1 <= c0) return hipSuccess;
    if (zero_first) {
        const uint64_t cnt = (uint64_t)(c1 - c0) * n.d.Ncol * n.d.M;
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((cnt + 255) / 256, 4096);
        hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, n.stream, Pg, cnt);
    }
    if (n.S_exc == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_move_P<true>, dim3(n.d.C, 16), dim3(256), 0, n.stream, n.d, n.srcmap,
                       n.rowptr, n.rev_srcd, n.rev_fwd, n.Pacc, Pg, c0, c1);
    return hipGetLastError();
}

hipError_t launch_P_from_forward(Net& n, float* Pg, uint32_t c0, uint32_t c1) {
    if (c1 <= c0 || n.S_exc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_move_P<false>, dim3(n.d.C, 16), dim3(256), 0, n.stream, n.d, n.srcmap,
                       n.rowptr, n.rev_srcd, n.rev_fwd, n.Pacc, Pg, c0, c1);
    return hipGetLastError();
}

// Canonical synapses [g_lo, g_hi) of rows [i0, i1) into device outputs at
// g - g_lo.  Pg: P of whole source columns in the forward layout starting at
// forward position pg_base (from launch_P_to_forward), or null.
hipError_t launch_read_rows(Net& n, uint32_t i0, uint32_t i1, uint64_t g_lo, uint64_t g_hi,
                            const float* Pg, uint64_t pg_base, uint32_t* tgt_out,
                            uint8_t* dly_out, float* w_out, float* P_out, float* D_out) {
    const uint32_t rows = i1 - i0;
    if (rows == 0) return hipSuccess;
    const uint32_t gb = (rows + 3) / 4;
    if (n.tgt16) {
        hipLaunchKernelGGL(k_read_rows<uint16_t>, dim3(gb), dim3(256), 0, n.stream, n.d, n.colmap,
                           n.seg_off, (const uint16_t*)n.tgt, n.w, n.Dacc, Pg, pg_base, i0, i1,
                           g_lo, g_hi, tgt_out, dly_out, w_out, P_out, D_out);
    } else {
        hipLaunchKernelGGL(k_read_rows<uint32_t>, dim3(gb), dim3(256), 0, n.stream, n.d, n.colmap,
                           n.seg_off, (const uint32_t*)n.tgt, n.w, n.Dacc, Pg, pg_base, i0, i1,
                           g_lo, g_hi, tgt_out, dly_out, w_out, P_out, D_out);
    }
    return hipGetLastError();
}

}  // namespace dpsnn
