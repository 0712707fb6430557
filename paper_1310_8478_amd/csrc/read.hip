// Read-back in canonical synapse order (id * M + j), independent of the
// device layout: each source row is redrawn and ranked exactly as the build
// placed it, which locates every synapse's forward position.
#include "net.h"

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

template <typename TgtT>
__global__ __launch_bounds__(256) void k_read_rows(Dims d, const uint32_t* __restrict__ colmap,
                                                   const uint64_t* __restrict__ seg_off,
                                                   const TgtT* __restrict__ tgt,
                                                   const float* __restrict__ w,
                                                   const float* __restrict__ Dacc,
                                                   const float* __restrict__ Pf, uint32_t i0,
                                                   uint32_t i1, uint32_t* __restrict__ o_tgt,
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
        if (valid) {
            const uint64_t pos =
                seg_off[(size_t)c * d.segs + (s.delay - 1u) * d.Ncol + l] + before + rank;
            const size_t o = (size_t)(row - i0) * d.M + j;
            const uint32_t wi = (uint32_t)tgt[pos];
            const uint32_t sl = wi / d.Ncol;
            if (o_tgt) o_tgt[o] = colmap[c * kSlots + sl] * d.Ncol + (wi - sl * d.Ncol);
            if (o_dly) o_dly[o] = (uint8_t)s.delay;
            if (o_w) o_w[o] = w[pos];
            if (o_D) o_D[o] = Dacc[pos];
            if (o_P) o_P[o] = Pf[pos];
        }
        placed += (uint32_t)__popcll(same_delay_r(act, bb, lane + 1));
    }
}

// P from reverse to forward order.  Workgroups (target column ct, slice y):
// an entry's source column is the column that reaches ct through the entry's
// slot, and its forward position is that column's block start plus rev_fwd.
__global__ __launch_bounds__(256) void k_scatter_P(Dims d, const uint32_t* __restrict__ srcmap,
                                                   const uint64_t* __restrict__ rowptr,
                                                   const uint32_t* __restrict__ rev_srcd,
                                                   const uint32_t* __restrict__ rev_fwd,
                                                   const float* __restrict__ P,
                                                   float* __restrict__ Pf) {
    const uint32_t ct = blockIdx.x;
    const uint64_t x0 = rowptr[(size_t)ct * d.Ncol], x1 = rowptr[(size_t)(ct + 1) * d.Ncol];
    const uint64_t stride = (uint64_t)gridDim.y * blockDim.x;
    for (uint64_t x = x0 + (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; x < x1; x += stride) {
        const uint32_t src = srcmap[ct * kSlots + (rev_srcd[x] >> 22)];
        Pf[(uint64_t)src * d.Ncol * d.M + rev_fwd[x]] = P[x];
    }
}

// The inverse: P[x] = Pf[forward position of x].
__global__ __launch_bounds__(256) void k_gather_P(Dims d, const uint32_t* __restrict__ srcmap,
                                                  const uint64_t* __restrict__ rowptr,
                                                  const uint32_t* __restrict__ rev_srcd,
                                                  const uint32_t* __restrict__ rev_fwd,
                                                  const float* __restrict__ Pf,
                                                  float* __restrict__ P) {
    const uint32_t ct = blockIdx.x;
    const uint64_t x0 = rowptr[(size_t)ct * d.Ncol], x1 = rowptr[(size_t)(ct + 1) * d.Ncol];
    const uint64_t stride = (uint64_t)gridDim.y * blockDim.x;
    for (uint64_t x = x0 + (uint64_t)blockIdx.y * blockDim.x + threadIdx.x; x < x1; x += stride) {
        const uint32_t src = srcmap[ct * kSlots + (rev_srcd[x] >> 22)];
        P[x] = Pf[(uint64_t)src * d.Ncol * d.M + rev_fwd[x]];
    }
}

}  // namespace

hipError_t launch_gather_P(Net& n, const float* Pf) {
    if (n.S_exc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_P, dim3(n.d.C, 16), dim3(256), 0, n.stream, n.d, n.srcmap,
                       n.rowptr, n.rev_srcd, n.rev_fwd, Pf, n.Pacc);
    return hipGetLastError();
}

hipError_t launch_scatter_P(Net& n, float* Pf) {
    hipError_t e = hipMemsetAsync(Pf, 0, sizeof(float) * n.S, n.stream);
    if (e != hipSuccess) return e;
    if (n.S_exc == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_P, dim3(n.d.C, 16), dim3(256), 0, n.stream, n.d, n.srcmap,
                       n.rowptr, n.rev_srcd, n.rev_fwd, n.Pacc, Pf);
    return hipGetLastError();
}

// Rows [i0, i1) (canonical synapses i0*M .. i1*M) into device outputs laid out
// (row - i0) * M + j.  Pf: P in forward layout (from launch_scatter_P) or null.
hipError_t launch_read_rows(Net& n, uint32_t i0, uint32_t i1, float* Pf, uint32_t* tgt_out,
                            uint8_t* dly_out, float* w_out, float* P_out, float* D_out) {
    const uint32_t rows = i1 - i0;
    if (rows == 0) return hipSuccess;
    const uint32_t gb = (rows + 3) / 4;
    if (n.tgt16) {
        hipLaunchKernelGGL(k_read_rows<uint16_t>, dim3(gb), dim3(256), 0, n.stream, n.d, n.colmap,
                           n.seg_off, (const uint16_t*)n.tgt, n.w, n.Dacc, Pf, i0, i1, tgt_out,
                           dly_out, w_out, P_out, D_out);
    } else {
        hipLaunchKernelGGL(k_read_rows<uint32_t>, dim3(gb), dim3(256), 0, n.stream, n.d, n.colmap,
                           n.seg_off, (const uint32_t*)n.tgt, n.w, n.Dacc, Pf, i0, i1, tgt_out,
                           dly_out, w_out, P_out, D_out);
    }
    return hipGetLastError();
}

}  // namespace dpsnn
