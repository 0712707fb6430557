// C ABI of libdpsnn: configuration checks, device memory, the build and step
// sequencing, and read-back.  Every device computation runs in the HIP
// kernels of build.hip, step.hip and read.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "net.h"

using namespace dpsnn;

namespace dpsnn {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

}  // namespace dpsnn

namespace {

#define DPSNN_HIP(expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(DPSNN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Derived {
    uint32_t N, C, Ncol, Ne, M, Dmax, W, R, M_own;
    uint64_t S, S_exc;
    bool tgt16;
    bool fwd_rev;  // consolidation's forward-to-reverse map is kept
};

bool finite_in(float x, float lo, float hi) { return std::isfinite(x) && x >= lo && x <= hi; }

int validate(const dpsnn_config* c, Derived* o) {
    if (!c) return fail(DPSNN_E_INVAL, "config is NULL");
    if (c->grid_x < 1 || c->grid_y < 1 || c->grid_x > 65535 || c->grid_y > 65535)
        return fail(DPSNN_E_INVAL, "grid_x and grid_y must be in 1..65535");
    if (c->neurons_per_column < 2 || c->neurons_per_column > 65535)
        return fail(DPSNN_E_INVAL, "neurons_per_column must be in 2..65535");
    if (!finite_in(c->exc_fraction, 0.0f, 1.0f)) return fail(DPSNN_E_INVAL, "exc_fraction must be in [0, 1]");
    const uint32_t Ncol = c->neurons_per_column;
    const uint32_t Ne = (uint32_t)std::floor((double)c->exc_fraction * (double)Ncol + 0.5);
    if (Ne < 1 || Ne > Ncol) return fail(DPSNN_E_INVAL, "a column needs at least one excitatory neuron");
    if (c->synapses_per_neuron < 1 || c->synapses_per_neuron > 65535)
        return fail(DPSNN_E_INVAL, "synapses_per_neuron must be in 1..65535");
    if (c->max_delay < 1 || c->max_delay > 31) return fail(DPSNN_E_INVAL, "max_delay must be in 1..31");
    if (c->conn_mode > 1u) return fail(DPSNN_E_INVAL, "conn_mode must be 0 or 1");
    if (c->conn_mode == 0u && !finite_in(c->own_fraction, 0.0f, 1.0f))
        return fail(DPSNN_E_INVAL, "own_fraction must be in [0, 1]");
    const uint64_t C = (uint64_t)c->grid_x * c->grid_y;
    const uint64_t N = C * Ncol;
    if (N >= (1ull << 26)) return fail(DPSNN_E_INVAL, "at most 2^26 - 1 neurons per network");
    const uint64_t S = N * c->synapses_per_neuron;
    if (S >= (1ull << 36)) return fail(DPSNN_E_INVAL, "at most 2^36 - 1 synapses per network");
    // kernels address one column's forward block and reverse rows with 32-bit
    // offsets: a column's block and the synapses that can reach it (from 13
    // columns) stay below 2^31
    if ((uint64_t)kSlots * Ncol * c->synapses_per_neuron >= (1ull << 31))
        return fail(DPSNN_E_INVAL, "13 x neurons_per_column x synapses_per_neuron must stay below 2^31");
    if (c->sum_mode == DPSNN_SUM_ORDERED && S >= (1ull << 32))
        return fail(DPSNN_E_INVAL, "ORDERED summation takes at most 2^32 - 1 synapses");
    if (!finite_in(c->w_exc_init, -1000.f, 1000.f) || !finite_in(c->w_inh, -1000.f, 1000.f) ||
        !finite_in(c->w_max, 0.f, 1000.f))
        return fail(DPSNN_E_INVAL, "weights must be finite, |w| <= 1000, w_max >= 0");
    if (!finite_in(c->a_plus, 0.f, 1000.f) || !finite_in(c->a_minus, 0.f, 1000.f))
        return fail(DPSNN_E_INVAL, "STDP amplitudes must be finite and >= 0");
    if (!finite_in(c->tau_plus, 1e-3f, 1000.f) || !finite_in(c->tau_minus, 1e-3f, 1000.f))
        return fail(DPSNN_E_INVAL, "STDP time constants must be in [1e-3, 1000] ms");
    if (!finite_in(c->wu_bias, -1000.f, 1000.f) || !finite_in(c->sd_decay, -1000.f, 1000.f))
        return fail(DPSNN_E_INVAL, "consolidation constants must be finite");
    if (!(std::isfinite(c->thalamic_rate) && c->thalamic_rate >= 0.f && c->thalamic_rate < 1024.f))
        return fail(DPSNN_E_INVAL, "thalamic_rate must be in [0, 1024)");
    if (!finite_in(c->thalamic_current, -1000.f, 1000.f))
        return fail(DPSNN_E_INVAL, "thalamic_current must be finite, |x| <= 1000");
    if (c->sum_mode > 2u) return fail(DPSNN_E_INVAL, "sum_mode must be 0, 1 or 2");
    uint32_t R = c->raster_steps ? c->raster_steps : 1024u;
    if (R < c->max_delay + 1u) return fail(DPSNN_E_INVAL, "raster_steps must be at least max_delay + 1");
    if (R > (1u << 20)) return fail(DPSNN_E_INVAL, "raster_steps must be at most 2^20");
    o->N = (uint32_t)N;
    o->C = (uint32_t)C;
    o->Ncol = Ncol;
    o->Ne = Ne;
    o->M = c->synapses_per_neuron;
    o->Dmax = c->max_delay;
    o->W = (Ncol + 63) / 64;
    o->R = R;
    o->M_own = (uint32_t)std::floor((double)c->own_fraction * (double)o->M + 0.5);
    if (o->M_own > o->M) o->M_own = o->M;
    o->S = S;
    o->S_exc = (uint64_t)C * Ne * o->M;
    o->tgt16 = (uint64_t)kSlots * Ncol <= 65536ull;
    // the map packs a reverse offset inside the target column (below
    // 13 * Ncol * M) into 28 bits next to the 4-bit slot
    o->fwd_rev = o->S_exc > 0 && (uint64_t)kSlots * Ncol * o->M <= (1ull << 28);
    return DPSNN_OK;
}

// Byte sizes of every device array, in allocation order.
std::vector<size_t> array_bytes(const dpsnn_config* c, const Derived& d) {
    // per-synapse arrays are padded to whole 4-element quads: the kernels read
    // aligned quads that may extend past the last synapse
    const size_t N = d.N, S = (d.S + 3) & ~(size_t)3, Se = (d.S_exc + 3) & ~(size_t)3;
    std::vector<size_t> b = {
        sizeof(uint32_t) * d.C * kSlots,                  // colmap
        sizeof(uint32_t) * d.C * kSlots,                  // srcmap
        sizeof(uint64_t) * ((size_t)d.C * d.Dmax * d.Ncol + 1),  // seg_off
        (d.tgt16 ? 2 : 4) * S,                            // tgt
        sizeof(float) * S,                                // w
        sizeof(float) * S,                                // D
        sizeof(uint64_t) * (N + 1),                       // rowptr
        sizeof(uint32_t) * N,                             // cursor
        sizeof(uint32_t) * Se,                            // rev_srcd
        sizeof(uint32_t) * Se,                            // rev_fwd
        sizeof(float) * Se,                               // P
        sizeof(float) * N, sizeof(float) * N,             // v, u
        (c->sum_mode == DPSNN_SUM_FIXED ? 8 : 4) * N,     // acc
        sizeof(uint2) * N, sizeof(int32_t) * N,           // hist (with t_old), t_last
        sizeof(uint64_t) * (size_t)d.R * d.C * d.W,       // ring
        sizeof(DevStats) * 64,                            // stats
        sizeof(uint64_t) * (N / 1024 + 2),                // scan_tmp
        sizeof(uint64_t) * ((size_t)d.C + 1),             // column starts of the reverse rows
    };
    if (d.fwd_rev) b.push_back(sizeof(uint32_t) * S);     // fwd_rev
    if (c->sum_mode == DPSNN_SUM_ORDERED) {
        b.push_back(sizeof(uint32_t) * N);                // ev_cnt
        b.push_back(sizeof(uint32_t) * (N + 1));          // ev_start
        b.push_back(sizeof(unsigned long long) * S);      // ev_key
        b.push_back(sizeof(float) * S);                   // ev_w
    }
    return b;
}

void* dalloc(Net& n, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    void* p = nullptr;
    if (n.dev.alloc) {
        p = n.dev.alloc(bytes, n.dev.stream, n.dev.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p) n.allocs.push_back({p, bytes});
    return p;
}

void dfree(Net& n, void* p, size_t bytes) {
    if (!p) return;
    if (n.dev.free) n.dev.free(p, bytes, n.dev.stream, n.dev.ctx);
    else (void)hipFree(p);
}

void release(Net* n) {
    if (!n) return;
    (void)hipSetDevice(n->dev.device);
    (void)hipStreamSynchronize(n->stream);
    release_launch_set_host(n->solo);
    for (auto& a : n->allocs) dfree(*n, a.p, a.bytes);
    n->allocs.clear();
    n->timers.release();
    delete n;
}

// STDP amplitudes A exp(-dt / tau) for dt = 0, 1, ...: evaluated in fp64,
// rounded once to fp32, values below FLT_MIN flushed to 0; the table ends
// where the amplitude becomes 0 (it decreases monotonically).
std::vector<float> amplitude_table(float A, float tau) {
    std::vector<float> out;
    for (uint32_t k = 0; k < (1u << 20); ++k) {
        const double x = (double)A * std::exp(-(double)k / (double)tau);
        float f = (float)x;
        if (std::fabs(f) < FLT_MIN) f = 0.0f;
        if (f == 0.0f) break;
        out.push_back(f);
    }
    return out;
}

// Largest-remainder split of M synapses over own column and the 12 neighbour
// slots with shares 7600/300x4/200x4/100x4 per 10000 (ties to the lower slot).
void paper_split(uint32_t M, uint32_t end[kSlots]) {
    static const uint32_t share[kSlots] = {7600, 300, 300, 300, 300, 200, 200, 200, 200,
                                           100, 100, 100, 100};
    uint32_t cnt[kSlots];
    uint64_t rem[kSlots];
    uint32_t total = 0;
    for (int s = 0; s < kSlots; ++s) {
        const uint64_t p = (uint64_t)share[s] * M;
        cnt[s] = (uint32_t)(p / 10000);
        rem[s] = p % 10000;
        total += cnt[s];
    }
    while (total < M) {
        int best = 0;
        for (int s = 1; s < kSlots; ++s)
            if (rem[s] > rem[best]) best = s;
        cnt[best]++;
        rem[best] = 0;
        total++;
    }
    uint32_t acc = 0;
    for (int s = 0; s < kSlots; ++s) {
        acc += cnt[s];
        end[s] = acc;
    }
}

const int kRingDx[12] = {1, -1, 0, 0, 1, -1, 1, -1, 2, -2, 0, 0};
const int kRingDy[12] = {0, 0, 1, -1, 1, 1, -1, -1, 0, 0, 2, -2};

int wrapi(int x, int n) {
    const int r = x % n;
    return r < 0 ? r + n : r;
}

template <typename T>
int upload(Net& n, T* dst, const std::vector<T>& src) {
    if (src.empty()) return DPSNN_OK;
    DPSNN_HIP(hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, n.stream));
    return DPSNN_OK;
}

}  // namespace

namespace dpsnn {

void destroy_net(Net* n) { release(n); }

// Device allocation through a dpsnn_device (callbacks or hipMalloc), recorded
// in `track` so that its owner frees it.
void* dev_alloc(const dpsnn_device& dev, hipStream_t stream, size_t bytes,
                std::vector<Net::Alloc>* track) {
    bytes = std::max<size_t>(bytes, 256);
    void* p = nullptr;
    if (dev.alloc) {
        p = dev.alloc(bytes, stream, dev.ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        p = nullptr;
    }
    if (p && track) track->push_back({p, bytes});
    return p;
}

void release_launch_set_host(LaunchSet& L) {
    if (L.graph) {
        (void)hipGraphExecDestroy(L.graph);
        L.graph = nullptr;
    }
    if (L.cap_stream) {
        (void)hipStreamDestroy(L.cap_stream);
        L.cap_stream = nullptr;
    }
    if (L.ev_copied) {
        if (L.copy_pending) (void)hipEventSynchronize(L.ev_copied);
        (void)hipEventDestroy(L.ev_copied);
        L.ev_copied = nullptr;
    }
    if (L.ev_host) {
        (void)hipHostFree(L.ev_host);
        L.ev_host = nullptr;
    }
    L.copy_pending = false;
}

void free_tracked(const dpsnn_device& dev, hipStream_t stream, std::vector<Net::Alloc>& allocs) {
    for (auto& a : allocs) {
        if (dev.free) dev.free(a.p, a.bytes, stream, dev.ctx);
        else (void)hipFree(a.p);
    }
    allocs.clear();
}

// Descriptor tables and block maps of a launch over `cnt` networks.  The host
// copies stay in L, so with sync == false the uploads may still be in flight
// on `stream` when this returns (L must then outlive them).
int make_launch_set(LaunchSet& L, Net* const* m, uint32_t cnt, const dpsnn_device& dev,
                    hipStream_t stream, std::vector<Net::Alloc>* track, bool sync) {
    L.K = cnt;
    L.max_ncol = 0;
    L.max_w = 0;
    L.min_col_syn = ~0ull;
    L.sum_mode = m[0]->cfg.sum_mode;
    L.tgt16 = m[0]->tgt16;
    std::vector<uint2>& col = L.host_col;
    std::vector<uint2>& neu = L.host_neu;
    col.clear();
    neu.clear();
    L.bmap_wu.assign(cnt, nullptr);
    L.n_wu.assign(cnt, 0);
    std::vector<std::vector<uint2>>& wu = L.host_wu;
    wu.assign(cnt, {});
    const uint64_t wchunk = 256ull * kWupdateItems;
    for (uint32_t k = 0; k < cnt; ++k) {
        const Dims& d = m[k]->d;
        L.max_ncol = std::max(L.max_ncol, d.Ncol);
        L.max_w = std::max(L.max_w, d.W);
        L.min_col_syn = std::min<uint64_t>(L.min_col_syn, (uint64_t)d.Ncol * d.M);
        for (uint32_t c = 0; c < d.C; ++c) col.push_back(make_uint2(k, c));
        for (uint32_t w0 = 0; w0 < d.C * d.W; w0 += 4) neu.push_back(make_uint2(k, w0));
        // consolidation: (target column, chunk of its reverse rows)
        const std::vector<uint64_t>& cr = m[k]->col_rev;
        if (cr.size() != (size_t)d.C + 1) return fail(DPSNN_E_INVAL, "network has no reverse index");
        for (uint32_t c = 0; c < d.C; ++c) {
            const uint64_t nch = (cr[c + 1] - cr[c] + wchunk - 1) / wchunk;
            for (uint64_t q = 0; q < nch; ++q) wu[k].push_back(make_uint2(c, (uint32_t)q));
        }
        if (wu[k].size() > 0x7FFFFFFFull) return fail(DPSNN_E_INVAL, "too many consolidation chunks");
    }
    // heaviest columns first (synapses per column), so that the longest
    // workgroups start early; stable, so a single network keeps its order
    if (cnt > 1) {
        std::stable_sort(col.begin(), col.end(), [&](const uint2& a, const uint2& b) {
            const uint64_t wa = (uint64_t)m[a.x]->d.Ncol * m[a.x]->d.M;
            const uint64_t wb = (uint64_t)m[b.x]->d.Ncol * m[b.x]->d.M;
            return wa > wb;
        });
    }
    // one network: workgroup i runs on XCD i mod 8 (round-robin dispatch), and
    // each XCD has its own L2.  XCD x gets the x-th eighth of the columns in
    // row-major order, walked column by column, so that the columns in flight
    // on one XCD form a compact block whose reachable neighbourhoods overlap
    // in its L2 (a few per cent faster on grids of 1024 columns and more)
    if (cnt == 1 && col.size() >= 64) {
        const uint32_t C = (uint32_t)col.size(), gx = m[0]->d.GX;
        std::vector<std::vector<uint32_t>> part(kXcds);
        for (uint32_t x = 0; x < kXcds; ++x) {
            const uint32_t a = (uint32_t)((uint64_t)C * x / kXcds);
            const uint32_t b = (uint32_t)((uint64_t)C * (x + 1) / kXcds);
            for (uint32_t c = a; c < b; ++c) part[x].push_back(c);
            std::stable_sort(part[x].begin(), part[x].end(), [&](uint32_t p, uint32_t q) {
                return p % gx != q % gx ? p % gx < q % gx : p / gx < q / gx;
            });
        }
        col.clear();
        size_t pos[kXcds] = {};
        for (size_t i = 0; col.size() < C; ++i) {
            const uint32_t x = (uint32_t)(i % kXcds);
            if (pos[x] < part[x].size()) col.push_back(make_uint2(0u, part[x][pos[x]++]));
        }
    }
    L.n_col = (uint32_t)col.size();
    L.n_neu = (uint32_t)neu.size();
    {
        double neurons = 0.0, est = 0.0;
        for (uint32_t k = 0; k < cnt; ++k) {
            neurons += (double)m[k]->d.N;
            est += m[k]->per_col * (double)m[k]->d.C;
        }
        L.avg_nwin = L.n_col ? (double)kSlots * neurons / (double)L.n_col : 0.0;
        L.per_col = L.n_col ? est / (double)L.n_col : 0.0;  // carried over from earlier sets
        L.sparse = L.per_col < L.avg_nwin;
        L.steps = L.copy_steps = L.base_steps = L.base_count = 0;
        L.copy_pending = false;
    }
    L.ev_count = (unsigned long long*)dev_alloc(dev, stream, sizeof(unsigned long long), track);
    if (!L.ev_count) return fail(DPSNN_E_NOMEM, "launch tables");
    DPSNN_HIP(hipMemsetAsync(L.ev_count, 0, sizeof(unsigned long long), stream));
    if (!L.ev_host) {
        void* hp = nullptr;
        if (hipHostMalloc(&hp, 2 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess)
            return fail(DPSNN_E_NOMEM, "pinned regime counter");
        L.ev_host = (unsigned long long*)hp;
    }
    if (!L.ev_copied) DPSNN_HIP(hipEventCreateWithFlags(&L.ev_copied, hipEventDisableTiming));
    L.descs = (NetDesc*)dev_alloc(dev, stream, sizeof(NetDesc) * cnt, track);
    L.bmap_col = (uint2*)dev_alloc(dev, stream, sizeof(uint2) * col.size(), track);
    L.bmap_neu = (uint2*)dev_alloc(dev, stream, sizeof(uint2) * neu.size(), track);
    if (!L.descs || !L.bmap_col || !L.bmap_neu) return fail(DPSNN_E_NOMEM, "launch tables");
    DPSNN_HIP(hipMemcpyAsync(L.bmap_col, col.data(), sizeof(uint2) * col.size(), hipMemcpyHostToDevice, stream));
    DPSNN_HIP(hipMemcpyAsync(L.bmap_neu, neu.data(), sizeof(uint2) * neu.size(), hipMemcpyHostToDevice, stream));
    for (uint32_t k = 0; k < cnt; ++k) {
        L.n_wu[k] = (uint32_t)wu[k].size();
        if (!L.n_wu[k]) continue;
        L.bmap_wu[k] = (uint2*)dev_alloc(dev, stream, sizeof(uint2) * wu[k].size(), track);
        if (!L.bmap_wu[k]) return fail(DPSNN_E_NOMEM, "launch tables");
        DPSNN_HIP(hipMemcpyAsync(L.bmap_wu[k], wu[k].data(), sizeof(uint2) * wu[k].size(),
                                 hipMemcpyHostToDevice, stream));
    }
    L.host_descs.resize(cnt);
    L.max_probes = 0;
    for (uint32_t k = 0; k < cnt; ++k) {
        L.host_descs[k] = m[k]->make_desc();
        L.max_probes = std::max(L.max_probes, m[k]->probe_n);
    }
    DPSNN_HIP(hipMemcpyAsync(L.descs, L.host_descs.data(), sizeof(NetDesc) * cnt, hipMemcpyHostToDevice, stream));
    if (sync) DPSNN_HIP(hipStreamSynchronize(stream));
    return DPSNN_OK;
}

}  // namespace dpsnn

namespace {

int refresh_descs(LaunchSet& L, Net* const* m, hipStream_t stream) {
    L.max_probes = 0;
    for (uint32_t k = 0; k < L.K; ++k) {
        L.host_descs[k] = m[k]->make_desc();
        L.max_probes = std::max(L.max_probes, m[k]->probe_n);
    }
    DPSNN_HIP(hipMemcpyAsync(L.descs, L.host_descs.data(), sizeof(NetDesc) * L.K, hipMemcpyHostToDevice, stream));
    DPSNN_HIP(hipStreamSynchronize(stream));
    return DPSNN_OK;
}

int apply_tuning(Tuning& tn, uint32_t key, uint32_t value) {
    switch (key) {
        case 0:
            if (value && value != 256 && value != 512 && value != 1024)
                return fail(DPSNN_E_INVAL, "delivery block must be 0 (automatic), 256, 512 or 1024");
            tn.deliver_block = value;
            return DPSNN_OK;
        case 1:
            if (value && value != 256 && value != 512 && value != 1024)
                return fail(DPSNN_E_INVAL, "LTP block must be 0 (automatic), 256, 512 or 1024");
            tn.ltp_block = value;
            return DPSNN_OK;
        case 2:
            if (value > 3) return fail(DPSNN_E_INVAL, "window must be 0 (off), 1 (all columns), 2 (own column) or 3 (automatic)");
            tn.window = value;
            return DPSNN_OK;
        case 3:
            if (value != 1 && value != 2 && value != 4 && value != 8)
                return fail(DPSNN_E_INVAL, "unroll must be 1, 2, 4 or 8");
            tn.unroll = value;
            return DPSNN_OK;
        case 4:
            if (value > 2) return fail(DPSNN_E_INVAL, "age window must be 0 (off), 1 (on) or 2 (automatic)");
            tn.age = value;
            return DPSNN_OK;
        case 5:
            if (value > 1024) return fail(DPSNN_E_INVAL, "column parts must be 0 (automatic) to 1024");
            tn.parts = value;
            return DPSNN_OK;
        case 6:
            if (value > 2) return fail(DPSNN_E_INVAL, "LTP staging must be 0 (off), 1 (on) or 2 (automatic)");
            tn.ltp_stage = value;
            return DPSNN_OK;
        case 7:
            tn.fuse = value;
            return DPSNN_OK;
        case 8:
            if (value > 1024) return fail(DPSNN_E_INVAL, "graph steps must be 0 (off) to 1024");
            tn.graph = value;
            return DPSNN_OK;
        case 9:
            if (value < 1 || value > 13) return fail(DPSNN_E_INVAL, "window split must be 1 to 13");
            tn.split = value;
            return DPSNN_OK;
        case 10:
            if (value > 13) return fail(DPSNN_E_INVAL, "partial window slots must be 0 (automatic) to 13");
            tn.own_slots = value;
            return DPSNN_OK;
        case 11:
            if (value > 2) return fail(DPSNN_E_INVAL, "sparse LTP must be 0 (off), 1 (on) or 2 (automatic)");
            tn.sparse_ltp = value;
            return DPSNN_OK;
        case 12:
            if (value > 2) return fail(DPSNN_E_INVAL, "sparse delivery must be 0 (off), 1 (on) or 2 (automatic)");
            tn.sparse_deliver = value;
            return DPSNN_OK;
        case 13:
            if (value > 8) return fail(DPSNN_E_INVAL, "columns per sparse LTP workgroup must be 0 (automatic) to 8");
            tn.ltp_cols = value;
            return DPSNN_OK;
        case 14:
            if (value > 1) return fail(DPSNN_E_INVAL, "consolidation must be 0 (two passes) or 1 (forward pass)");
            tn.consolidate = value;
            return DPSNN_OK;
        default:
            return fail(DPSNN_E_INVAL, "unknown tuning key");
    }
}

// Online autotuner: each candidate shape runs `steps` steps (two interleaved
// rounds).  With LTP and delivery fused (the default) a candidate is one
// workgroup size for both plus the delivery unroll, ranked by their combined
// time; with fusion off the fastest delivery shape and the fastest LTP
// workgroup size are kept separately.
int autotune(LaunchSet& L, Tuning& tn, Timers& tm, hipStream_t stream, Net* const* m, uint32_t steps) {
    if (steps == 0) return fail(DPSNN_E_INVAL, "steps_per_trial must be positive");
    struct Cand { uint32_t block, unroll; };
    const Cand dcand[] = {{256, 4}, {512, 4}, {1024, 4}, {256, 8}, {512, 8}, {1024, 8}};
    const uint32_t lcand[] = {256, 512, 1024};
    const size_t nd = sizeof(dcand) / sizeof(dcand[0]);
    const bool joint = tn.fuse != 0;
    std::vector<double> dms(nd, 0.0), lms(3, 0.0);
    std::vector<uint64_t> dn(nd, 0), ln(3, 0);
    Timers probe;
    probe.on = true;
    const Tuning base = tn;
    for (int round = 0; round < 2; ++round) {
        for (size_t c = 0; c < nd; ++c) {
            Tuning trial = base;
            trial.deliver_block = dcand[c].block;
            trial.unroll = dcand[c].unroll;
            trial.ltp_block = joint ? dcand[c].block : lcand[c % 3];
            for (uint32_t s = 0; s < steps; ++s) {
                hipError_t e = launch_step_set(L, trial, probe, stream, m);
                if (e != hipSuccess) { probe.release(); return fail(DPSNN_E_DEVICE, hipGetErrorString(e)); }
            }
            if (hipStreamSynchronize(stream) != hipSuccess) { probe.release(); return fail(DPSNN_E_DEVICE, "sync"); }
            double before[4] = {probe.ms[0], probe.ms[1], probe.ms[2], probe.ms[3]};
            uint64_t nbefore[4] = {probe.n[0], probe.n[1], probe.n[2], probe.n[3]};
            probe.collect();
            if (joint) {  // one step = LTP (if launched apart) + delivery
                dms[c] += (probe.ms[0] - before[0]) + (probe.ms[1] - before[1]);
                dn[c] += probe.n[1] - nbefore[1];
            } else {
                dms[c] += probe.ms[1] - before[1];
                dn[c] += probe.n[1] - nbefore[1];
                lms[c % 3] += probe.ms[0] - before[0];
                ln[c % 3] += probe.n[0] - nbefore[0];
            }
        }
    }
    probe.release();
    size_t bd = 0, bl = 0;
    for (size_t c = 1; c < nd; ++c)
        if (dn[c] && (!dn[bd] || dms[c] / dn[c] < dms[bd] / dn[bd])) bd = c;
    if (dn[bd]) { tn.deliver_block = dcand[bd].block; tn.unroll = dcand[bd].unroll; }
    if (joint) {
        if (dn[bd]) tn.ltp_block = dcand[bd].block;
    } else {
        for (size_t c = 1; c < 3; ++c)
            if (ln[c] && (!ln[bl] || lms[c] / ln[c] < lms[bl] / ln[bl])) bl = c;
        if (ln[bl]) tn.ltp_block = lcand[bl];
    }
    (void)tm;
    return DPSNN_OK;
}

}  // namespace

NetDesc Net::make_desc() const {
    NetDesc nd;
    std::memset(&nd, 0, sizeof(nd));
    nd.d = d;
    nd.t0 = t;
    nd.colmap = colmap; nd.srcmap = srcmap; nd.seg_off = seg_off; nd.tgt = tgt;
    nd.w = w; nd.Dacc = Dacc; nd.rowptr = rowptr; nd.rev_srcd = rev_srcd; nd.rev_fwd = rev_fwd;
    nd.fwd_rev = fwd_rev;
    nd.Pacc = Pacc; nd.v = v; nd.u = u; nd.acc = acc; nd.hist = hist;
    nd.t_last = t_last; nd.ring = ring; nd.tp = tp; nd.tm = tm; nd.tp_len = tp_len;
    nd.tm_len = tm_len; nd.stats = stats; nd.thal_whole = thal_whole; nd.thal_thr = thal_thr;
    nd.thal_mv = cfg.thalamic_current; nd.stim_t = stim_t; nd.stim_id = stim_id;
    nd.stim_mv = stim_mv; nd.stim_n = (uint32_t)stim_n;
    nd.weight_update_period = cfg.weight_update_period; nd.wu_bias = cfg.wu_bias;
    nd.sd_decay = cfg.sd_decay; nd.w_max = cfg.w_max; nd.S_exc = S_exc;
    nd.ev_cnt = ev_cnt; nd.ev_start = ev_start; nd.ev_key = ev_key; nd.ev_w = ev_w;
    nd.cursor = cursor;
    nd.probe_id = probe_id; nd.probe_buf = probe_buf; nd.probe_n = probe_n;
    return nd;
}

struct dpsnn_batch {
    std::vector<Net*> members;
    hipStream_t stream = nullptr;
    dpsnn_device dev;
    LaunchSet L;
    Tuning tune;
    Timers timers;
    std::vector<Net::Alloc> allocs;
};

// ---- checkpoints -------------------------------------------------------
// A checkpoint holds the configuration and the dynamic state; the
// connectivity is regenerated from the seed when it is loaded.  Layout: the
// header, then the arrays of ckpt_parts in order, each padded to 16 bytes.
// P is stored in the forward layout, which the configuration fixes: the
// order inside a reverse row is a property of the build (rows of more than
// 8192 entries keep the order of its atomics).
namespace {

constexpr char kCkptMagic[8] = {'D', 'P', 'S', 'N', 'N', 'C', 'K', '1'};
constexpr uint32_t kCkptVersion = 1;

struct CkptHeader {
    char magic[8];
    uint32_t version, header_bytes;
    dpsnn_config cfg;
    uint64_t t, consolidations, stim_n, total_bytes;
};

struct CkptPart {
    void* dev;
    size_t bytes;
};

size_t pad16(size_t x) { return (x + 15) & ~(size_t)15; }

// Byte sizes of the checkpoint arrays, in file order; the raster ring is
// entry kCkptRing.
constexpr uint32_t kMaxProbes = 1u << 16;  // state probes of one network
constexpr size_t kCkptRing = 4;
constexpr size_t kCkptP = 8;   // P, stored in the forward layout

std::vector<size_t> ckpt_sizes(uint64_t N, uint64_t C, uint64_t W, uint64_t R, uint64_t S,
                               uint64_t stim_n) {
    return {4 * N, 4 * N, sizeof(uint2) * N, 4 * N, sizeof(uint64_t) * R * C * W,
            sizeof(DevStats) * 64, 4 * S, 4 * S, 4 * S, 4 * stim_n, 4 * stim_n, 4 * stim_n};
}

std::vector<CkptPart> ckpt_parts(const Net& n, uint64_t stim_n) {
    const std::vector<size_t> b = ckpt_sizes(n.d.N, n.d.C, n.d.W, n.d.R, n.S, stim_n);
    void* const dev[] = {n.v, n.u, n.hist, n.t_last, n.ring, n.stats, n.w, n.Dacc,
                         nullptr,  // P in the forward layout (through a buffer)
                         n.stim_t, n.stim_id, n.stim_mv};
    std::vector<CkptPart> parts(b.size());
    for (size_t k = 0; k < b.size(); ++k) parts[k] = {dev[k], b[k]};
    return parts;
}

uint64_t ckpt_total(const std::vector<size_t>& sizes) {
    uint64_t tot = pad16(sizeof(CkptHeader));
    for (size_t b : sizes) tot += pad16(b);
    return tot;
}

uint64_t ckpt_total(const std::vector<CkptPart>& parts) {
    uint64_t tot = pad16(sizeof(CkptHeader));
    for (const CkptPart& q : parts) tot += pad16(q.bytes);
    return tot;
}

// The raster words of a checkpoint hold no spike beyond a column's last
// neuron (delivery decodes source neurons from these bits).
bool ckpt_raster_in_range(const unsigned char* buf, const std::vector<size_t>& sizes,
                          const Derived& d) {
    if (d.Ncol % 64u == 0u) return true;
    const uint64_t keep = (1ull << (d.Ncol % 64u)) - 1ull;
    size_t off = pad16(sizeof(CkptHeader));
    for (size_t k = 0; k < kCkptRing; ++k) off += pad16(sizes[k]);
    for (uint64_t rc = 0; rc < (uint64_t)d.R * d.C; ++rc) {
        uint64_t word;
        std::memcpy(&word, buf + off + ((rc + 1) * d.W - 1) * sizeof(uint64_t), sizeof(word));
        if (word & ~keep) return false;
    }
    return true;
}

// Device scratch of a read-back: P of whole source columns in the forward
// layout (groups of columns, so a read of a few rows touches one column), and
// staging for the requested outputs.  Bounded independently of the network
// size; allocated through the network's allocator (callbacks or hipMalloc)
// for the call and freed before it returns.
constexpr size_t kReadPBytes = 32ull << 20;      // P of at least one whole column
constexpr size_t kReadStageBytes = 8ull << 20;   // staging, at least one row

size_t pad256(size_t x) { return (x + 255) & ~(size_t)255; }

struct ReadPlan {
    uint32_t i0 = 0, i1 = 0, cA = 0, cB = 0;
    uint32_t group = 1;        // source columns per P group
    uint32_t stage_rows = 1;   // rows per staging chunk
    size_t per_syn = 0;        // staged bytes per synapse
    size_t pg_bytes = 0, stage_bytes = 0;
    size_t bytes() const { return pg_bytes + stage_bytes; }
};

size_t stage_bytes_for(uint32_t rows, uint32_t M, bool tgt, bool dly, bool w, bool P, bool D) {
    const size_t m = (size_t)rows * M;
    return (tgt ? pad256(4 * m) : 0) + (dly ? pad256(m) : 0) + (w ? pad256(4 * m) : 0) +
           (P ? pad256(4 * m) : 0) + (D ? pad256(4 * m) : 0);
}

// The scratch layout of a read of canonical synapses [first, first + count)
// within `limit` bytes; false if not even one column and one row fit.
bool plan_read(const Net& n, uint64_t first, uint64_t count, bool tgt, bool dly, bool w,
                      bool P, bool D, size_t p_budget, size_t stage_budget, size_t limit,
                      ReadPlan& pl) {
    const uint32_t M = n.d.M, Ncol = n.d.Ncol;
    const uint64_t colb = 4ull * Ncol * M;
    pl.i0 = (uint32_t)(first / M);
    pl.i1 = (uint32_t)((first + count + M - 1) / M);
    pl.cA = pl.i0 / Ncol;
    pl.cB = (pl.i1 - 1) / Ncol + 1;
    pl.per_syn = (tgt ? 4 : 0) + (dly ? 1 : 0) + (w ? 4 : 0) + (P ? 4 : 0) + (D ? 4 : 0);
    const uint32_t rows = pl.i1 - pl.i0;
    pl.stage_rows = (uint32_t)std::max<uint64_t>(
        1, std::min<uint64_t>(rows, stage_budget / std::max<size_t>(1, (size_t)M * pl.per_syn)));
    pl.group = P ? (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(pl.cB - pl.cA, p_budget / colb))
                 : pl.cB - pl.cA;
    for (;;) {
        pl.pg_bytes = P ? pad256((size_t)pl.group * colb) : 0;
        pl.stage_bytes = stage_bytes_for(pl.stage_rows, M, tgt, dly, w, P, D);
        if (pl.bytes() <= limit) return true;
        if (P && pl.group > 1) pl.group = (pl.group + 1) / 2;
        else if (pl.stage_rows > 1) pl.stage_rows = (pl.stage_rows + 1) / 2;
        else return false;
    }
}

// Scratch bytes a read of the whole network may take (counted in the
// footprint, so that reads of a served job stay inside its reservation).
uint64_t read_reserve_bytes(uint64_t C, uint64_t Ncol, uint64_t M) {
    const uint64_t colb = 4ull * Ncol * M;
    const uint64_t group = std::max<uint64_t>(1, std::min<uint64_t>(C, kReadPBytes / colb));
    const uint64_t rows = std::max<uint64_t>(1, std::min<uint64_t>(C * Ncol, kReadStageBytes / (17ull * M)));
    return pad256(group * colb) + 4 * pad256(4 * rows * M) + pad256(rows * M);
}

// Save and load move P between the reverse order and the forward layout in
// groups of whole source columns through a transient device buffer from the
// network's allocator: all columns at once if kCkptPBytes allows, else the
// largest group the allocator grants, halving down to one column.
constexpr uint64_t kCkptPBytes = 1ull << 30;

struct PGroups {
    Net* n = nullptr;
    float* buf = nullptr;
    size_t bytes = 0;
    uint32_t group = 0;   // source columns per group
    ~PGroups() {
        if (buf) {
            (void)hipStreamSynchronize(n->stream);
            dfree(*n, buf, bytes);
        }
    }
};

bool alloc_pgroups(Net* n, PGroups& g) {
    g.n = n;
    const uint64_t colb = 4ull * n->d.Ncol * n->d.M;
    uint64_t want = std::max<uint64_t>(1, std::min<uint64_t>(n->d.C, kCkptPBytes / colb));
    for (;;) {
        g.bytes = std::max<size_t>((size_t)(want * colb), 256);
        g.buf = static_cast<float*>(dev_alloc(n->dev, n->stream, g.bytes, nullptr));
        if (g.buf) {
            g.group = (uint32_t)want;
            return true;
        }
        if (want == 1) return false;
        want = (want + 1) / 2;
    }
}

}  // namespace

extern "C" {

const char* dpsnn_last_error(void) { return g_err.c_str(); }

int dpsnn_default_config(dpsnn_config* c) {
    if (!c) return fail(DPSNN_E_INVAL, "config is NULL");
    std::memset(c, 0, sizeof(*c));
    c->grid_x = 2;
    c->grid_y = 2;
    c->neurons_per_column = 1250;
    c->exc_fraction = 0.8f;
    c->synapses_per_neuron = 100;
    c->conn_mode = DPSNN_CONN_CONFIG;
    c->own_fraction = 0.5f;
    c->max_delay = 20;
    c->w_exc_init = 6.0f;
    c->w_inh = -5.0f;
    c->w_max = 10.0f;
    c->a_plus = 0.1f;
    c->a_minus = 0.12f;
    c->tau_plus = 20.0f;
    c->tau_minus = 20.0f;
    c->weight_update_period = 1000;
    c->wu_bias = 0.01f;
    c->sd_decay = 0.9f;
    c->thalamic_rate = 1.0f;
    c->thalamic_current = 20.0f;
    c->seed = 1310;
    c->sum_mode = DPSNN_SUM_FIXED;
    c->raster_steps = 0;
    return DPSNN_OK;
}

int dpsnn_footprint_bytes(const dpsnn_config* cfg, uint64_t* bytes) {
    Derived d;
    int rc = validate(cfg, &d);
    if (rc) return rc;
    if (!bytes) return fail(DPSNN_E_INVAL, "bytes is NULL");
    uint64_t tot = 0;
    for (size_t b : array_bytes(cfg, d)) tot += std::max<size_t>(b, 256);
    // STDP amplitude tables, as long as the build makes them
    tot += std::max<size_t>(4 * std::max<size_t>(amplitude_table(cfg->a_plus, cfg->tau_plus).size(), 1), 256);
    tot += std::max<size_t>(4 * std::max<size_t>(amplitude_table(cfg->a_minus, cfg->tau_minus).size(), 1), 256);
    // the network's own launch tables: event counter, descriptor, block maps
    // of columns and raster words, consolidation chunks (at most one per
    // 256 * kWupdateItems reverse entries of a column, plus one per column)
    const uint64_t wu_chunks = d.S_exc / (256ull * kWupdateItems) + d.C;
    tot += 256 + std::max<uint64_t>(sizeof(NetDesc), 256) + std::max<uint64_t>(8ull * d.C, 256) +
           std::max<uint64_t>(8ull * ((d.C * d.W + 3) / 4), 256) + std::max<uint64_t>(8ull * wu_chunks, 256);
    // the scratch of a read-back (dpsnn_read_weights, dpsnn_read_connectivity)
    tot += read_reserve_bytes(d.C, d.Ncol, d.M);
    *bytes = tot;
    return DPSNN_OK;
}

int dpsnn_build_network(const dpsnn_config* cfg, const dpsnn_device* dev, dpsnn_net** out) {
    if (!out) return fail(DPSNN_E_INVAL, "out is NULL");
    *out = nullptr;
    Derived dv;
    int rc = validate(cfg, &dv);
    if (rc) return rc;
    if (!dev) return fail(DPSNN_E_INVAL, "device is NULL");
    if ((dev->alloc == nullptr) != (dev->free == nullptr))
        return fail(DPSNN_E_INVAL, "alloc and free callbacks must be given together");
    int ndev = 0;
    DPSNN_HIP(hipGetDeviceCount(&ndev));
    if (dev->device < 0 || dev->device >= ndev) return fail(DPSNN_E_INVAL, "no such HIP device");
    DPSNN_HIP(hipSetDevice(dev->device));

    Net* n = new Net();
    n->cfg = *cfg;
    if (n->cfg.raster_steps == 0) n->cfg.raster_steps = dv.R;
    n->dev = *dev;
    n->stream = (hipStream_t)dev->stream;
    n->S = dv.S;
    n->S_exc = dv.S_exc;
    n->tgt16 = dv.tgt16;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev->device) == hipSuccess &&
        lds > 0)
        n->tune.max_lds = (size_t)lds;

    Dims& d = n->d;
    std::memset(&d, 0, sizeof(d));
    d.N = dv.N; d.C = dv.C; d.Ncol = dv.Ncol; d.Ne = dv.Ne; d.M = dv.M; d.Dmax = dv.Dmax;
    d.GX = cfg->grid_x; d.GY = cfg->grid_y; d.W = dv.W; d.R = dv.R;
    d.conn_mode = cfg->conn_mode; d.M_own = dv.M_own;
    paper_split(dv.M, d.paper_end);
    d.key0 = (uint32_t)(cfg->seed & 0xFFFFFFFFu);
    d.key1 = (uint32_t)(cfg->seed >> 32);
    d.w_exc = cfg->w_exc_init; d.w_inh = cfg->w_inh;
    d.segs = dv.Dmax * dv.Ncol;
    d.ncol_magic = (uint32_t)(((1ull << 32) + dv.Ncol - 1) / dv.Ncol);
    const double r = (double)cfg->thalamic_rate;
    const double fl = std::floor(r);
    n->thal_whole = (uint32_t)fl;
    n->thal_thr = (uint32_t)((r - fl) * 4294967296.0);

    const std::vector<size_t> sz = array_bytes(cfg, dv);
    std::vector<void*> p(sz.size(), nullptr);
    for (size_t k = 0; k < sz.size(); ++k) {
        p[k] = dalloc(*n, sz[k]);
        if (!p[k]) {
            release(n);
            return fail(DPSNN_E_NOMEM, "device allocation of " + std::to_string(sz[k]) + " bytes failed");
        }
    }
    size_t k = 0;
    n->colmap = (uint32_t*)p[k++]; n->srcmap = (uint32_t*)p[k++]; n->seg_off = (uint64_t*)p[k++];
    n->tgt = p[k++]; n->w = (float*)p[k++]; n->Dacc = (float*)p[k++];
    n->rowptr = (uint64_t*)p[k++]; n->cursor = (uint32_t*)p[k++];
    n->rev_srcd = (uint32_t*)p[k++]; n->rev_fwd = (uint32_t*)p[k++]; n->Pacc = (float*)p[k++];
    n->v = (float*)p[k++]; n->u = (float*)p[k++]; n->acc = p[k++];
    n->hist = (uint2*)p[k++]; n->t_last = (int32_t*)p[k++];
    n->ring = (uint64_t*)p[k++]; n->stats = (DevStats*)p[k++]; n->scan_tmp = (uint64_t*)p[k++];
    n->col_rev_dev = (uint64_t*)p[k++];
    if (dv.fwd_rev) n->fwd_rev = (uint32_t*)p[k++];
    if (cfg->sum_mode == DPSNN_SUM_ORDERED) {
        n->ev_cnt = (uint32_t*)p[k++]; n->ev_start = (uint32_t*)p[k++];
        n->ev_key = (unsigned long long*)p[k++]; n->ev_w = (float*)p[k++];
    }

    // column maps
    std::vector<uint32_t> colmap((size_t)dv.C * kSlots), srcmap((size_t)dv.C * kSlots);
    for (uint32_t c = 0; c < dv.C; ++c) {
        const int cx = (int)(c % cfg->grid_x), cy = (int)(c / cfg->grid_x);
        colmap[(size_t)c * kSlots] = c;
        srcmap[(size_t)c * kSlots] = c;
        for (int q = 1; q < kSlots; ++q) {
            const int gx = (int)cfg->grid_x, gy = (int)cfg->grid_y;
            colmap[(size_t)c * kSlots + q] =
                (uint32_t)(wrapi(cy + kRingDy[q - 1], gy) * gx + wrapi(cx + kRingDx[q - 1], gx));
            srcmap[(size_t)c * kSlots + q] =
                (uint32_t)(wrapi(cy - kRingDy[q - 1], gy) * gx + wrapi(cx - kRingDx[q - 1], gx));
        }
    }
    std::vector<float> tp = amplitude_table(cfg->a_plus, cfg->tau_plus);
    std::vector<float> tm = amplitude_table(cfg->a_minus, cfg->tau_minus);
    n->tp_len = (uint32_t)tp.size();
    n->tm_len = (uint32_t)tm.size();
    n->tp = (float*)dalloc(*n, sizeof(float) * std::max<size_t>(tp.size(), 1));
    n->tm = (float*)dalloc(*n, sizeof(float) * std::max<size_t>(tm.size(), 1));
    if (!n->tp || !n->tm) {
        release(n);
        return fail(DPSNN_E_NOMEM, "device allocation of STDP tables failed");
    }
#define DPSNN_TRY(expr)             \
    do {                            \
        int rc_ = (expr);           \
        if (rc_) {                  \
            release(n);             \
            return rc_;             \
        }                           \
    } while (0)
#define DPSNN_TRY_HIP(expr)                                                                   \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            release(n);                                                                       \
            return fail(DPSNN_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
        }                                                                                     \
    } while (0)
    DPSNN_TRY(upload(*n, n->colmap, colmap));
    DPSNN_TRY(upload(*n, n->srcmap, srcmap));
    DPSNN_TRY(upload(*n, n->tp, tp));
    DPSNN_TRY(upload(*n, n->tm, tm));
    const size_t accb = (cfg->sum_mode == DPSNN_SUM_FIXED ? 8 : 4) * (size_t)dv.N;
    DPSNN_TRY_HIP(hipMemsetAsync(n->Dacc, 0, sizeof(float) * dv.S, n->stream));
    DPSNN_TRY_HIP(hipMemsetAsync(n->Pacc, 0, sizeof(float) * std::max<uint64_t>(dv.S_exc, 1), n->stream));
    DPSNN_TRY_HIP(hipMemsetAsync(n->acc, 0, accb, n->stream));
    DPSNN_TRY_HIP(hipMemsetAsync(n->ring, 0, sizeof(uint64_t) * (size_t)dv.R * dv.C * dv.W, n->stream));
    DPSNN_TRY_HIP(hipMemsetAsync(n->stats, 0, sizeof(DevStats) * 64, n->stream));
    if (n->ev_cnt) {
        DPSNN_TRY_HIP(hipMemsetAsync(n->ev_cnt, 0, sizeof(uint32_t) * dv.N, n->stream));
        DPSNN_TRY_HIP(hipMemsetAsync(n->ev_start, 0, sizeof(uint32_t) * (dv.N + 1), n->stream));
    }
    DPSNN_TRY_HIP(launch_build(*n));
    // where each target column's reverse rows start (consolidation's work
    // map); the reverse index must hold exactly the excitatory synapses
    n->col_rev.assign((size_t)dv.C + 1, 0);
    DPSNN_TRY_HIP(hipMemcpyAsync(n->col_rev.data(), n->col_rev_dev, sizeof(uint64_t) * ((size_t)dv.C + 1),
                                 hipMemcpyDeviceToHost, n->stream));
    DPSNN_TRY_HIP(hipMemsetAsync(n->cursor, 0, sizeof(uint32_t) * dv.N, n->stream));
    DPSNN_TRY_HIP(hipStreamSynchronize(n->stream));
    if (n->col_rev[dv.C] != dv.S_exc) {
        release(n);
        return fail(DPSNN_E_DEVICE, "reverse index size mismatch after build");
    }
    {
        Net* one[1] = {n};
        DPSNN_TRY(make_launch_set(n->solo, one, 1, n->dev, n->stream, &n->allocs, true));
    }
#undef DPSNN_TRY
#undef DPSNN_TRY_HIP
    *out = reinterpret_cast<dpsnn_net*>(n);
    return DPSNN_OK;
}

int dpsnn_step(dpsnn_net* h, uint32_t n_steps) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    if (n->in_batch) return fail(DPSNN_E_INVAL, "the network belongs to a batch; step the batch");
    if ((uint64_t)n->t + n_steps >= (1ull << 31)) return fail(DPSNN_E_RANGE, "step count overflow");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    if (n->desc_dirty) {
        Net* one[1] = {n};
        int rc = refresh_descs(n->solo, one, n->stream);
        if (rc) return rc;
        n->desc_dirty = false;
    }
    Net* one[1] = {n};
    DPSNN_HIP(launch_steps(n->solo, n->tune, n->timers, n->stream, one, n_steps));
    return DPSNN_OK;
}

int dpsnn_sync(dpsnn_net* h) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    return DPSNN_OK;
}

int dpsnn_time(dpsnn_net* h, uint32_t* t) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n || !t) return fail(DPSNN_E_INVAL, "NULL argument");
    *t = n->t;
    return DPSNN_OK;
}

int dpsnn_read_spikes(dpsnn_net* h, uint32_t t_begin, uint32_t t_end, uint32_t* times,
                      uint32_t* ids, size_t cap, size_t* n_out) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n || !n_out) return fail(DPSNN_E_INVAL, "NULL argument");
    *n_out = 0;
    if (t_end < t_begin) return fail(DPSNN_E_INVAL, "t_end < t_begin");
    if (t_begin < 1) t_begin = 1;
    if (t_end <= t_begin) return DPSNN_OK;
    const uint32_t now = n->t;  // latest stamp
    if (t_end > now + 1) return fail(DPSNN_E_RANGE, "range reaches past the last simulated step");
    const Dims& d = n->d;
    if (now >= d.R && t_begin < now - d.R + 1)
        return fail(DPSNN_E_RANGE, "range starts before the retained raster window");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    const size_t words = (size_t)d.C * d.W;
    std::vector<uint64_t> buf(words * (t_end - t_begin));
    for (uint32_t s = t_begin; s < t_end; ++s) {
        DPSNN_HIP(hipMemcpy(buf.data() + (size_t)(s - t_begin) * words,
                            n->ring + (size_t)(s % d.R) * words, words * sizeof(uint64_t),
                            hipMemcpyDeviceToHost));
    }
    size_t count = 0;
    for (uint64_t x : buf) count += (size_t)__builtin_popcountll(x);
    *n_out = count;
    if (count > cap) return fail(DPSNN_E_BUFSZ, "spike buffer too small");
    if (count && (!times || !ids)) return fail(DPSNN_E_INVAL, "NULL output buffer");
    size_t o = 0;
    for (uint32_t s = t_begin; s < t_end; ++s) {
        const uint64_t* row = buf.data() + (size_t)(s - t_begin) * words;
        for (uint32_t c = 0; c < d.C; ++c) {
            for (uint32_t w = 0; w < d.W; ++w) {
                uint64_t m = row[(size_t)c * d.W + w];
                while (m) {
                    const uint32_t b = (uint32_t)__builtin_ctzll(m);
                    m &= m - 1;
                    times[o] = s;
                    ids[o] = c * d.Ncol + w * 64 + b;
                    ++o;
                }
            }
        }
    }
    return DPSNN_OK;
}

// Reads canonical synapses [first, first + count) in groups of whole source
// columns: P of a group is moved from the reverse order into the forward
// layout of the scratch, then the rows are staged and copied to the caller's
// host arrays.  ws / ws_bytes: a caller-provided device region (no
// allocation), or null to allocate through the network's allocator.
static int read_rows_common(Net* n, uint64_t first, uint64_t count, uint32_t* tgt, uint8_t* dly,
                            float* w, float* P, float* D, void* ws = nullptr, size_t ws_bytes = 0) {
    if (first > n->S || count > n->S - first) return fail(DPSNN_E_RANGE, "synapse range out of bounds");
    if (count == 0) return DPSNN_OK;
    DPSNN_HIP(hipSetDevice(n->dev.device));
    const uint32_t M = n->d.M, Ncol = n->d.Ncol;
    const uint64_t colsz = (uint64_t)Ncol * M;
    ReadPlan pl;
    const size_t limit = ws ? ws_bytes : ~(size_t)0;
    if (!plan_read(*n, first, count, tgt, dly, w, P, D, kReadPBytes, kReadStageBytes, limit, pl))
        return fail(DPSNN_E_INVAL, "one column of this network does not fit the read workspace");
    unsigned char* base = static_cast<unsigned char*>(ws);
    const size_t nbytes = std::max<size_t>(pl.bytes(), 256);
    if (!base) {
        base = static_cast<unsigned char*>(dev_alloc(n->dev, n->stream, nbytes, nullptr));
        if (!base) return fail(DPSNN_E_NOMEM, "read scratch of " + std::to_string(nbytes) + " bytes");
    }
    auto done = [&](int rc) {
        (void)hipStreamSynchronize(n->stream);
        if (base && !ws) dfree(*n, base, nbytes);
        return rc;
    };
    float* Pg = P ? reinterpret_cast<float*>(base) : nullptr;
    unsigned char* st = base + pl.pg_bytes;
    const size_t sm = (size_t)pl.stage_rows * M;
    uint32_t* d_tgt = nullptr; uint8_t* d_dly = nullptr; float *d_w = nullptr, *d_P = nullptr, *d_D = nullptr;
    if (tgt) { d_tgt = reinterpret_cast<uint32_t*>(st); st += pad256(4 * sm); }
    if (dly) { d_dly = st; st += pad256(sm); }
    if (w) { d_w = reinterpret_cast<float*>(st); st += pad256(4 * sm); }
    if (P) { d_P = reinterpret_cast<float*>(st); st += pad256(4 * sm); }
    if (D) { d_D = reinterpret_cast<float*>(st); st += pad256(4 * sm); }
    for (uint32_t c0 = pl.cA; c0 < pl.cB; c0 += pl.group) {
        const uint32_t c1 = std::min<uint32_t>(pl.cB, c0 + pl.group);
        hipError_t e = P ? launch_P_to_forward(*n, Pg, c0, c1, false) : hipSuccess;
        if (e != hipSuccess) return done(fail(DPSNN_E_DEVICE, hipGetErrorString(e)));
        const uint32_t r_lo = std::max<uint32_t>(pl.i0, c0 * Ncol);
        const uint32_t r_hi = std::min<uint32_t>(pl.i1, c1 * Ncol);
        for (uint32_t r0 = r_lo; r0 < r_hi; r0 += pl.stage_rows) {
            const uint32_t r1 = std::min<uint32_t>(r_hi, r0 + pl.stage_rows);
            const uint64_t g0 = std::max<uint64_t>((uint64_t)r0 * M, first);
            const uint64_t g1 = std::min<uint64_t>((uint64_t)r1 * M, first + count);
            e = launch_read_rows(*n, r0, r1, g0, g1, Pg, (uint64_t)c0 * colsz, d_tgt, d_dly, d_w, d_P, d_D);
            if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
            const size_t m = (size_t)(g1 - g0), o = (size_t)(g0 - first);
            if (e == hipSuccess && tgt) e = hipMemcpy(tgt + o, d_tgt, 4 * m, hipMemcpyDeviceToHost);
            if (e == hipSuccess && dly) e = hipMemcpy(dly + o, d_dly, m, hipMemcpyDeviceToHost);
            if (e == hipSuccess && w) e = hipMemcpy(w + o, d_w, 4 * m, hipMemcpyDeviceToHost);
            if (e == hipSuccess && P) e = hipMemcpy(P + o, d_P, 4 * m, hipMemcpyDeviceToHost);
            if (e == hipSuccess && D) e = hipMemcpy(D + o, d_D, 4 * m, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return done(fail(DPSNN_E_DEVICE, hipGetErrorString(e)));
        }
    }
    return done(DPSNN_OK);
}

// ---- read-back without allocation --------------------------------------
// A library-owned workspace for callers that cannot allocate device memory.
// `scratch` names a device array; on the host the name is only a stand-in,
// so host code uses the address hipGetSymbolAddress returned for the current
// device (each GPU holds its own copy of the array).
static __device__ __align__(256) unsigned char scratch[DPSNN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch`, looked up once per device.
int scratch_for(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return fail(DPSNN_E_INVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DPSNN_E_DEVICE, std::string("workspace address: ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return DPSNN_OK;
}

}  // namespace

int dpsnn_read_weights_noalloc(dpsnn_net* h, uint64_t first, uint64_t count, float* w, float* P,
                               float* D) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    void* ws = nullptr;
    const int rc = scratch_for(n->dev.device, &ws);
    if (rc) return rc;
    return read_rows_common(n, first, count, nullptr, nullptr, w, P, D, ws, DPSNN_NOALLOC_SCRATCH_BYTES);
}

int dpsnn_read_weights(dpsnn_net* h, uint64_t first, uint64_t count, float* w, float* P, float* D) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    return read_rows_common(n, first, count, nullptr, nullptr, w, P, D);
}

int dpsnn_read_connectivity(dpsnn_net* h, uint64_t first, uint64_t count, uint32_t* target,
                            uint8_t* delay) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    return read_rows_common(n, first, count, target, delay, nullptr, nullptr, nullptr);
}

int dpsnn_read_state(dpsnn_net* h, float* v, float* u) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    if (v) DPSNN_HIP(hipMemcpy(v, n->v, sizeof(float) * n->d.N, hipMemcpyDeviceToHost));
    if (u) DPSNN_HIP(hipMemcpy(u, n->u, sizeof(float) * n->d.N, hipMemcpyDeviceToHost));
    return DPSNN_OK;
}

int dpsnn_get_stats(dpsnn_net* h, dpsnn_stats* st) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n || !st) return fail(DPSNN_E_INVAL, "NULL argument");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    DevStats hs[64];
    DPSNN_HIP(hipMemcpy(hs, n->stats, sizeof(hs), hipMemcpyDeviceToHost));
    std::memset(st, 0, sizeof(*st));
    for (int k = 0; k < 64; ++k) {
        st->spikes += hs[k].spikes;
        st->events += hs[k].events;
        st->ltp_visits += hs[k].ltp_visits;
        st->events_exc += hs[k].events_exc;
    }
    st->steps = n->t;
    st->consolidations = n->consolidations;
    st->graph_steps = n->graph_steps;
    n->timers.collect();
    st->ms_ltp = n->timers.ms[0]; st->ms_deliver = n->timers.ms[1];
    st->ms_neuron = n->timers.ms[2]; st->ms_wupdate = n->timers.ms[3];
    st->n_ltp = n->timers.n[0]; st->n_deliver = n->timers.n[1];
    st->n_neuron = n->timers.n[2]; st->n_wupdate = n->timers.n[3];
    return DPSNN_OK;
}

int dpsnn_set_stimulus(dpsnn_net* h, const uint32_t* t, const uint32_t* id, const float* mv, size_t cnt) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    if (cnt && (!t || !id || !mv)) return fail(DPSNN_E_INVAL, "NULL stimulus arrays");
    for (size_t e = 0; e < cnt; ++e) {
        if (id[e] >= n->d.N) return fail(DPSNN_E_INVAL, "stimulus neuron id out of range");
        if (!std::isfinite(mv[e]) || std::fabs(mv[e]) > 1e6f) return fail(DPSNN_E_INVAL, "stimulus value out of range");
    }
    if (cnt > 0xFFFFFFFFull) return fail(DPSNN_E_INVAL, "too many stimulus entries");
    if (n->in_batch) return fail(DPSNN_E_INVAL, "set the stimulus before adding the network to a batch");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    std::vector<size_t> order(cnt);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return t[a] < t[b]; });
    std::vector<uint32_t> sid(cnt), st(cnt);
    std::vector<float> smv(cnt);
    for (size_t e = 0; e < cnt; ++e) {
        sid[e] = id[order[e]];
        smv[e] = mv[order[e]];
        st[e] = t[order[e]];
    }
    // replace the previous list
    auto drop = [&](void* p) {
        if (!p) return;
        for (size_t a = 0; a < n->allocs.size(); ++a) {
            if (n->allocs[a].p == p) {
                dfree(*n, p, n->allocs[a].bytes);
                n->allocs.erase(n->allocs.begin() + (long)a);
                break;
            }
        }
    };
    drop(n->stim_t);
    drop(n->stim_id);
    drop(n->stim_mv);
    n->stim_t = nullptr;
    n->stim_id = nullptr;
    n->stim_mv = nullptr;
    n->stim_n = 0;
    n->desc_dirty = true;
    if (cnt == 0) return DPSNN_OK;
    n->stim_t = (uint32_t*)dalloc(*n, sizeof(uint32_t) * cnt);
    n->stim_id = (uint32_t*)dalloc(*n, sizeof(uint32_t) * cnt);
    n->stim_mv = (float*)dalloc(*n, sizeof(float) * cnt);
    if (!n->stim_t || !n->stim_id || !n->stim_mv) return fail(DPSNN_E_NOMEM, "stimulus buffers");
    DPSNN_HIP(hipMemcpy(n->stim_t, st.data(), sizeof(uint32_t) * cnt, hipMemcpyHostToDevice));
    DPSNN_HIP(hipMemcpy(n->stim_id, sid.data(), sizeof(uint32_t) * cnt, hipMemcpyHostToDevice));
    DPSNN_HIP(hipMemcpy(n->stim_mv, smv.data(), sizeof(float) * cnt, hipMemcpyHostToDevice));
    n->stim_n = cnt;
    return DPSNN_OK;
}

int dpsnn_set_probes(dpsnn_net* h, const uint32_t* ids, uint32_t count) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    if (count && !ids) return fail(DPSNN_E_INVAL, "NULL probe ids");
    if (count > kMaxProbes) return fail(DPSNN_E_INVAL, "too many probes");
    for (uint32_t e = 0; e < count; ++e)
        if (ids[e] >= n->d.N) return fail(DPSNN_E_INVAL, "probe neuron id out of range");
    if (n->in_batch) return fail(DPSNN_E_INVAL, "set probes before adding the network to a batch");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    auto drop = [&](void* p) {
        if (!p) return;
        for (size_t a = 0; a < n->allocs.size(); ++a) {
            if (n->allocs[a].p == p) {
                dfree(*n, p, n->allocs[a].bytes);
                n->allocs.erase(n->allocs.begin() + (long)a);
                break;
            }
        }
    };
    drop(n->probe_id);
    drop(n->probe_buf);
    n->probe_id = nullptr;
    n->probe_buf = nullptr;
    n->probe_n = 0;
    n->desc_dirty = true;
    if (count == 0) return DPSNN_OK;
    n->probe_id = (uint32_t*)dalloc(*n, sizeof(uint32_t) * count);
    n->probe_buf = (float*)dalloc(*n, sizeof(float) * 2 * (size_t)count * n->d.R);
    if (!n->probe_id || !n->probe_buf) {
        drop(n->probe_id);
        drop(n->probe_buf);
        n->probe_id = nullptr;
        n->probe_buf = nullptr;
        return fail(DPSNN_E_NOMEM, "probe buffers");
    }
    DPSNN_HIP(hipMemcpy(n->probe_id, ids, sizeof(uint32_t) * count, hipMemcpyHostToDevice));
    n->probe_n = count;
    n->probe_from = n->t + 1;
    return DPSNN_OK;
}

int dpsnn_read_probes(dpsnn_net* h, uint32_t t_begin, uint32_t t_end, float* v, float* u) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    if (t_end < t_begin) return fail(DPSNN_E_INVAL, "t_end < t_begin");
    if (t_end == t_begin) return DPSNN_OK;
    if (!n->probe_n) return fail(DPSNN_E_INVAL, "no probes are set");
    const uint32_t now = n->t, R = n->d.R;
    if (t_begin < n->probe_from || t_end > now + 1)
        return fail(DPSNN_E_RANGE, "steps outside the recorded probe range");
    if (now >= R && t_begin < now - R + 1)
        return fail(DPSNN_E_RANGE, "steps before the retained probe window");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    const size_t pn = n->probe_n;
    std::vector<float> row(2 * pn);
    for (uint32_t s = t_begin; s < t_end; ++s) {
        DPSNN_HIP(hipMemcpy(row.data(), n->probe_buf + (size_t)(s % R) * 2 * pn, sizeof(float) * 2 * pn,
                            hipMemcpyDeviceToHost));
        if (v) std::memcpy(v + (size_t)(s - t_begin) * pn, row.data(), sizeof(float) * pn);
        if (u) std::memcpy(u + (size_t)(s - t_begin) * pn, row.data() + pn, sizeof(float) * pn);
    }
    return DPSNN_OK;
}

int dpsnn_set_timing(dpsnn_net* h, int enable) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    n->timers.on = enable != 0;
    return DPSNN_OK;
}

int dpsnn_set_tuning(dpsnn_net* h, uint32_t key, uint32_t value) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    return apply_tuning(n->tune, key, value);
}

int dpsnn_autotune(dpsnn_net* h, uint32_t steps_per_trial) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n) return fail(DPSNN_E_INVAL, "net is NULL");
    if (n->in_batch) return fail(DPSNN_E_INVAL, "the network belongs to a batch; tune the batch");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    Net* one[1] = {n};
    if (n->desc_dirty) {
        int rc = refresh_descs(n->solo, one, n->stream);
        if (rc) return rc;
        n->desc_dirty = false;
    }
    return autotune(n->solo, n->tune, n->timers, n->stream, one, steps_per_trial);
}

int dpsnn_get_config(dpsnn_net* h, dpsnn_config* cfg) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n || !cfg) return fail(DPSNN_E_INVAL, "NULL argument");
    *cfg = n->cfg;
    return DPSNN_OK;
}

int dpsnn_checkpoint_bytes(dpsnn_net* h, uint64_t* bytes) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n || !bytes) return fail(DPSNN_E_INVAL, "NULL argument");
    *bytes = ckpt_total(ckpt_parts(*n, n->stim_n));
    return DPSNN_OK;
}

int dpsnn_save(dpsnn_net* h, void* buf, uint64_t cap) {
    Net* n = reinterpret_cast<Net*>(h);
    if (!n || !buf) return fail(DPSNN_E_INVAL, "NULL argument");
    const std::vector<CkptPart> parts = ckpt_parts(*n, n->stim_n);
    const uint64_t total = ckpt_total(parts);
    if (cap < total) return fail(DPSNN_E_BUFSZ, "checkpoint buffer too small");
    DPSNN_HIP(hipSetDevice(n->dev.device));
    DPSNN_HIP(hipStreamSynchronize(n->stream));
    unsigned char* out = static_cast<unsigned char*>(buf);
    CkptHeader hd;
    std::memset(&hd, 0, sizeof(hd));
    std::memcpy(hd.magic, kCkptMagic, sizeof(kCkptMagic));
    hd.version = kCkptVersion;
    hd.header_bytes = (uint32_t)sizeof(CkptHeader);
    hd.cfg = n->cfg;
    hd.t = n->t;
    hd.consolidations = n->consolidations;
    hd.stim_n = n->stim_n;
    hd.total_bytes = total;
    std::memset(out, 0, pad16(sizeof(hd)));
    std::memcpy(out, &hd, sizeof(hd));
    hipError_t e = hipSuccess;
    size_t off = pad16(sizeof(hd));
    size_t off_P = 0;
    for (size_t k = 0; k < parts.size(); ++k) {
        const CkptPart& q = parts[k];
        if (k == kCkptP) off_P = off;
        else if (e == hipSuccess && q.bytes) e = hipMemcpy(out + off, q.dev, q.bytes, hipMemcpyDeviceToHost);
        off += pad16(q.bytes);
    }
    if (e != hipSuccess) return fail(DPSNN_E_DEVICE, hipGetErrorString(e));
    // P in the forward layout, a group of source columns at a time
    PGroups pg;
    if (!alloc_pgroups(n, pg)) return fail(DPSNN_E_NOMEM, "checkpoint P buffer (one column)");
    const uint64_t colsz = (uint64_t)n->d.Ncol * n->d.M;
    for (uint32_t c0 = 0; c0 < n->d.C && e == hipSuccess; c0 += pg.group) {
        const uint32_t c1 = std::min<uint32_t>(n->d.C, c0 + pg.group);
        e = launch_P_to_forward(*n, pg.buf, c0, c1, true);
        if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
        if (e == hipSuccess)
            e = hipMemcpy(out + off_P + 4 * (size_t)c0 * colsz, pg.buf, 4 * (size_t)(c1 - c0) * colsz,
                          hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) return fail(DPSNN_E_DEVICE, hipGetErrorString(e));
    return DPSNN_OK;
}

int dpsnn_load(const void* buf, uint64_t size, const dpsnn_device* dev, dpsnn_net** out) {
    if (!out) return fail(DPSNN_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!buf || size < sizeof(CkptHeader)) return fail(DPSNN_E_INVAL, "not a checkpoint (too short)");
    CkptHeader hd;
    std::memcpy(&hd, buf, sizeof(hd));
    if (std::memcmp(hd.magic, kCkptMagic, sizeof(kCkptMagic)) != 0)
        return fail(DPSNN_E_INVAL, "not a checkpoint (bad magic)");
    if (hd.version != kCkptVersion || hd.header_bytes != sizeof(CkptHeader))
        return fail(DPSNN_E_INVAL, "checkpoint of another format version");
    Derived dv;
    int rc = validate(&hd.cfg, &dv);
    if (rc) return rc;
    if (hd.cfg.raster_steps != dv.R || hd.t >= (1ull << 31) || hd.stim_n > 0xFFFFFFFFull ||
        hd.total_bytes != size)
        return fail(DPSNN_E_INVAL, "inconsistent checkpoint header");
    // contents are checked on the host, before any device work
    const std::vector<size_t> sizes = ckpt_sizes(dv.N, dv.C, dv.W, dv.R, dv.S, hd.stim_n);
    if (ckpt_total(sizes) != size)
        return fail(DPSNN_E_INVAL, "checkpoint size does not match its configuration");
    if (!ckpt_raster_in_range(static_cast<const unsigned char*>(buf), sizes, dv))
        return fail(DPSNN_E_INVAL, "checkpoint raster has spikes beyond a column's last neuron");
    dpsnn_net* h = nullptr;
    rc = dpsnn_build_network(&hd.cfg, dev, &h);
    if (rc) return rc;
    Net* n = reinterpret_cast<Net*>(h);
    const unsigned char* in = static_cast<const unsigned char*>(buf);
    const size_t stim_off = [&] {
        size_t o = pad16(sizeof(CkptHeader));
        const std::vector<CkptPart> p0 = ckpt_parts(*n, hd.stim_n);
        for (size_t k = 0; k + 3 < p0.size(); ++k) o += pad16(p0[k].bytes);
        return o;
    }();
    if (ckpt_total(ckpt_parts(*n, hd.stim_n)) != size) {
        release(n);
        return fail(DPSNN_E_INVAL, "checkpoint size does not match its configuration");
    }
    // the stimulus list first (it allocates), then every state array
    if (hd.stim_n) {
        const uint32_t* st = reinterpret_cast<const uint32_t*>(in + stim_off);
        const uint32_t* si = reinterpret_cast<const uint32_t*>(in + stim_off + pad16(4 * hd.stim_n));
        const float* sm = reinterpret_cast<const float*>(in + stim_off + 2 * pad16(4 * hd.stim_n));
        rc = dpsnn_set_stimulus(h, st, si, sm, (size_t)hd.stim_n);
        if (rc) {
            release(n);
            return rc;
        }
    }
    const std::vector<CkptPart> parts = ckpt_parts(*n, hd.stim_n);
    hipError_t e = hipSuccess;
    size_t off = pad16(sizeof(CkptHeader));
    size_t off_P = 0;
    for (size_t k = 0; k + 3 < parts.size(); ++k) {
        const CkptPart& q = parts[k];
        if (k == kCkptP) off_P = off;
        else if (e == hipSuccess && q.bytes) e = hipMemcpy(q.dev, in + off, q.bytes, hipMemcpyHostToDevice);
        off += pad16(q.bytes);
    }
    {
        // P from the forward layout, a group of source columns at a time
        PGroups pg;
        if (e == hipSuccess && !alloc_pgroups(n, pg)) {
            release(n);
            return fail(DPSNN_E_NOMEM, "checkpoint P buffer (one column)");
        }
        const uint64_t colsz = (uint64_t)n->d.Ncol * n->d.M;
        for (uint32_t c0 = 0; c0 < n->d.C && e == hipSuccess; c0 += pg.group) {
            const uint32_t c1 = std::min<uint32_t>(n->d.C, c0 + pg.group);
            e = hipStreamSynchronize(n->stream);  // the previous group has been consumed
            if (e == hipSuccess)
                e = hipMemcpy(pg.buf, in + off_P + 4 * (size_t)c0 * colsz, 4 * (size_t)(c1 - c0) * colsz,
                              hipMemcpyHostToDevice);
            if (e == hipSuccess) e = launch_P_from_forward(*n, pg.buf, c0, c1);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
    }
    if (e != hipSuccess) {
        release(n);
        return fail(DPSNN_E_DEVICE, std::string("checkpoint upload failed: ") + hipGetErrorString(e));
    }
    n->t = (uint32_t)hd.t;
    n->consolidations = hd.consolidations;
    n->desc_dirty = true;  // descriptors take t0 = t at the next step
    *out = h;
    return DPSNN_OK;
}

void dpsnn_destroy(dpsnn_net* h) {
    Net* n = reinterpret_cast<Net*>(h);
    if (n && n->in_batch) {
        fail(DPSNN_E_INVAL, "destroying a network that belongs to a batch");
        return;
    }
    if (n && n->owner) {
        fail(DPSNN_E_INVAL, "a server job's network is freed by dpsnn_server_release");
        return;
    }
    release(n);
}

int dpsnn_batch_create(dpsnn_net* const* nets, uint32_t n_nets, dpsnn_batch** out) {
    if (!out) return fail(DPSNN_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!nets || n_nets == 0) return fail(DPSNN_E_INVAL, "a batch needs at least one network");
    std::vector<Net*> m(n_nets);
    for (uint32_t k = 0; k < n_nets; ++k) {
        m[k] = reinterpret_cast<Net*>(nets[k]);
        if (!m[k]) return fail(DPSNN_E_INVAL, "NULL network in batch");
        if (m[k]->in_batch) return fail(DPSNN_E_INVAL, "a network is already in a batch");
        for (uint32_t q = 0; q < k; ++q)
            if (m[q] == m[k]) return fail(DPSNN_E_INVAL, "a network appears twice in the batch");
        if (m[k]->dev.device != m[0]->dev.device || m[k]->stream != m[0]->stream)
            return fail(DPSNN_E_INVAL, "batch members must share device and stream");
        if (m[k]->cfg.sum_mode != m[0]->cfg.sum_mode || m[k]->tgt16 != m[0]->tgt16)
            return fail(DPSNN_E_INVAL, "batch members must share summation mode and target width");
    }
    if (m[0]->cfg.sum_mode == DPSNN_SUM_ORDERED)
        return fail(DPSNN_E_INVAL, "ORDERED summation runs one network at a time");
    DPSNN_HIP(hipSetDevice(m[0]->dev.device));
    dpsnn_batch* b = new dpsnn_batch();
    b->members = m;
    b->stream = m[0]->stream;
    b->dev = m[0]->dev;
    b->tune = m[0]->tune;
    int rc = make_launch_set(b->L, b->members.data(), n_nets, b->dev, b->stream, &b->allocs, true);
    if (rc) {
        release_launch_set_host(b->L);
        free_tracked(b->dev, b->stream, b->allocs);
        delete b;
        return rc;
    }
    for (Net* x : m) x->in_batch = true;
    *out = b;
    return DPSNN_OK;
}

int dpsnn_batch_step(dpsnn_batch* b, uint32_t n_steps) {
    if (!b) return fail(DPSNN_E_INVAL, "batch is NULL");
    for (Net* x : b->members)
        if ((uint64_t)x->t + n_steps >= (1ull << 31)) return fail(DPSNN_E_RANGE, "step count overflow");
    // members' descriptors cannot change while they are in the batch (their
    // stimulus is fixed), so the tables uploaded at creation stay valid
    DPSNN_HIP(hipSetDevice(b->dev.device));
    DPSNN_HIP(launch_steps(b->L, b->tune, b->timers, b->stream, b->members.data(), n_steps));
    return DPSNN_OK;
}

int dpsnn_batch_get_stats(dpsnn_batch* b, dpsnn_stats* st) {
    if (!b || !st) return fail(DPSNN_E_INVAL, "NULL argument");
    std::memset(st, 0, sizeof(*st));
    for (Net* x : b->members) {
        dpsnn_stats one;
        int rc = dpsnn_get_stats(reinterpret_cast<dpsnn_net*>(x), &one);
        if (rc) return rc;
        st->steps += one.steps;
        st->spikes += one.spikes;
        st->events += one.events;
        st->ltp_visits += one.ltp_visits;
        st->consolidations += one.consolidations;
        st->events_exc += one.events_exc;
        st->graph_steps += one.graph_steps;
    }
    b->timers.collect();
    st->ms_ltp = b->timers.ms[0]; st->ms_deliver = b->timers.ms[1];
    st->ms_neuron = b->timers.ms[2]; st->ms_wupdate = b->timers.ms[3];
    st->n_ltp = b->timers.n[0]; st->n_deliver = b->timers.n[1];
    st->n_neuron = b->timers.n[2]; st->n_wupdate = b->timers.n[3];
    return DPSNN_OK;
}

int dpsnn_batch_set_timing(dpsnn_batch* b, int enable) {
    if (!b) return fail(DPSNN_E_INVAL, "batch is NULL");
    b->timers.on = enable != 0;
    return DPSNN_OK;
}

int dpsnn_batch_set_tuning(dpsnn_batch* b, uint32_t key, uint32_t value) {
    if (!b) return fail(DPSNN_E_INVAL, "batch is NULL");
    return apply_tuning(b->tune, key, value);
}

int dpsnn_batch_autotune(dpsnn_batch* b, uint32_t steps_per_trial) {
    if (!b) return fail(DPSNN_E_INVAL, "batch is NULL");
    DPSNN_HIP(hipSetDevice(b->dev.device));
    return autotune(b->L, b->tune, b->timers, b->stream, b->members.data(), steps_per_trial);
}

void dpsnn_batch_destroy(dpsnn_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->dev.device);
    (void)hipStreamSynchronize(b->stream);
    release_launch_set_host(b->L);
    free_tracked(b->dev, b->stream, b->allocs);
    b->timers.release();
    for (Net* x : b->members) x->in_batch = false;
    delete b;
}

}  // extern "C"
