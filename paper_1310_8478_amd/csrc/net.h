// Host-side network object of libdpsnn and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "dev_common.h"
#include "dpsnn.h"

namespace dpsnn {

constexpr uint32_t kXcds = 8;  // accelerator dies (XCDs) of the GPU, each with its own L2

// Launch-shape knobs; results never depend on them.  "Auto" values follow the
// launch set's measured regime: sparse (at least 2048 columns, and a source
// column delivers fewer events per step than its current window has entries)
// or dense.
struct Tuning {
    uint32_t deliver_block = 0;   // 256, 512, 1024; 0 auto (sparse 256, dense 1024)
    uint32_t ltp_block = 0;       // 256, 512, 1024; 0 auto (sparse 256, dense 1024)
    uint32_t window = 3;          // 0 off, 1 all 13 columns, 2 partial (own_slots); 3 auto (2 / 1)
    uint32_t unroll = 4;           // events (quads) in flight per lane in delivery
    uint32_t age = 2;             // LDS target spike ages: 0 off, 1 on, 2 auto (off / on)
    uint32_t parts = 0;           // workgroups per column (0: chosen per launch set)
    uint32_t ltp_stage = 2;       // LDS source spike history in LTP: 0, 1, 2 auto (0 / 1)
    uint32_t fuse = 0xFFFFFFFFu;  // LTP + delivery as one kernel up to this many workgroups each
    uint32_t graph = 8;           // steps per captured graph; 0 = every step launched directly
    uint32_t split = 1;           // workgroups sharing a column's full window by slot (1..13)
    uint32_t own_slots = 0;       // slots of the partial window (window 2), 1..13; 0 auto (3 / 1)
    uint32_t sparse_ltp = 2;      // wavefront-level LTP: 0 off, 1 on, 2 auto (on / off)
    uint32_t sparse_deliver = 2;  // wavefront-level delivery (and LTP): 0 off, 1 on, 2 auto (off)
    uint32_t ltp_cols = 0;        // target columns per sparse LTP workgroup, 1..8; 0 auto
    uint32_t consolidate = 1;     // 1: one forward-order pass where fwd_rev exists; 0: two passes
    size_t max_lds = 65536;
};

// Per-kernel device timers (the paper's per-block profiling, Table 2).
struct Timers {
    bool on = false;
    struct Timed { int kind; hipEvent_t a, b; };
    std::vector<Timed> pending;
    std::vector<hipEvent_t> pool;
    double ms[4] = {0, 0, 0, 0};
    uint64_t n[4] = {0, 0, 0, 0};
    void begin(int kind, hipStream_t s);
    void end(hipStream_t s);
    void collect();   // after a synchronisation: fold pending events into ms / n
    void release();
};

// The device tables of one launch over K networks: their descriptors and
// block maps (network, column), (network, first raster word), and per network
// the consolidation chunks.  A single network is a set of one.
struct LaunchSet {
    uint32_t K = 0;
    NetDesc* descs = nullptr;
    uint2* bmap_col = nullptr;
    uint32_t n_col = 0;
    uint2* bmap_neu = nullptr;
    uint32_t n_neu = 0;
    std::vector<uint2*> bmap_wu;
    std::vector<uint32_t> n_wu;
    uint32_t max_ncol = 0, max_w = 0, sum_mode = 0;
    uint64_t min_col_syn = 0;     // fewest synapses of one column over the members
    double avg_nwin = 0.0;        // mean current-window entries (13 x Ncol) per column
    bool tgt16 = true;
    // regime estimate: delivered events per column and step, from a device
    // counter copied to pinned host memory every few steps without waiting
    unsigned long long* ev_count = nullptr;  // device (one of the set's tables)
    unsigned long long* ev_host = nullptr;   // pinned host copy
    hipEvent_t ev_copied = nullptr;
    bool copy_pending = false;
    uint64_t steps = 0, copy_steps = 0, base_steps = 0, base_count = 0;
    double per_col = 0.0;
    // regime with hysteresis: sparse below 0.8 window entries per column, dense
    // above 1.0, unchanged in between
    bool sparse = true;
    // captured graph of graph_steps steps (launch shapes graph_tune), and the
    // stream it was captured on
    hipGraphExec_t graph = nullptr;
    hipStream_t cap_stream = nullptr;
    uint32_t graph_steps = 0;
    Tuning graph_tune;
    uint32_t graph_probes = 0;
    // most state probes of one member (0: no probe kernel in the step)
    uint32_t max_probes = 0;
    // host copies of the uploaded tables (t0 mirrors the device descriptors)
    std::vector<NetDesc> host_descs;
    std::vector<uint2> host_col, host_neu;
    std::vector<std::vector<uint2>> host_wu;
};

// Device arrays of one network.  Layout (all device memory):
//   forward synapses, "column-delay-major": the synapses of column c occupy
//   [c*Ncol*M, (c+1)*Ncol*M); inside, segment (d, l) holds the synapses of
//   local neuron l with delay d in ascending j, segments ordered by d then l,
//   so all sources of a column that share a delay are contiguous.
//     seg_off[c*segs + (d-1)*Ncol + l] = first position of segment (d, l),
//     seg_off[C*segs] = N*M (so the end of a segment is the next entry);
//     positions are 64-bit, offsets inside one column's block fit 32 bits.
//     Kernels address a column through pointers offset by its block start
//     rounded down to a multiple of 4, so 32-bit offsets keep the 16-byte
//     alignment of the synapse quads.
//     tgt[pos] = slot*Ncol + local target (window index); w[pos]; D[pos].
//   reverse index of excitatory synapses, rows by global target id:
//     rowptr[k] .. rowptr[k+1] (64-bit); rev_srcd = slot<<22 | local source<<6
//     | delay; rev_fwd = forward position minus the source column's block
//     start (32-bit); P = potentiation accumulator.  Rows up to 8192 entries
//     are sorted by (rev_srcd, rev_fwd), so each source column's entries in
//     a row are contiguous.
//   fwd_rev: forward position -> source slot and reverse entry (consolidation).
//   raster ring: R slots of C*W 64-bit words; stamp s lives in slot s % R.
struct Net {
    dpsnn_config cfg;
    dpsnn_device dev;
    Dims d;
    hipStream_t stream = nullptr;
    uint32_t t = 0;                // host mirror of the device clock
    bool tgt16 = true;
    bool in_batch = false;
    void* owner = nullptr;         // the job server holding this network, if any
    uint64_t S = 0, S_exc = 0;

    // allocations
    struct Alloc { void* p; size_t bytes; };
    std::vector<Alloc> allocs;

    uint32_t* colmap = nullptr;   // [C*13] column reached from c through slot q
    uint32_t* srcmap = nullptr;   // [C*13] column that reaches c through slot q
    uint64_t* seg_off = nullptr;  // [C*segs + 1]
    void* tgt = nullptr;          // uint16_t or uint32_t [S]
    float* w = nullptr;           // [S]
    float* Dacc = nullptr;        // [S]
    uint64_t* rowptr = nullptr;   // [N+1]
    uint32_t* cursor = nullptr;   // [N] build scratch; ORDERED event cursor afterwards
    uint32_t* rev_srcd = nullptr; // [S_exc]
    uint32_t* rev_fwd = nullptr;  // [S_exc]
    float* Pacc = nullptr;        // [S_exc]
    // [S] (when 13 * Ncol * M <= 2^28, else null): slot << 28 | reverse
    // entry minus the first reverse position of the target column reached
    // through slot; 0xFFFFFFFF at inhibitory positions
    uint32_t* fwd_rev = nullptr;
    float* v = nullptr;
    float* u = nullptr;
    void* acc = nullptr;          // long long[N] (FIXED) or float[N]
    // [N] x: bit b set if spiked at (latest stamp time) - b; y: latest stamp
    // older than that 32-step window (int32), so one 8-byte load gives both
    uint2* hist = nullptr;
    int32_t* t_last = nullptr;    // [N] latest stamp
    uint64_t* ring = nullptr;     // [R*C*W]
    float* tp = nullptr;          // [tp_len] LTP amplitudes by dt
    float* tm = nullptr;          // [tm_len] LTD amplitudes by dt
    uint32_t tp_len = 0, tm_len = 0;
    DevStats* stats = nullptr;    // [64] spread counters
    uint64_t* scan_tmp = nullptr; // block sums of the device-wide scans
    uint64_t* col_rev_dev = nullptr;  // [C+1] copy source of col_rev
    // ORDERED mode event buffers
    uint32_t* ev_cnt = nullptr;   // [N]
    uint32_t* ev_start = nullptr; // [N+1]
    unsigned long long* ev_key = nullptr;  // [S]
    float* ev_w = nullptr;        // [S]
    // state probes: v and u of chosen neurons after every step (the paper's
    // optional trace of individual neurons' state variables)
    uint32_t* probe_id = nullptr; // [probe_n]
    float* probe_buf = nullptr;   // [R][2][probe_n]
    uint32_t probe_n = 0;
    uint32_t probe_from = 0;      // first step count recorded

    // stimulus, sorted by step (stable)
    uint32_t* stim_t = nullptr;
    uint32_t* stim_id = nullptr;
    float* stim_mv = nullptr;
    size_t stim_n = 0;

    // host mirrors
    uint64_t consolidations = 0;
    uint64_t graph_steps = 0;     // steps run as replays of a captured graph
    uint32_t thal_whole = 0, thal_thr = 0;

    Tuning tune;
    Timers timers;
    LaunchSet solo;               // this network alone
    bool desc_dirty = true;
    double per_col = 0.0;         // last regime estimate of a set holding this network
    std::vector<uint64_t> col_rev;  // [C+1] reverse positions where each target column starts

    NetDesc make_desc() const;
};

// Host helpers shared by the C ABI files (api.cpp, serve.cpp).
// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string& msg);
void* dev_alloc(const dpsnn_device& dev, hipStream_t stream, size_t bytes,
                std::vector<Net::Alloc>* track);
void free_tracked(const dpsnn_device& dev, hipStream_t stream, std::vector<Net::Alloc>& allocs);
int make_launch_set(LaunchSet& L, Net* const* m, uint32_t cnt, const dpsnn_device& dev,
                    hipStream_t stream, std::vector<Net::Alloc>* track, bool sync);
// Frees every device allocation of n (after synchronising its stream) and n.
void destroy_net(Net* n);
// Host resources of a launch set (pinned copy, event); the device tables are
// freed with their owner's tracked allocations.
void release_launch_set_host(LaunchSet& L);

// launchers (return hipError_t)
hipError_t launch_build(Net& n);
// One step of every network of the set; members[k] is the network of slot k.
hipError_t launch_step_set(LaunchSet& L, const Tuning& tune, Timers& tm, hipStream_t stream,
                           Net* const* members);
// n_steps steps of the set, runs of tune.graph steps as captured graphs.
hipError_t launch_steps(LaunchSet& L, const Tuning& tune, Timers& tm, hipStream_t stream,
                        Net* const* members, uint32_t n_steps);
hipError_t launch_read_rows(Net& n, uint32_t i0, uint32_t i1, uint64_t g_lo, uint64_t g_hi,
                            const float* Pg, uint64_t pg_base, uint32_t* tgt_out,
                            uint8_t* dly_out, float* w_out, float* P_out, float* D_out);
// P between the reverse order (a property of the build) and the forward
// layout (fixed by the configuration), for the
// source columns [c0, c1): Pg holds their forward blocks back to back
// ((c1 - c0) * Ncol * M floats).  To the forward layout, inhibitory positions
// are left as they are unless zero_first clears the range first.
hipError_t launch_P_to_forward(Net& n, float* Pg, uint32_t c0, uint32_t c1, bool zero_first);
hipError_t launch_P_from_forward(Net& n, float* Pg, uint32_t c0, uint32_t c1);
hipError_t scan_u32(Net& n, hipStream_t stream, const uint32_t* in, uint32_t* out, uint32_t count);
hipError_t scan_u32_u64(Net& n, hipStream_t stream, const uint32_t* in, uint64_t* out, uint32_t count);

}  // namespace dpsnn
