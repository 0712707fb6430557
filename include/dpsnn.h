/*
 * dpsnn.h — C ABI of the MI355X DPSNN-STDP step library (libdpsnn.so).
 *
 * The library simulates, on one GPU, the 1 ms step of a 2-D grid of cortical
 * columns of Izhikevich neurons with individual axonal delays and
 * spike-timing-dependent plasticity, as described in Paolucci et al.,
 * arXiv 1310.8478 (Sec. 2, "Methods").  Each step runs, in order:
 *   LTP of the incoming synapses of the neurons that fired in the previous
 *   step (Sec. 2, loop item 2.1); delivery of queued axonal spikes to the
 *   synapses whose delay matches (items 2.3-2.4), current injection and LTD
 *   (items 2.5-2.6); the neuron update with the thalamic input and the
 *   raster (item 2.7); and, every weight_update_period steps, the long-term
 *   plasticity consolidation (Sec. 3, Table 2, last row).
 *
 * Conventions for every entry point:
 *   - Return 0 (DPSNN_OK) on success, a negative DPSNN_E_* code on failure;
 *     dpsnn_last_error() then returns a thread-local message.  The library
 *     never aborts the process.
 *   - Host pointers belong to the caller and are only read or written during
 *     the call.  Device memory is owned by the network and released by
 *     dpsnn_destroy().
 *   - All device work is enqueued on the stream given at build time; the
 *     read_* calls synchronise that stream before returning.
 *   - Neuron ids are global: id = column * neurons_per_column + local, with
 *     column = cy * grid_x + cx; local ids below round(exc_fraction *
 *     neurons_per_column) are excitatory (RS), the rest inhibitory (FS).
 *   - Synapses are addressed canonically by g = id * synapses_per_neuron + j,
 *     j in [0, synapses_per_neuron), independently of the device layout.
 *   - Spike stamps: a neuron that crosses threshold while step t (0-based)
 *     is computed gets stamp t + 1; stamps therefore lie in 1..steps_done.
 */
#ifndef DPSNN_H
#define DPSNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPSNN_OK        0
#define DPSNN_E_INVAL  (-1)   /* invalid argument or configuration */
#define DPSNN_E_NOMEM  (-2)   /* a device allocation failed */
#define DPSNN_E_DEVICE (-3)   /* a HIP runtime call failed */
#define DPSNN_E_RANGE  (-4)   /* requested steps are not (or no longer) held */
#define DPSNN_E_BUFSZ  (-5)   /* caller buffer too small; *n_out holds the size needed */
#define DPSNN_E_TIMEOUT (-6)  /* a wait ended before the job finished */
#define DPSNN_E_CANCELED (-7) /* the job was cancelled (dpsnn_server_cancel) */

/* Current summation modes (the paper fixes no order or precision for the
 * sum of currents arriving in one step; Sec. 2, "Projection of synapses"). */
#define DPSNN_SUM_ORDERED 0u  /* fp32 left fold: thalamic picks, stimulus list,
                                 then deliveries by (delay, source id, synapse j);
                                 a reference mode: each step also writes every
                                 event's key and sorts them per target, several
                                 times slower than FIXED at paper rates and far
                                 slower when every input arrives every step */
#define DPSNN_SUM_ATOMIC  1u  /* fp32, unordered atomics: not bit-reproducible
                                 (a source column's contributions to one target
                                 are summed exactly, then rounded to fp32 once
                                 and added with an atomic in arbitrary order) */
#define DPSNN_SUM_FIXED   2u  /* each term rounded to a multiple of 2^-32, summed
                                 exactly in int64, the total rounded once to fp32 */

#define DPSNN_CONN_CONFIG 0u  /* own_fraction of exc synapses to the own column,
                                 the rest uniform over the 12 neighbour columns */
#define DPSNN_CONN_PAPER  1u  /* 76 % own, 3 % each first, 2 % each second, 1 %
                                 each third neighbour (Sec. 3, after Table 1) */

/* Network description.  Cited values are the paper's; the others are the
 * measured workloads' constants. */
typedef struct dpsnn_config {
    uint32_t grid_x, grid_y;          /* CFX x CFY columns, periodic (Sec. 2) */
    uint32_t neurons_per_column;      /* 2 .. 65535 */
    float    exc_fraction;            /* 0.8 (Sec. 2, neuron model) */
    uint32_t synapses_per_neuron;     /* M, 1 .. 65535 (Sec. 2, projection) */
    uint32_t conn_mode;               /* DPSNN_CONN_* */
    float    own_fraction;            /* used by DPSNN_CONN_CONFIG */
    uint32_t max_delay;               /* 1 .. 31 ms; exc delays uniform in 1..max */
    float    w_exc_init, w_inh, w_max;
    float    a_plus, a_minus, tau_plus, tau_minus;  /* STDP rule (Sec. 2) */
    uint32_t weight_update_period;    /* steps; 0 disables consolidation */
    float    wu_bias, sd_decay;       /* w += bias + (P - D); P <- decay*(P - D) */
    float    thalamic_rate;           /* events per column per ms, [0, 1024) */
    float    thalamic_current;        /* mV per thalamic event */
    uint64_t seed;                    /* Philox key for connectivity and input */
    uint32_t sum_mode;                /* DPSNN_SUM_* */
    uint32_t raster_steps;            /* steps of raster kept on device;
                                         0 = default (1024); at least max_delay+1 */
} dpsnn_config;

/* Device, stream and allocator.  alloc/free may be NULL, in which case the
 * library calls hipMalloc/hipFree.  alloc returns device memory of at least
 * `bytes` bytes usable on `stream`, or NULL on failure. */
typedef struct dpsnn_device {
    int   device;                     /* HIP device ordinal */
    void *stream;                     /* hipStream_t; NULL = the null stream */
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void  (*free)(void *ptr, size_t bytes, void *stream, void *ctx);
    void *ctx;
} dpsnn_device;

typedef struct dpsnn_stats {
    uint64_t steps;           /* steps simulated */
    uint64_t spikes;          /* spikes emitted (raster rows) */
    uint64_t events;          /* synaptic deliveries (one per synapse per arrival) */
    uint64_t ltp_visits;      /* incoming excitatory synapses walked by LTP */
    uint64_t consolidations;  /* weight-update passes run */
    uint64_t events_exc;      /* deliveries through excitatory (plastic) synapses */
    /* per-kernel device time, accumulated only while timing is enabled;
     * when LTP and delivery run as one kernel (dpsnn_set_tuning key 7) their
     * time is counted under delivery */
    double   ms_ltp, ms_deliver, ms_neuron, ms_wupdate;
    uint64_t n_ltp, n_deliver, n_neuron, n_wupdate;
    uint64_t graph_steps;     /* steps run as replays of a captured graph */
} dpsnn_stats;

typedef struct dpsnn_net dpsnn_net;

/* Fill *cfg with the defaults: 2x2 grid, 1250 neurons per column, M = 100,
 * configuration-mode connectivity, the constants listed in the paper and the
 * workloads, fixed-point summation. */
int dpsnn_default_config(dpsnn_config *cfg);

/* Device bytes that dpsnn_build_network would allocate for *cfg, without
 * allocating: the network arrays of the construction phase (Sec. 2, "Initial
 * construction of the connectivity infrastructure": forward synapse lists of
 * every neuron, the incoming-synapse index, neuron state), the STDP tables,
 * the network's launch tables, and the bounded scratch of one read-back
 * (dpsnn_read_weights / dpsnn_read_connectivity).  A checkpoint save or load
 * takes a further transient buffer (see dpsnn_save).  DPSNN_E_INVAL if *cfg
 * is invalid. */
int dpsnn_footprint_bytes(const dpsnn_config *cfg, uint64_t *bytes);

/* Generate the network on the device (Sec. 2, "Initial construction of the
 * connectivity infrastructure" and "Distributed generation of reproducible
 * connections"): every synapse is drawn from a counter-based generator keyed
 * by (seed) with counter (id, j), so the network does not depend on launch
 * shapes.  On success *out owns all device state; the call returns after the
 * build has completed on the stream.  Size limits (DPSNN_E_INVAL beyond
 * them): fewer than 2^26 neurons, fewer than 2^36 synapses (2^32 with
 * DPSNN_SUM_ORDERED), and 13 x neurons_per_column x synapses_per_neuron
 * below 2^31.  The build sorts each reverse row of up to 8192 entries by
 * source, so the device layout is deterministic; results never depend on
 * it. */
int dpsnn_build_network(const dpsnn_config *cfg, const dpsnn_device *dev, dpsnn_net **out);

/* Enqueue n_steps 1 ms steps (Sec. 2, loop items 2.1-2.7, plus the periodic
 * consolidation).  Asynchronous on the network's stream, except that the
 * call waits when it gets more than about 16 steps ahead of the device (the
 * automatic launch shapes follow a measured event rate at most that stale).
 * Runs of G steps (dpsnn_set_tuning key 8, default 8) that hold no
 * consolidation and not the first step are enqueued as one replay of a HIP
 * graph captured for that run length and the current launch shapes (captured
 * again when either changes); with timing enabled every step is launched
 * directly.  The results are the same either way. */
int dpsnn_step(dpsnn_net *net, uint32_t n_steps);

/* Wait for all enqueued work of the network: every step enqueued so far has
 * completed (the end of the paper's per-step loop, Sec. 2, items 2.1-2.7). */
int dpsnn_sync(dpsnn_net *net);

/* Steps completed so far (the next step index). */
int dpsnn_time(dpsnn_net *net, uint32_t *t);

/* The spike list observable (Sec. 2, "Production of observables": times and
 * ids of the spikes): spikes with stamp in [t_begin, t_end), sorted by
 * (stamp, id), written to times[] and ids[] (each of capacity cap).  *n_out
 * receives the number of spikes.  DPSNN_E_RANGE if the range reaches past
 * the last step or before the retained raster window; DPSNN_E_BUFSZ if cap
 * is too small (*n_out then holds the count needed).  No device memory is
 * allocated. */
int dpsnn_read_spikes(dpsnn_net *net, uint32_t t_begin, uint32_t t_end,
                      uint32_t *times, uint32_t *ids, size_t cap, size_t *n_out);

/* The synaptic-value observable (Sec. 2, "Production of observables"; STDP
 * rule of Sec. 2): for canonical synapses [first, first + count), weight w,
 * potentiation accumulator P and depression accumulator D (the synaptic
 * derivative is P - D), written to the caller's host arrays in canonical
 * order.  Any output pointer may be NULL.  DPSNN_E_RANGE if the range passes
 * the last synapse.  The call allocates one transient device scratch through
 * the network's allocator (the dpsnn_device callbacks, else hipMalloc) and
 * frees it before returning: staging of at most 8 MiB and, when P is asked
 * for, P of whole source columns (at most 32 MiB, at least one column's
 * neurons_per_column x synapses_per_neuron floats); it scales with the
 * columns the range spans, not with the network.  DPSNN_E_NOMEM if that
 * allocation fails. */
int dpsnn_read_weights(dpsnn_net *net, uint64_t first, uint64_t count,
                       float *w, float *P, float *D);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * same read as dpsnn_read_weights, with the same results, but its scratch is
 * a library-owned static device workspace of DPSNN_NOALLOC_SCRATCH_BYTES on
 * each GPU (held until the process ends) instead of an allocation; the call
 * allocates no device memory.  DPSNN_E_INVAL if one source column's P
 * (neurons_per_column x synapses_per_neuron x 4 bytes) plus one row of
 * staging does not fit the workspace.  Every call on one GPU uses that GPU's
 * workspace, which keeps the last call's contents (nothing in it needs to
 * start at zero): calls that overlap in time on the same GPU, from several
 * host threads, race and must be serialised by the caller. */
#define DPSNN_NOALLOC_SCRATCH_BYTES (32u << 20)
int dpsnn_read_weights_noalloc(dpsnn_net *net, uint64_t first, uint64_t count,
                               float *w, float *P, float *D);

/* The connectivity observable (Sec. 2, "Projection of synapses": each
 * synapse's target and axonal delay) of canonical synapses [first, first +
 * count): global target id and delay in ms, in canonical order.  Either
 * pointer may be NULL.  Transient staging of at most 8 MiB through the
 * network's allocator, as dpsnn_read_weights. */
int dpsnn_read_connectivity(dpsnn_net *net, uint64_t first, uint64_t count,
                            uint32_t *target, uint8_t *delay);

/* Membrane potential v and recovery variable u of every neuron (Sec. 2,
 * observables); arrays of length grid_x*grid_y*neurons_per_column. */
int dpsnn_read_state(dpsnn_net *net, float *v, float *u);

/* Counters and per-block timers (Sec. 3, Table 2's per-block profiling;
 * "Production of observables" for the spike count): steps, spikes, delivered
 * events, LTP visits, consolidations, and the per-kernel device time
 * accumulated while dpsnn_set_timing is on.  Synchronises the stream. */
int dpsnn_get_stats(dpsnn_net *net, dpsnn_stats *stats);

/* External stimulus (test hook): entry e adds mv[e] to the input current of
 * neuron id[e] in step t[e], after the thalamic input.  Replaces any previous
 * list.  n may be 0 to clear. */
int dpsnn_set_stimulus(dpsnn_net *net, const uint32_t *t, const uint32_t *id,
                       const float *mv, size_t n);

/* State probes (Sec. 2, "Production of observables": the trace of the
 * membrane potential and other state variables of individual neurons can be
 * activated).  After every later step the library records v and u of the
 * `count` neurons ids[0..count) on the device (a ring of raster_steps rows).
 * Replaces any previous probe set; count = 0 removes it.  At most 65536
 * probes; DPSNN_E_INVAL for an id out of range or a network in a batch.
 * The probe buffers (2 x count x raster_steps floats) come from the
 * network's allocator. */
int dpsnn_set_probes(dpsnn_net *net, const uint32_t *ids, uint32_t count);
/* Probed state after steps s in [t_begin, t_end) (s = number of steps
 * completed, as spike stamps): v[(s - t_begin) * count + p] and likewise u,
 * for probe p in the order given to dpsnn_set_probes.  Either pointer may be
 * NULL.  DPSNN_E_RANGE for steps not recorded (before the probes were set,
 * past the last step, or older than raster_steps). */
int dpsnn_read_probes(dpsnn_net *net, uint32_t t_begin, uint32_t t_end, float *v, float *u);

/* Per-kernel device timers (Table 2's per-block profiling): when enabled,
 * every kernel launch of dpsnn_step is bracketed by events and its duration
 * accumulated into dpsnn_stats at the next dpsnn_get_stats. */
int dpsnn_set_timing(dpsnn_net *net, int enable);

/* Launch-shape knobs (results never depend on them).  "Automatic" values
 * (the defaults) follow the measured regime of the launch: a launch is
 * sparse when its source columns deliver fewer events per step than their
 * current window has entries (with hysteresis: sparse below 0.8 of that,
 * dense above it) and it has enough work to fill the GPU with small
 * workgroups: at least 2048 columns, or at least 64 columns whose column
 * parts (key 5) give at least 512 workgroups; every other launch is dense.
 *   key 0: delivery workgroup size 256, 512, 1024; 0 = automatic (256 / 1024)
 *   key 1: LTP workgroup size 256, 512, 1024; 0 = automatic (256 / 1024)
 *   key 2: LDS current window in delivery: 1 = over all 13 reachable
 *          columns, 2 = a partial window (the own column and the nearest
 *          slots, key 10), 0 = off; 3 = automatic (2 / 1); a window that does
 *          not fit in LDS falls back to 2, then 0
 *   key 3: delivery unroll U = 1, 2, 4 or 8 (default 4): each lane keeps
 *          max(1, U / 2) quads of 4 consecutive synapses in flight
 *   key 4: LDS copy of the targets' spike ages in delivery: 1 on, 0 off,
 *          2 = automatic (off / on)
 *   key 5: workgroups per column in delivery and LTP: 0 = automatic (sets of
 *          fewer than 512 columns split each column's work), 1 .. 1024 = that
 *          many; summation mode ORDERED always 1
 *   key 6: LDS copy of the sources' spike history in LTP: 1 allowed, 0 off,
 *          2 = automatic (off / allowed)
 *   key 7: LTP and delivery run as one kernel when each launch has at most
 *          this many workgroups and both use the same workgroup size
 *          (default 2^32 - 1, i.e. always; 0 = never)
 *   key 8: steps per captured graph G, 0 .. 1024 (default 8; 0 = every step
 *          launched directly)
 *   key 9: with the full window (key 2 = 1), workgroups that share one
 *          source column's window by target slot, 1 .. 13 (default 1): each
 *          reads all the column's events and delivers those whose target it
 *          owns; a smaller LDS window per workgroup for latency-bound
 *          networks with few columns
 *   key 10: slots of the partial window (key 2 = 2), 1 .. 13: the own column
 *          first, then the nearest neighbour slots; events to other slots
 *          take global atomics; 0 = automatic (3 / 1)
 *   key 11: wavefront-level LTP for sparse columns (the spiking neurons of
 *          a wavefront's raster words gathered into its lanes, their reverse
 *          rows spread over the lanes a quad at a time, the own column's
 *          spike history in LDS when key 6 allows): 0 off, 1 on,
 *          2 = automatic (on / off)
 *   key 12: wavefront-level delivery for sparse columns (one excitatory
 *          (source, delay) segment per lane, two inhibitory spikes per
 *          wavefront at a time, 256-thread workgroups with the key 10 window;
 *          LTP then also by key 11's body): 0 off, 1 on, 2 = automatic
 *          (off: measured slower than the run-based path); not used with
 *          DPSNN_SUM_ORDERED
 *   key 13: target columns per workgroup of the key 11 LTP, 1 .. 8, for
 *          single networks with unsplit columns (key 5): a workgroup's time is
 *          set by its chain of dependent loads more than by its work, so
 *          fewer workgroups with more columns finish sooner; 0 = automatic
 *   key 14: consolidation (Sec. 3, Table 2, "long term synaptic
 *          plasticity"): 1 (default) one pass in forward order through the
 *          network's forward-to-reverse map, kept when 13 x
 *          neurons_per_column x synapses_per_neuron <= 2^28; 0 two passes
 *          (reverse, then forward order), the form used without the map
 * (sparse / dense choice in parentheses) */
int dpsnn_set_tuning(dpsnn_net *net, uint32_t key, uint32_t value);

/* Online autotuner of the launch shapes (the knobs of dpsnn_set_tuning):
 * steps the network steps_per_trial steps under each candidate shape, in two
 * interleaved rounds, and keeps the fastest: with LTP and delivery fused (key
 * 7, the default) one workgroup size for both plus the delivery unroll, by
 * their combined time; otherwise the delivery and LTP shapes separately.  The
 * network advances by those steps; its results do not depend on the shapes. */
int dpsnn_autotune(dpsnn_net *net, uint32_t steps_per_trial);

/* The network's configuration (raster_steps as resolved at build). */
int dpsnn_get_config(dpsnn_net *net, dpsnn_config *cfg);

/* ---- Checkpoints ------------------------------------------------------
 * A checkpoint holds the configuration and the dynamic state after the last
 * completed step: v, u, spike history, latest spike stamps, the raster ring,
 * w, P, D, the stimulus list, the clock and the counters (the paper warms a
 * network for 8 s before measuring; a checkpoint skips that).  Connectivity
 * is not stored: dpsnn_load regenerates it from the seed, exactly as the
 * build drew it.  A loaded network continues bit for bit as the saved one
 * would have in the reproducible summation modes.  Launch shapes, timers and
 * the regime estimate are not stored. */

/* Bytes dpsnn_save writes for this network. */
int dpsnn_checkpoint_bytes(dpsnn_net *net, uint64_t *bytes);
/* Write the checkpoint into the caller's host buffer buf of cap bytes
 * (DPSNN_E_BUFSZ if too small); waits for the network's stream.  P moves to
 * the forward layout through a transient device buffer from the network's
 * allocator: at most 1 GiB (all columns when they fit), halved on allocation
 * failure down to one column; DPSNN_E_NOMEM if even that fails.  dpsnn_load
 * takes the same buffer. */
int dpsnn_save(dpsnn_net *net, void *buf, uint64_t cap);
/* Build a network on *dev from a checkpoint of `size` bytes (as written by
 * dpsnn_save) and restore its state; DPSNN_E_INVAL if buf is not a whole,
 * consistent checkpoint of this format: header, configuration, total size
 * and raster (no spike bit beyond a column's last neuron) are checked on the
 * host before any device work.  *out is owned by the caller. */
int dpsnn_load(const void *buf, uint64_t size, const dpsnn_device *dev, dpsnn_net **out);

void dpsnn_destroy(dpsnn_net *net);

/* ---- Batches: many independent networks advanced together ----------------
 * A batch steps several networks (of any grid size, M, seed and thalamic
 * rate) with one launch per kernel: every workgroup looks up its network and
 * column in a device table.  Each network's results are exactly those of its
 * own run (the draws are keyed by the network's seed and global ids).
 * Members must share the device and stream, use DPSNN_SUM_FIXED or
 * DPSNN_SUM_ATOMIC (all the same) and the same target-index width (13 x
 * neurons_per_column <= 65536 for all or for none).  While in a batch a
 * network is stepped only through it; its read_* calls work as usual. */
typedef struct dpsnn_batch dpsnn_batch;

int dpsnn_batch_create(dpsnn_net *const *nets, uint32_t n_nets, dpsnn_batch **out);
/* n_steps steps of every member, graphed like dpsnn_step (one graph holds the
 * whole batch's kernels for G steps). */
int dpsnn_batch_step(dpsnn_batch *batch, uint32_t n_steps);
/* Sums of the members' counters; per-kernel timers of the batch's launches. */
int dpsnn_batch_get_stats(dpsnn_batch *batch, dpsnn_stats *stats);
int dpsnn_batch_set_timing(dpsnn_batch *batch, int enable);
int dpsnn_batch_set_tuning(dpsnn_batch *batch, uint32_t key, uint32_t value);
int dpsnn_batch_autotune(dpsnn_batch *batch, uint32_t steps_per_trial);
/* Releases the batch's tables; the member networks stay valid and can be
 * stepped alone again. */
void dpsnn_batch_destroy(dpsnn_batch *batch);

/* ---- Serving: a continuous-batching job server -------------------------
 * A job is a network configuration plus a number of steps; its result is the
 * network after those steps, exactly as dpsnn_build_network + dpsnn_step
 * would leave it (every draw is keyed by the job's seed and global ids).
 * A server runs jobs on one device with two threads of its own:
 *   - the builder admits queued jobs strictly in submission order while the
 *     admitted jobs' footprints (dpsnn_footprint_bytes) fit the byte budget
 *     and fewer than max_jobs are admitted, and generates each job's network
 *     on the server's build stream;
 *   - the stepper advances every built job on the server's step stream in
 *     quanta of at most max_quantum steps (a quantum also ends where the
 *     first running job finishes): jobs sharing the summation mode and the
 *     target-index width step together with one launch per kernel, each
 *     DPSNN_SUM_ORDERED job alone.  Built jobs join, and finished jobs leave,
 *     between quanta; the host stays at most one quantum ahead of the device.
 * A job is DONE when its last step has completed on the device.  Its network
 * then stays on the device, owned by the server, for the read_* calls and
 * dpsnn_get_stats (which use the server's read stream; dpsnn_step also works
 * on it), and its footprint stays reserved until dpsnn_server_release.
 * dpsnn_destroy refuses such a network.
 * The device's alloc/free callbacks (thread-safe; called from the server's
 * threads and from dpsnn_server_release) serve every device allocation of the
 * jobs; without callbacks the server allocates with hipMallocAsync and frees
 * with hipFreeAsync on its own streams.  Its stream field is ignored.
 * All entry points may be called from any host thread. */
typedef struct dpsnn_server dpsnn_server;

#define DPSNN_JOB_QUEUED  0   /* submitted, not admitted yet */
#define DPSNN_JOB_RUNNING 1   /* admitted: being built or stepped */
#define DPSNN_JOB_DONE    2   /* all steps completed; results readable */
#define DPSNN_JOB_FAILED  3   /* build or step failed, or the server shut down */

typedef struct dpsnn_job_info {
    uint64_t   id;
    int32_t    status;           /* DPSNN_JOB_* */
    int32_t    error;            /* DPSNN_E_* code when FAILED, else 0 */
    uint32_t   steps;            /* steps requested */
    uint32_t   steps_launched;   /* steps enqueued on the device so far */
    uint64_t   footprint;        /* device bytes reserved for the job */
    /* seconds on the server clock (dpsnn_server_clock); 0 = not reached */
    double     t_submit, t_admit, t_built, t_done;
    dpsnn_net *net;              /* the job's network once DONE, else NULL */
    char       message[160];     /* failure message when FAILED */
} dpsnn_job_info;

typedef struct dpsnn_server_stats {
    uint64_t submitted, completed, failed, released;
    uint64_t queued, running;        /* jobs in each state now */
    uint64_t quanta;                 /* quanta launched by the stepper */
    uint64_t set_steps;              /* launches of one step over one job group */
    uint64_t job_steps;              /* steps launched, summed over jobs */
    uint64_t budget_bytes, reserved_bytes, peak_reserved_bytes;
    uint64_t peak_running;           /* most jobs admitted at once */
} dpsnn_server_stats;

/* budget_bytes = 0 takes 90 % of the device memory free at creation.
 * max_quantum: steps per quantum (0 = 8).  max_jobs: jobs admitted at once
 * (0 = 256). */
int dpsnn_server_create(const dpsnn_device *dev, uint64_t budget_bytes, uint32_t max_quantum,
                        uint32_t max_jobs, dpsnn_server **out);
/* Queue a job of `steps` steps (1 .. 2^20 - 1).  If cfg->raster_steps is 0
 * the job keeps the raster of its whole run (raster_steps = steps + 1).
 * DPSNN_E_INVAL for an invalid configuration, DPSNN_E_NOMEM if its footprint
 * exceeds the whole budget.  Never blocks on device work. */
int dpsnn_server_submit(dpsnn_server *srv, const dpsnn_config *cfg, uint32_t steps,
                        uint64_t *job);
/* Current state of a job; DPSNN_E_INVAL for an unknown or released id. */
int dpsnn_server_query(dpsnn_server *srv, uint64_t job, dpsnn_job_info *info);
/* Block until the job is DONE or FAILED (timeout_s < 0: no limit), then
 * fill *info.  DPSNN_E_TIMEOUT (with *info filled) if the time ran out.  A
 * job this call returns as DONE or FAILED counts as collected:
 * dpsnn_server_wait_any does not return it. */
int dpsnn_server_wait(dpsnn_server *srv, uint64_t job, double timeout_s, dpsnn_job_info *info);
/* Block until some job finishes that no earlier dpsnn_server_wait_any or
 * dpsnn_server_wait call returned; jobs are returned in the order they
 * finished.  DPSNN_E_TIMEOUT if none finished in time. */
int dpsnn_server_wait_any(dpsnn_server *srv, double timeout_s, dpsnn_job_info *info);
/* Cancel a QUEUED or RUNNING job; returns at once.  A queued job becomes
 * FAILED (error DPSNN_E_CANCELED) immediately; a job being built or stepped
 * becomes FAILED (DPSNN_E_CANCELED) once no launched work uses its network:
 * after its build, or after the quantum in flight at the call (it may
 * advance by that quantum).  The other jobs' results are unchanged.  Its
 * network and footprint are then freed by dpsnn_server_release, as for any
 * finished job.  DPSNN_E_INVAL for an unknown, released or finished job. */
int dpsnn_server_cancel(dpsnn_server *srv, uint64_t job);
/* Free a DONE or FAILED job's network and return its footprint to the
 * budget.  DPSNN_E_INVAL if the job is still queued or running, or if its
 * network belongs to a batch. */
int dpsnn_server_release(dpsnn_server *srv, uint64_t job);
int dpsnn_server_get_stats(dpsnn_server *srv, dpsnn_server_stats *stats);
/* Seconds since the server was created (steady clock). */
int dpsnn_server_clock(dpsnn_server *srv, double *seconds);
/* Stop both threads after the quanta already launched, mark jobs that were
 * still queued or running FAILED, and free every job's network.  No other
 * call on the server may be in progress or follow. */
void dpsnn_server_destroy(dpsnn_server *srv);

/* Message of the last failure on the calling thread ("" if none). */
const char *dpsnn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DPSNN_H */
