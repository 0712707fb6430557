/*
 * Reference CPU simulator ("the oracle") for the DPSNN-STDP 1 ms step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so the tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU library against a plain,
 * slow, obviously correct implementation.  It shares no code, header, table
 * or constant generator with the GPU library.
 *
 * Paper: Paolucci et al., "Distributed simulation of polychronous and plastic
 * spiking neural networks: strong and weak scaling of a representative
 * mini-application benchmark executed on a small-scale commodity cluster"
 * (arXiv 1310.8478).  Citations name the paper's sections, equations and
 * tables.
 *
 * Everything here is single-threaded C99, fp32 state with no contraction
 * (build with -ffp-contract=off, no fast-math, round-to-nearest, no FTZ).
 * Where the paper is silent the reading taken is stated at the point of use;
 * the same list of readings is kept with the design notes of the project.
 *
 * Parity status per function (what pins it in the CPU test suite):
 *   orc_philox            pinned: published known-answer vectors (Salmon et al.)
 *   synapse generation    pinned: exact structural invariants + chi-square
 *   thalamic picks        pinned: exact counts + chi-square uniformity
 *   neuron update         pinned: closed-form fixed points, saddle-node bound,
 *                                 1 us fp64 Euler regime comparison
 *   delivery / currents   pinned: independent dense brute-force simulator,
 *                                 hand-traced chains, event-count invariant,
 *                                 exact rational sum (fixed-point mode)
 *   STDP LTP / LTD        pinned: post-hoc pair checker from raster alone,
 *                                 hand-computed table values
 *   weight consolidation  pinned: post-hoc recomputation + range invariants;
 *                         the rule's constants are a reading (parity of the
 *                         rule itself against the paper is unpinned: the
 *                         paper names the block but gives no formula).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <float.h>

/* ------------------------------------------------------------------------- */
/* Configuration (own definition; mirrors the fields of the public C ABI but  */
/* is declared independently so that the oracle shares no header with it).   */
/* ------------------------------------------------------------------------- */
typedef struct {
    uint32_t grid_x, grid_y;          /* column grid CFX x CFY (Sec. 2, "reproducible connections") */
    uint32_t neurons_per_column;      /* 1000 in the paper, 1250 in the measured workloads */
    float    exc_fraction;            /* 0.8: 80 % RS / 20 % FS (Sec. 2, neuron model) */
    uint32_t synapses_per_neuron;     /* M (Sec. 2, projection of synapses) */
    uint32_t conn_mode;               /* 0: own_fraction + uniform over 12 neighbours; 1: 76/3/2/1 % quotas */
    float    own_fraction;
    uint32_t max_delay;               /* 20 ms (Sec. 2, projection of synapses) */
    float    w_exc_init, w_inh, w_max;
    float    a_plus, a_minus, tau_plus, tau_minus;   /* STDP rule, Sec. 2 */
    uint32_t weight_update_period;    /* steps between consolidations */
    float    wu_bias, sd_decay;       /* consolidation constants (reading) */
    float    thalamic_rate;           /* events per column per ms (Sec. 2) */
    float    thalamic_current;        /* mV per thalamic event */
    uint64_t seed;
    uint32_t sum_mode;                /* 0: ordered fp32 left fold; 2: fixed-point int64 */
} orc_config;

#define ORC_SUM_ORDERED 0u
#define ORC_SUM_FIXED   2u

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator, written from its published          */
/* definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy  */
/* as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with      */
/* multipliers 0xD2511F53 and 0xCD9E8D57, and a Weyl key schedule with        */
/* increments 0x9E3779B9 and 0xBB67AE85 applied between rounds.              */
/* ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Map a uniform 32-bit word to [0, n): floor(x * n / 2^32). */
static uint32_t mulhi_range(uint32_t x, uint32_t n)
{
    return (uint32_t)(((uint64_t)x * (uint64_t)n) >> 32);
}

#define TAG_SYN  0x53594E00u   /* counter word 2 for synapse draws */
#define TAG_THAL 0x5448414Cu   /* counter word 2 for thalamic draws */
#define ORC_MAX_THAL 1024u     /* thalamic events per column per ms (rate < 1024) */

static void draw(const orc_config *cfg, uint32_t w0, uint32_t w1, uint32_t tag, uint32_t w3,
                 uint32_t out[4])
{
    uint32_t ctr[4] = { w0, w1, tag, w3 };
    uint32_t key[2] = { (uint32_t)(cfg->seed & 0xFFFFFFFFu), (uint32_t)(cfg->seed >> 32) };
    orc_philox(ctr, key, out);
}

/* ------------------------------------------------------------------------- */
/* Derived sizes.                                                             */
/* ------------------------------------------------------------------------- */
static uint32_t exc_per_column(const orc_config *cfg)
{
    /* 80 % excitatory (Sec. 2, neuron model): round(exc_fraction * Ncol). */
    return (uint32_t)floor((double)cfg->exc_fraction * (double)cfg->neurons_per_column + 0.5);
}

static uint32_t own_quota(const orc_config *cfg)
{
    return (uint32_t)floor((double)cfg->own_fraction * (double)cfg->synapses_per_neuron + 0.5);
}

/* Neighbour rings of the column grid (Sec. 2, "Bidimensional arrays of neural
 * columns"): read as the square-lattice first, second and third nearest
 * neighbours, four of each (distance 1, sqrt 2, 2). */
static const int RING_DX[12] = { 1, -1, 0,  0,  1, -1,  1, -1,  2, -2, 0,  0 };
static const int RING_DY[12] = { 0,  0, 1, -1,  1,  1, -1, -1,  0,  0, 2, -2 };

/* Paper-mode quotas in units of 1/10000: 76 % own column, 3 % to each of the
 * four first neighbours, 2 % to each second and 1 % to each third neighbour
 * (Sec. 3, text after Table 1).  Slot 0 is the own column, slot s>0 is ring
 * offset s-1. */
static const uint32_t PAPER_QUOTA[13] = { 7600, 300, 300, 300, 300, 200, 200, 200, 200,
                                          100, 100, 100, 100 };

/* Largest-remainder apportionment of M synapses over the 13 slots; ties in
 * the remainder go to the lower slot index. */
static void paper_blocks(uint32_t M, uint32_t count[13])
{
    uint64_t rem[13];
    uint32_t used = 0;
    for (int s = 0; s < 13; ++s) {
        uint64_t prod = (uint64_t)PAPER_QUOTA[s] * M;
        count[s] = (uint32_t)(prod / 10000u);
        rem[s] = prod % 10000u;
        used += count[s];
    }
    while (used < M) {
        int best = 0;
        for (int s = 1; s < 13; ++s) if (rem[s] > rem[best]) best = s;
        count[best] += 1; rem[best] = 0; used += 1;
    }
}

static int wrap(int x, int n) { int r = x % n; return r < 0 ? r + n : r; }

/* One synapse (i, j) by definition (Sec. 2, "Projection of synapses" and
 * "Bidimensional arrays"): returns target neuron, delay and initial weight. */
void orc_synapse(const orc_config *cfg, uint32_t i, uint32_t j,
                 uint32_t *tgt, uint32_t *delay, float *w0)
{
    const uint32_t Ncol = cfg->neurons_per_column;
    const uint32_t Ne = exc_per_column(cfg);
    const uint32_t c = i / Ncol, l = i % Ncol;
    const int cx = (int)(c % cfg->grid_x), cy = (int)(c / cfg->grid_x);
    uint32_t x[4];
    draw(cfg, i, j, TAG_SYN, 0u, x);

    if (l >= Ne) {
        /* Inhibitory: excitatory neurons of the own column only, minimum delay. */
        *tgt = c * Ncol + mulhi_range(x[1], Ne);
        *delay = 1u;
        *w0 = cfg->w_inh;
        return;
    }
    int slot; /* 0 = own column, 1..12 = ring offset slot-1 */
    if (cfg->conn_mode == 1u) {
        uint32_t cnt[13];
        paper_blocks(cfg->synapses_per_neuron, cnt);
        uint32_t acc = 0; slot = 12;
        for (int s = 0; s < 13; ++s) { acc += cnt[s]; if (j < acc) { slot = s; break; } }
    } else {
        slot = (j < own_quota(cfg)) ? 0 : 1 + (int)mulhi_range(x[0], 12u);
    }
    int tx = cx, ty = cy;
    if (slot > 0) {
        tx = wrap(cx + RING_DX[slot - 1], (int)cfg->grid_x);
        ty = wrap(cy + RING_DY[slot - 1], (int)cfg->grid_y);
    }
    uint32_t tc = (uint32_t)ty * cfg->grid_x + (uint32_t)tx;
    uint32_t lt;
    if (tc == c) {
        /* own column (also when a wrapped neighbour lands on it): never self */
        uint32_t r = mulhi_range(x[1], Ncol - 1u);
        lt = r + (r >= l ? 1u : 0u);
    } else {
        lt = mulhi_range(x[1], Ncol);
    }
    *tgt = tc * Ncol + lt;
    *delay = 1u + mulhi_range(x[2], cfg->max_delay);
    *w0 = cfg->w_exc_init;
}

/* Thalamic picks of column c in step t (Sec. 2, "reproducible ... thalamic
 * stimulus": a prescribed number of events per ms per column).  The count is
 * floor(r) plus one Bernoulli(frac r) draw; each pick is a uniform neuron of
 * the column.  Writes up to cap local indices, returns the count. */
uint32_t orc_thalamic(const orc_config *cfg, uint32_t c, uint32_t t, uint32_t *picks, uint32_t cap)
{
    const double r = (double)cfg->thalamic_rate;
    const double fl = floor(r);
    const uint32_t whole = (uint32_t)fl;
    const uint32_t thr = (uint32_t)((r - fl) * 4294967296.0);
    uint32_t y[4];
    draw(cfg, c, t, TAG_THAL, 0u, y);
    uint32_t n = whole + (y[0] < thr ? 1u : 0u);
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t call = k / 3u, word = 1u + k % 3u;
        uint32_t z[4];
        draw(cfg, c, t, TAG_THAL, call, z);
        if (k < cap) picks[k] = mulhi_range(z[word], cfg->neurons_per_column);
    }
    return n;
}

/* STDP table values (Sec. 2, STDP equation): evaluated in fp64, rounded once
 * to fp32; values below FLT_MIN are flushed to 0 (reading). */
float orc_tp(const orc_config *cfg, uint32_t delta)
{
    double v = (double)cfg->a_plus * exp(-(double)delta / (double)cfg->tau_plus);
    float f = (float)v;
    return (fabsf(f) < FLT_MIN) ? 0.0f : f;
}

float orc_tm(const orc_config *cfg, uint32_t delta)
{
    double v = (double)cfg->a_minus * exp(-(double)delta / (double)cfg->tau_minus);
    float f = (float)v;
    return (fabsf(f) < FLT_MIN) ? 0.0f : f;
}

/* Fixed-point quantisation of a current contribution: x * 2^32 rounded to the
 * nearest integer (ties to even).  The current is then the fp32 value nearest
 * to the exact fixed-point sum (reading: the paper fixes no summation order
 * or precision for the total incoming current). */
static int64_t q32(float x)
{
    float s = x * 4294967296.0f;     /* exact power-of-two scaling */
    return (int64_t)llrintf(s);
}

static float dq32(int64_t a)
{
    float f = (float)a;              /* one rounding, to nearest */
    return f * (1.0f / 4294967296.0f);
}

/* ------------------------------------------------------------------------- */
/* Izhikevich neuron, one 1 ms step (Sec. 2 neuron model; Sec. 3: v is         */
/* integrated with two 0.5 ms sub-steps).  The printed recovery equation        */
/* reads a(bv - c); the reading here is a(bv - u), the form of the cited        */
/* Izhikevich (2003) model, which is the only one with the resting state the   */
/* paper describes.  u is advanced once per ms with the new v.  Returns 1 if   */
/* the neuron fired (v >= v_peak = 30), after applying the reset.              */
/* ------------------------------------------------------------------------- */
int orc_neuron_step(float *vp, float *up, float I, float a, float b, float c, float d)
{
    float v = *vp, u = *up;
    for (int h = 0; h < 2; ++h) {
        float e = 0.04f * v;
        e = e * v;
        e = e + 5.0f * v;
        e = e + 140.0f;
        e = e - u;
        e = e + I;
        v = v + 0.5f * e;
    }
    float bv = b * v;
    u = u + a * (bv - u);
    int fired = 0;
    if (v >= 30.0f) { v = c; u = u + d; fired = 1; }
    *vp = v; *up = u;
    return fired;
}

static void neuron_params(uint32_t l, uint32_t Ne, float *a, float *b, float *c, float *d)
{
    if (l < Ne) { *a = 0.02f; *b = 0.2f; *c = -65.0f; *d = 8.0f; }   /* RS */
    else        { *a = 0.1f;  *b = 0.2f; *c = -65.0f; *d = 2.0f; }   /* FS */
}

/* Single neuron under a constant input, for closed-form checks: runs T steps
 * from v = -65, u = b v and writes the step index (1-based stamp) of every
 * spike into stamps (up to cap); returns the spike count. Final v, u out. */
uint32_t orc_single_neuron(int fs, float I, uint32_t T, uint32_t *stamps, uint32_t cap,
                           float *v_out, float *u_out)
{
    float a, b, c, d;
    neuron_params(fs ? 1u : 0u, 1u, &a, &b, &c, &d);
    float v = -65.0f, u = b * v;
    uint32_t n = 0;
    for (uint32_t t = 0; t < T; ++t) {
        if (orc_neuron_step(&v, &u, I, a, b, c, d)) {
            if (n < cap) stamps[n] = t + 1u;
            ++n;
        }
    }
    *v_out = v; *u_out = u;
    return n;
}

/* ------------------------------------------------------------------------- */
/* Network state.                                                             */
/* ------------------------------------------------------------------------- */
typedef struct { int32_t *s; uint32_t n, cap; } stamp_list;

typedef struct {
    uint32_t t; uint32_t id; float mv;
} stim_entry;

typedef struct orc_net {
    orc_config cfg;
    uint32_t N, Ncol, Ne, M, Dmax, C;
    /* synapses in canonical (i, j) order */
    uint32_t *tgt; uint8_t *dly; float *w, *P, *D;
    /* per neuron, its j indices ordered by (delay, j): dord[i*M + r]; the
     * block of delay d is [dptr[i*(Dmax+1)+d-1], dptr[i*(Dmax+1)+d]) */
    uint32_t *dord; uint32_t *dptr;
    /* incoming excitatory synapses per neuron (global index i*M+j) */
    uint64_t *in_ptr; uint64_t *in_syn;
    /* neuron state */
    float *v, *u, *accf; int64_t *acci;
    stamp_list *hist;
    /* raster: ids in stamp order, ascending id within a stamp */
    uint32_t *r_id; uint32_t *r_t; uint64_t r_n, r_cap;
    uint64_t *step_start;     /* step_start[s] = first raster row with stamp s; size T_cap+2 */
    uint32_t T_cap;
    uint32_t t;               /* next step to run */
    /* stimulus list */
    stim_entry *stim; uint64_t n_stim;
    /* counters */
    uint64_t n_events, n_ltp_visits, n_ltp_updates, n_ltd_updates, n_spikes, n_thal;
} orc_net;

static void *xcalloc(size_t n, size_t sz) { return n ? calloc(n, sz) : NULL; }

void orc_destroy(orc_net *net);

/* Build the network (Sec. 2 "Initial construction"): every synapse is drawn
 * by definition; the per-delay ordering and the incoming lists are plain
 * index structures over the canonical arrays. T_cap bounds the number of
 * steps that can be simulated (size of the stamp index). */
orc_net *orc_create(const orc_config *cfg, uint32_t T_cap)
{
    orc_net *net = (orc_net *)calloc(1, sizeof(orc_net));
    if (!net) return NULL;
    net->cfg = *cfg;
    net->Ncol = cfg->neurons_per_column;
    net->C = cfg->grid_x * cfg->grid_y;
    net->N = net->C * net->Ncol;
    net->Ne = exc_per_column(cfg);
    net->M = cfg->synapses_per_neuron;
    net->Dmax = cfg->max_delay;
    net->T_cap = T_cap;
    const uint64_t S = (uint64_t)net->N * net->M;
    const uint32_t N = net->N, M = net->M, Dmax = net->Dmax;

    net->tgt = (uint32_t *)xcalloc(S, sizeof(uint32_t));
    net->dly = (uint8_t *)xcalloc(S, 1);
    net->w = (float *)xcalloc(S, sizeof(float));
    net->P = (float *)xcalloc(S, sizeof(float));
    net->D = (float *)xcalloc(S, sizeof(float));
    net->dord = (uint32_t *)xcalloc(S, sizeof(uint32_t));
    net->dptr = (uint32_t *)xcalloc((uint64_t)N * (Dmax + 1), sizeof(uint32_t));
    net->in_ptr = (uint64_t *)xcalloc((uint64_t)N + 1, sizeof(uint64_t));
    net->v = (float *)xcalloc(N, sizeof(float));
    net->u = (float *)xcalloc(N, sizeof(float));
    net->accf = (float *)xcalloc(N, sizeof(float));
    net->acci = (int64_t *)xcalloc(N, sizeof(int64_t));
    net->hist = (stamp_list *)xcalloc(N, sizeof(stamp_list));
    net->step_start = (uint64_t *)xcalloc((uint64_t)T_cap + 2, sizeof(uint64_t));
    if (!net->tgt || !net->dly || !net->w || !net->P || !net->D || !net->dord || !net->dptr ||
        !net->in_ptr || !net->v || !net->u || !net->accf || !net->acci || !net->hist ||
        !net->step_start) { orc_destroy(net); return NULL; }

    for (uint32_t i = 0; i < N; ++i) {
        for (uint32_t j = 0; j < M; ++j) {
            uint32_t tg, d; float w0;
            orc_synapse(cfg, i, j, &tg, &d, &w0);
            uint64_t g = (uint64_t)i * M + j;
            net->tgt[g] = tg; net->dly[g] = (uint8_t)d; net->w[g] = w0;
        }
        /* stable ordering of j by delay */
        uint32_t *ptr = net->dptr + (uint64_t)i * (Dmax + 1);
        ptr[0] = 0;
        uint32_t r = 0;
        for (uint32_t d = 1; d <= Dmax; ++d) {
            for (uint32_t j = 0; j < M; ++j)
                if (net->dly[(uint64_t)i * M + j] == d) net->dord[(uint64_t)i * M + r++] = j;
            ptr[d] = r;
        }
    }
    /* incoming excitatory synapses, ascending global index */
    uint64_t n_in = 0;
    for (uint32_t i = 0; i < N; ++i) {
        if (i % net->Ncol >= net->Ne) continue;
        for (uint32_t j = 0; j < M; ++j) net->in_ptr[net->tgt[(uint64_t)i * M + j] + 1] += 1;
    }
    for (uint32_t k = 0; k < N; ++k) net->in_ptr[k + 1] += net->in_ptr[k];
    n_in = net->in_ptr[N];
    net->in_syn = (uint64_t *)xcalloc(n_in ? n_in : 1, sizeof(uint64_t));
    uint64_t *fill = (uint64_t *)xcalloc((uint64_t)N + 1, sizeof(uint64_t));
    if (!net->in_syn || !fill) { free(fill); orc_destroy(net); return NULL; }
    for (uint32_t i = 0; i < N; ++i) {
        if (i % net->Ncol >= net->Ne) continue;
        for (uint32_t j = 0; j < M; ++j) {
            uint64_t g = (uint64_t)i * M + j;
            uint32_t k = net->tgt[g];
            net->in_syn[net->in_ptr[k] + fill[k]++] = g;
        }
    }
    free(fill);

    /* initial state: v = c = -65, u = b v, no spikes */
    for (uint32_t k = 0; k < N; ++k) {
        float a, b, c, d;
        neuron_params(k % net->Ncol, net->Ne, &a, &b, &c, &d);
        net->v[k] = c;
        net->u[k] = b * c;
    }
    net->r_cap = 1024;
    net->r_id = (uint32_t *)malloc(net->r_cap * sizeof(uint32_t));
    net->r_t = (uint32_t *)malloc(net->r_cap * sizeof(uint32_t));
    if (!net->r_id || !net->r_t) { orc_destroy(net); return NULL; }
    net->t = 0;
    return net;
}

void orc_destroy(orc_net *net)
{
    if (!net) return;
    free(net->tgt); free(net->dly); free(net->w); free(net->P); free(net->D);
    free(net->dord); free(net->dptr); free(net->in_ptr); free(net->in_syn);
    free(net->v); free(net->u); free(net->accf); free(net->acci);
    if (net->hist) for (uint32_t k = 0; k < net->N; ++k) free(net->hist[k].s);
    free(net->hist); free(net->r_id); free(net->r_t); free(net->step_start); free(net->stim);
    free(net);
}

int orc_set_stimulus(orc_net *net, const uint32_t *t, const uint32_t *id, const float *mv, uint64_t n)
{
    free(net->stim); net->stim = NULL; net->n_stim = 0;
    if (n == 0) return 0;
    net->stim = (stim_entry *)malloc(n * sizeof(stim_entry));
    if (!net->stim) return -1;
    for (uint64_t e = 0; e < n; ++e) {
        if (id[e] >= net->N) return -2;
        net->stim[e].t = t[e]; net->stim[e].id = id[e]; net->stim[e].mv = mv[e];
    }
    net->n_stim = n;
    return 0;
}

/* Latest stamp of neuron k that is <= limit; returns 0 if none, else 1. */
static int latest_stamp(const orc_net *net, uint32_t k, int64_t limit, int32_t *out)
{
    const stamp_list *h = &net->hist[k];
    for (uint32_t e = h->n; e > 0; --e) {
        if ((int64_t)h->s[e - 1] <= limit) { *out = h->s[e - 1]; return 1; }
    }
    return 0;
}

static int push_stamp(stamp_list *h, int32_t s)
{
    if (h->n == h->cap) {
        uint32_t nc = h->cap ? 2u * h->cap : 8u;
        int32_t *p = (int32_t *)realloc(h->s, nc * sizeof(int32_t));
        if (!p) return -1;
        h->s = p; h->cap = nc;
    }
    h->s[h->n++] = s;
    return 0;
}

static int push_raster(orc_net *net, uint32_t t, uint32_t id)
{
    if (net->r_n == net->r_cap) {
        uint64_t nc = net->r_cap * 2u;
        uint32_t *a = (uint32_t *)realloc(net->r_id, nc * sizeof(uint32_t));
        if (!a) return -1;
        net->r_id = a;
        uint32_t *b = (uint32_t *)realloc(net->r_t, nc * sizeof(uint32_t));
        if (!b) return -1;
        net->r_t = b; net->r_cap = nc;
    }
    net->r_id[net->r_n] = id; net->r_t[net->r_n] = t; net->r_n++;
    return 0;
}

/* F(s): raster rows with stamp s (rows are appended in stamp order). */
static void spikes_at(const orc_net *net, uint32_t s, uint64_t *b, uint64_t *e)
{
    *b = net->step_start[s];
    *e = net->step_start[s + 1];
}

/* One 1 ms step t, in the order of the paper's simulation loop (Sec. 2,
 * "Mixed time-driven and event driven simulation", items 2.1-2.7), followed
 * by the periodic consolidation of the "long term synaptic plasticity" block
 * (Sec. 3, Table 2). */
static int step_once(orc_net *net)
{
    const orc_config *cfg = &net->cfg;
    const uint32_t t = net->t;
    const uint32_t N = net->N, M = net->M, Dmax = net->Dmax, Ncol = net->Ncol;
    const int fixed = (cfg->sum_mode == ORC_SUM_FIXED);

    /* 2.1 LTP: every neuron k stamped t potentiates its incoming excitatory
     * synapses.  Synapse (p -> k, delay d): the latest spike of p whose
     * arrival (stamp + d) is not after t pairs with this post spike;
     * dt = t_post - t_pre - d >= 0 and P += A+ exp(-dt/tau+). */
    if (t >= 1) {
        uint64_t b, e;
        spikes_at(net, t, &b, &e);
        for (uint64_t r = b; r < e; ++r) {
            uint32_t k = net->r_id[r];
            for (uint64_t x = net->in_ptr[k]; x < net->in_ptr[k + 1]; ++x) {
                uint64_t g = net->in_syn[x];
                uint32_t p = (uint32_t)(g / M);
                uint32_t d = net->dly[g];
                int32_t tp;
                net->n_ltp_visits++;
                if (latest_stamp(net, p, (int64_t)t - d, &tp)) {
                    uint32_t dt = (uint32_t)((int64_t)t - d - tp);
                    net->P[g] = net->P[g] + orc_tp(cfg, dt);
                    net->n_ltp_updates++;
                }
            }
        }
    }

    /* External input: thalamic picks of every column, then the stimulus list. */
    uint32_t picks[ORC_MAX_THAL];
    for (uint32_t c = 0; c < net->C; ++c) {
        uint32_t n = orc_thalamic(cfg, c, t, picks, ORC_MAX_THAL);
        if (n > ORC_MAX_THAL) return -3;
        for (uint32_t k = 0; k < n; ++k) {
            uint32_t id = c * Ncol + picks[k];
            if (fixed) net->acci[id] += q32(cfg->thalamic_current);
            else net->accf[id] = net->accf[id] + cfg->thalamic_current;
            net->n_thal++;
        }
    }
    for (uint64_t e = 0; e < net->n_stim; ++e) {
        if (net->stim[e].t != t) continue;
        uint32_t id = net->stim[e].id;
        if (fixed) net->acci[id] += q32(net->stim[e].mv);
        else net->accf[id] = net->accf[id] + net->stim[e].mv;
    }

    /* 2.3-2.6 delivery: a spike stamped s reaches the synapses of delay d in
     * step s + d - 1 (it first moves the target's potential at s + d).  The
     * synapse injects W into its target (Sec. 2, projection of synapses) and
     * the target's latest spike, which precedes the arrival, depresses it:
     * dt = t_post - t_pre - d < 0, D += A- exp(dt/tau-).  Order: delay
     * ascending, source id ascending, synapse index ascending. */
    for (uint32_t d = 1; d <= Dmax; ++d) {
        int64_t s = (int64_t)t - (int64_t)d + 1;
        if (s < 1) continue;
        uint64_t b, e;
        spikes_at(net, (uint32_t)s, &b, &e);
        for (uint64_t r = b; r < e; ++r) {
            uint32_t i = net->r_id[r];
            const uint32_t *ptr = net->dptr + (uint64_t)i * (Dmax + 1);
            int exc = (i % Ncol) < net->Ne;
            for (uint32_t x = ptr[d - 1]; x < ptr[d]; ++x) {
                uint32_t j = net->dord[(uint64_t)i * M + x];
                uint64_t g = (uint64_t)i * M + j;
                uint32_t k = net->tgt[g];
                if (fixed) net->acci[k] += q32(net->w[g]);
                else net->accf[k] = net->accf[k] + net->w[g];
                net->n_events++;
                if (exc) {
                    int32_t tq;
                    if (latest_stamp(net, k, (int64_t)t, &tq)) {
                        uint32_t dt = (uint32_t)((int64_t)t + 1 - tq);
                        net->D[g] = net->D[g] + orc_tm(cfg, dt);
                        net->n_ltd_updates++;
                    }
                }
            }
        }
    }

    /* 2.7 neuron dynamics and raster: fired neurons get stamp t + 1. */
    net->step_start[t + 1] = net->r_n;
    for (uint32_t k = 0; k < N; ++k) {
        float a, b, c, d;
        neuron_params(k % Ncol, net->Ne, &a, &b, &c, &d);
        float I = fixed ? dq32(net->acci[k]) : net->accf[k];
        if (orc_neuron_step(&net->v[k], &net->u[k], I, a, b, c, d)) {
            if (push_stamp(&net->hist[k], (int32_t)(t + 1)) != 0) return -1;
            if (push_raster(net, t + 1, k) != 0) return -1;
            net->n_spikes++;
        }
        net->accf[k] = 0.0f;
        net->acci[k] = 0;
    }
    net->step_start[t + 2] = net->r_n;

    /* Long-term plasticity: every weight_update_period steps each excitatory
     * synapse folds its derivative sd = P - D into the weight (reading:
     * w += bias + sd, clamped to [0, w_max]; sd decays by sd_decay). */
    if (cfg->weight_update_period > 0 && (t + 1) % cfg->weight_update_period == 0) {
        for (uint32_t i = 0; i < N; ++i) {
            if (i % Ncol >= net->Ne) continue;
            for (uint32_t j = 0; j < M; ++j) {
                uint64_t g = (uint64_t)i * M + j;
                float sd = net->P[g] - net->D[g];
                float x = net->w[g] + (cfg->wu_bias + sd);
                if (x < 0.0f) x = 0.0f;
                if (x > cfg->w_max) x = cfg->w_max;
                net->w[g] = x;
                net->P[g] = cfg->sd_decay * sd;
                net->D[g] = 0.0f;
            }
        }
    }
    net->t = t + 1;
    return 0;
}

int orc_run(orc_net *net, uint32_t n_steps)
{
    for (uint32_t s = 0; s < n_steps; ++s) {
        if (net->t + 1 > net->T_cap) return -4;
        int rc = step_once(net);
        if (rc != 0) return rc;
    }
    return 0;
}

uint32_t orc_time(const orc_net *net) { return net->t; }
uint64_t orc_raster_count(const orc_net *net) { return net->r_n; }

void orc_get_raster(const orc_net *net, uint32_t *times, uint32_t *ids)
{
    memcpy(times, net->r_t, net->r_n * sizeof(uint32_t));
    memcpy(ids, net->r_id, net->r_n * sizeof(uint32_t));
}

void orc_get_synapses(const orc_net *net, uint64_t first, uint64_t count, uint32_t *tgt,
                      uint8_t *dly, float *w, float *P, float *D)
{
    if (tgt) memcpy(tgt, net->tgt + first, count * sizeof(uint32_t));
    if (dly) memcpy(dly, net->dly + first, count);
    if (w) memcpy(w, net->w + first, count * sizeof(float));
    if (P) memcpy(P, net->P + first, count * sizeof(float));
    if (D) memcpy(D, net->D + first, count * sizeof(float));
}

void orc_get_state(const orc_net *net, float *v, float *u)
{
    memcpy(v, net->v, net->N * sizeof(float));
    memcpy(u, net->u, net->N * sizeof(float));
}

/* counters: events, ltp visits, ltp updates, ltd updates, spikes, thalamic */
void orc_get_counters(const orc_net *net, uint64_t out[6])
{
    out[0] = net->n_events; out[1] = net->n_ltp_visits; out[2] = net->n_ltp_updates;
    out[3] = net->n_ltd_updates; out[4] = net->n_spikes; out[5] = net->n_thal;
}

uint32_t orc_num_neurons(const orc_net *net) { return net->N; }
uint32_t orc_exc_per_column(const orc_config *cfg) { return exc_per_column(cfg); }
void orc_paper_blocks(uint32_t M, uint32_t out[13]) { paper_blocks(M, out); }
int64_t orc_q32(float x) { return q32(x); }
float orc_dq32(int64_t a) { return dq32(a); }
