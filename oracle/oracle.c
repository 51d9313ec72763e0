/*
 * CPU oracle (test infrastructure; see oracle.h).  Plain C, FP64, single
 * thread, compiled with -ffp-contract=off so every product and sum below is
 * rounded exactly as written.
 *
 * What it follows:
 *  - neuron: LIF of Sec. I-A (Eq. 1) with threshold, reset and refractory
 *    period (Eq. 2), integrated exactly over each step (the ODE is linear
 *    between spikes, so the step map is the matrix exponential of the linear
 *    system; the closed forms are derived in the comments of constants());
 *  - synapses: current-based delta, exponential or alpha kernels (the
 *    current form of Eq. 3; the conductance factor is not modelled);
 *  - step order of Sec. II-B: the input a neuron consumes at step n is the
 *    sum of the weights of all synapses whose source spiked at n - d;
 *    then every neuron updates and new spikes are emitted;
 *  - delivery is event driven: after the update of step n, each spiking
 *    source pushes its weights into a per-target ring of pending input,
 *    slot (n + d) mod D.  Pushing sources in ascending id and their edges in
 *    canonical order fixes the summation order of every slot.
 * Parity of each function: see the tests in tests/test_oracle_*.py.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Euler's number, rounded to double */
#define EULER_E 2.71828182845904523536

static char g_err[512];
static void set_err(const char* m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char* orc_last_error(void) { return g_err; }

/* ------------------------------------------------------------------ */
/* Philox4x64-10, from its published definition (Salmon, Moraes, Dror,
   Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of
   two 64x64->128 multiplications with the Philox multipliers, xor of the
   high halves with the other counter words and the round key, and a Weyl
   increment of the key between rounds. */
static void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += W0;
        k1 += W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t tag,
                   uint64_t seed, uint64_t inst, uint64_t out[4]) {
    uint64_t c[4] = {c0, c1, c2, tag};
    uint64_t k[2] = {seed, inst};
    orc_philox4x64_10(c, k, out);
}

/* floor(u * n / 2^64): an integer uniform on [0, n). */
static uint64_t range64(uint64_t u, uint64_t n) {
    uint64_t hi, lo;
    mulhilo64(u, n, &hi, &lo);
    return hi;
}
static double unit53(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }
static double unit53_open0(uint64_t u) { return (double)((u >> 11) + 1) * 0x1.0p-53; }

/* ------------------------------------------------------------------ */
/* Poisson counts by inversion of the CDF against 32-bit uniforms u:
   count = #{m : u >= thr[m]}, thr[m] = floor(F(m) 2^32), for every m whose
   threshold is below 2^32 - 1 (the tail left out is below 2^-32).  The CDF
   F(m) = sum_{k<=m} e^-l l^k / k! is accumulated term by term,
   p_k = p_{k-1} * l / k. */
int orc_poisson_table(double lambda, uint32_t* thr, int cap) {
    if (!(lambda >= 0.0) || lambda > 50.0) { set_err("poisson lambda out of range [0, 50]"); return -1; }
    if (lambda == 0.0) return 0;
    double p = exp(-lambda);
    double F = p;
    int m = 0;
    while (m < cap) {
        double t = F * 4294967296.0;
        if (t >= 4294967295.0) break;     /* remaining tail below 2^-32 */
        thr[m] = (uint32_t)t;
        m += 1;
        p = p * lambda / (double)m;
        F = F + p;
    }
    if (m == cap) { set_err("poisson table capacity exceeded"); return -2; }
    return m;
}

/* ------------------------------------------------------------------ */
typedef struct {
    double P22, P20, P11, P21, P31, P32, P21s, P22s, jump, conv, tpeak;
    int n_ref;
} consts_t;

/* Membrane response to a unit synaptic current at t (ms) (for the PSP peak).
   exp: I(s) = e^{-s/ts}; alpha: I(s) = (s/ts) e^{1-s/ts}.
   V(t) = (1/C) int_0^t e^{-(t-s)/tm} I(s) ds. With a = 1/ts - 1/tm:
   exp:   V = e^{-t/tm} (1 - e^{-a t}) / (C a)
   alpha: V = (e / (C ts)) e^{-t/tm} (1 - e^{-a t}(1 + a t)) / a^2
   and dV/dt = -V/tm + I(t)/C. */
static double psp_v(int model, double t, double tm, double ts, double C) {
    double a = 1.0 / ts - 1.0 / tm;
    if (model == ORC_EXP) {
        if (a == 0.0) return exp(-t / tm) * t / C;
        return exp(-t / tm) * (-expm1(-a * t)) / (C * a);
    }
    if (a == 0.0) return (EULER_E / (C * ts)) * exp(-t / tm) * t * t / 2.0;
    return (EULER_E / (C * ts)) * exp(-t / tm) * (1.0 - exp(-a * t) * (1.0 + a * t)) / (a * a);
}
static double psp_dv(int model, double t, double tm, double ts, double C) {
    double I = (model == ORC_EXP) ? exp(-t / ts) : (t / ts) * exp(1.0 - t / ts);
    return -psp_v(model, t, tm, ts, C) / tm + I / C;
}

static int constants(const orc_spec* s, consts_t* k) {
    double dt = s->dt, tm = s->tau_m, ts = s->tau_syn, C = s->C_m;
    if (!(dt > 0) || !(tm > 0) || !(C > 0)) { set_err("dt, tau_m, C_m must be > 0"); return -1; }
    if (s->model != ORC_DELTA && !(ts > 0)) { set_err("tau_syn must be > 0"); return -1; }
    if (s->model == ORC_COND && s->weight_unit != ORC_UNIT_NATIVE) {
        set_err("conductance synapses take native weights (nS)"); return -1;
    }
    memset(k, 0, sizeof *k);
    /* dU/dt = -U/tm + I/C: over dt, U -> e^{-dt/tm} U, and a constant
       current I_e adds (tm/C)(1 - e^{-dt/tm}) I_e. */
    k->P22 = exp(-dt / tm);
    k->P20 = -(tm / C) * expm1(-dt / tm);
    k->jump = 1.0;
    k->conv = 1.0;
    if (s->model == ORC_COND) {
        k->P11 = exp(-dt / ts);   /* conductance decay per step */
    } else if (s->model != ORC_DELTA) {
        /* synaptic kernel decays with e^{-dt/ts}; a current I present at the
           start of the step adds int_0^dt e^{-(dt-s)/tm} e^{-s/ts} ds / C
           = e^{-dt/tm}(1 - e^{-a dt})/(C a) to U (a = 1/ts - 1/tm). */
        double a = 1.0 / ts - 1.0 / tm;
        k->P11 = exp(-dt / ts);
        if (a == 0.0) k->P21 = k->P22 * dt / C;
        else k->P21 = k->P22 * (-expm1(-a * dt)) / (C * a);
        if (s->model == ORC_ALPHA) {
            /* alpha: y1' = -y1/ts, y2' = y1 - y2/ts (y2 is the current).
               y2 gains dt e^{-dt/ts} y1; U gains
               int_0^dt e^{-(dt-s)/tm} s e^{-s/ts} ds / C
               = e^{-dt/tm} (1 - e^{-a dt}(1 + a dt)) / (C a^2) per unit y1. */
            k->P21s = dt * k->P11;
            k->P22s = k->P11;
            k->P32 = k->P21;
            if (a == 0.0) k->P31 = k->P22 * dt * dt / (2.0 * C);
            else k->P31 = k->P22 * (1.0 - exp(-a * dt) * (1.0 + a * dt)) / (C * a * a);
            k->jump = EULER_E / ts;   /* current peaks at the weight, at t = ts */
        }
        if (s->weight_unit == ORC_UNIT_PSP_MV) {
            /* peak of the PSP of a unit current: bisection on dV/dt */
            double lo = 0.0, hi = 50.0 * (ts > tm ? ts : tm);
            for (int it = 0; it < 400; ++it) {
                double mid = 0.5 * (lo + hi);
                if (psp_dv(s->model, mid, tm, ts, C) > 0.0) lo = mid; else hi = mid;
            }
            double tp = 0.5 * (lo + hi);
            k->tpeak = tp;
            k->conv = 1.0 / psp_v(s->model, tp, tm, ts, C);
        }
    }
    k->n_ref = (int)floor(s->t_ref / dt + 0.5);
    if (k->n_ref < 0) k->n_ref = 0;
    return 0;
}

int orc_constants(const orc_spec* s, double out[12]) {
    consts_t k;
    if (constants(s, &k)) return -1;
    out[0] = k.P22; out[1] = k.P20; out[2] = k.P11; out[3] = k.P21; out[4] = k.P31;
    out[5] = k.P32; out[6] = k.P21s; out[7] = k.P22s; out[8] = k.jump; out[9] = k.conv;
    out[10] = (double)k.n_ref; out[11] = k.tpeak;
    return 0;
}

/* ------------------------------------------------------------------ */
struct orc_net {
    int model;
    consts_t k;
    double gL, dt_C, Eex, Ein, I_e;          /* conductance model (Eex, Ein relative to E_L) */
    double* ring_in;                         /* conductance model: inhibitory arrivals, like ring */
    double E_L, theta, Ur, P20Ie, w_ext;     /* theta, Ur relative to E_L */
    int64_t N, E;
    int32_t n_inst;
    int64_t* inst_off;        /* [n_inst + 1] */
    int32_t* inst_of;         /* [N] */
    uint64_t seed;
    /* canonical in-edges */
    int64_t* inptr;           /* [N + 1] */
    int32_t* src;             /* [E] global source id */
    double* w;                /* [E] native weight */
    int32_t* d;               /* [E] delay in steps */
    int32_t* tgt;             /* [E] global target id */
    /* out-edges: canonical edge ids grouped by source, ascending */
    int64_t* outptr;          /* [N + 1] */
    uint32_t* outidx;         /* [E] */
    int32_t dmin, dmax, D;
    /* poisson */
    uint32_t thr[64];
    int n_thr;
    /* selection */
    int64_t n_sel;
    int64_t* sel;             /* [n_sel] or NULL */
    int64_t* col_of;          /* [N] column in traces, -1 if not recorded */
    int64_t n_rec;
    /* state */
    double *U, *y1, *y2, *ring;
    int32_t* r;
    double *U0, *y10, *y20;
    int32_t* r0;
    int64_t t;
    double events;
    /* spike log */
    int64_t *log_step, *log_id;
    int64_t n_log, cap_log;
    /* plasticity */
    int stdp;
    double dt;
    int64_t stdp_lo, stdp_hi;               /* plastic population [lo, hi) */
    double s_lambda, s_alpha, s_mu, s_tp, s_tm, s_w0, s_wmax;
    unsigned char* plastic;                 /* [E] */
    double* x_last;                         /* [N] x_j just after its last spike */
    int64_t* q_last;                        /* [N] last spike step, -1: none */
    int64_t** hp;                           /* [N] post spike steps, ascending */
    double** hy;                            /* [N] y_i just after each of them */
    int64_t *hn, *hcap;                     /* [N] */
};

void orc_free(orc_net* n) {
    if (!n) return;
    free(n->inst_off); free(n->inst_of); free(n->inptr); free(n->src); free(n->w);
    free(n->d); free(n->tgt); free(n->outptr); free(n->outidx); free(n->sel); free(n->col_of);
    free(n->U); free(n->y1); free(n->y2); free(n->ring); free(n->ring_in); free(n->r);
    free(n->U0); free(n->y10); free(n->y20); free(n->r0);
    free(n->log_step); free(n->log_id);
    if (n->hp) for (int64_t i = 0; i < n->N; ++i) { free(n->hp[i]); free(n->hy[i]); }
    free(n->hp); free(n->hy); free(n->hn); free(n->hcap);
    free(n->plastic); free(n->x_last); free(n->q_last);
    free(n);
}

typedef struct { int32_t* src; double* w; int32_t* d; int64_t n, cap; } edgebuf;
static int eb_push(edgebuf* b, int32_t s, double w, int32_t d) {
    if (b->n == b->cap) {
        int64_t nc = b->cap ? b->cap * 2 : 1024;
        int32_t* ns = (int32_t*)realloc(b->src, (size_t)nc * sizeof(int32_t));
        if (!ns) return -1;
        b->src = ns;
        double* nw = (double*)realloc(b->w, (size_t)nc * sizeof(double));
        if (!nw) return -1;
        b->w = nw;
        int32_t* nd = (int32_t*)realloc(b->d, (size_t)nc * sizeof(int32_t));
        if (!nd) return -1;
        b->d = nd;
        b->cap = nc;
    }
    b->src[b->n] = s; b->w[b->n] = w; b->d[b->n] = d; b->n++;
    return 0;
}

/* The draws of one synapse (target tl, projection pl, slot) come from one
   Philox block with counter (tl, slot, pl, 1): word 0 picks the source,
   word 1 an integer-uniform delay, words 2 and 3 a Box-Muller pair whose
   first normal perturbs the weight and whose second perturbs a normal
   delay. */
static void edge_draws(uint64_t seed, uint64_t inst, int64_t tl, int64_t slot, int64_t pl,
                       uint64_t words[4], double* z0, double* z1) {
    philox((uint64_t)tl, (uint64_t)slot, (uint64_t)pl, 1, seed, inst, words);
    double u1 = unit53_open0(words[2]);
    double u2 = unit53(words[3]);
    double rr = sqrt(-2.0 * log(u1));
    double th = 6.283185307179586 * u2;
    *z0 = rr * cos(th);
    *z1 = rr * sin(th);
}

static double edge_weight(const orc_proj* pr, double z0, double conv) {
    double w;
    if (pr->w_sd == 0.0) {
        w = pr->w_mean;
    } else {
        double t = pr->w_sd * z0;
        w = pr->w_mean + t;
        if (pr->w_mean > 0.0 && w < 0.0) w = 0.0;
        if (pr->w_mean < 0.0 && w > 0.0) w = 0.0;
    }
    if (conv != 1.0) w = w * conv;
    return w;
}

static int32_t steps_of(double ms, double dt) {
    double x = ms / dt + 0.5;
    double f = floor(x);
    if (f < 1.0) return 1;
    if (f > 1e9) return 1000000000;
    return (int32_t)f;
}

static int32_t edge_delay(const orc_proj* pr, uint64_t w1, double z1, double dt) {
    if (pr->delay_kind == ORC_DELAY_CONST) return steps_of(pr->d0, dt);
    if (pr->delay_kind == ORC_DELAY_UNIFORM_INT) {
        int64_t lo = (int64_t)pr->d0, hi = (int64_t)pr->d1;
        return (int32_t)(lo + (int64_t)range64(w1, (uint64_t)(hi - lo + 1)));
    }
    double t = pr->d1 * z1;
    return steps_of(pr->d0 + t, dt);
}

static int is_selected(const orc_spec* s, int64_t g, int64_t* cursor) {
    if (!s->sel) return 1;
    while (*cursor < s->n_sel && s->sel[*cursor] < g) (*cursor)++;
    return *cursor < s->n_sel && s->sel[*cursor] == g;
}

orc_net* orc_build(const orc_spec* s, uint64_t seed) {
    consts_t k;
    if (constants(s, &k)) return NULL;
    if (s->model < 0 || s->model > 3) { set_err("bad model"); return NULL; }
    if (s->n_instances < 1 || s->n_pops < 1) { set_err("need at least one instance and population"); return NULL; }
    if (!(s->V_reset < s->V_th)) { set_err("V_reset must be below V_th"); return NULL; }
    orc_net* n = (orc_net*)calloc(1, sizeof(orc_net));
    if (!n) { set_err("out of memory"); return NULL; }
    n->model = s->model;
    n->k = k;
    n->seed = seed;
    n->E_L = s->E_L;
    n->theta = s->V_th - s->E_L;
    n->Ur = s->V_reset - s->E_L;
    n->P20Ie = k.P20 * s->I_e;
    n->w_ext = (s->weight_unit == ORC_UNIT_PSP_MV && k.conv != 1.0) ? s->w_ext * k.conv : s->w_ext;
    n->n_thr = orc_poisson_table(s->poisson_lambda, n->thr, 64);
    if (n->n_thr < 0) { orc_free(n); return NULL; }

    /* populations -> global ranges */
    int64_t* pop_off = (int64_t*)calloc((size_t)s->n_pops + 1, sizeof(int64_t));
    int64_t* pop_local = (int64_t*)calloc((size_t)s->n_pops + 1, sizeof(int64_t));
    n->n_inst = s->n_instances;
    n->inst_off = (int64_t*)calloc((size_t)s->n_instances + 1, sizeof(int64_t));
    if (!pop_off || !pop_local || !n->inst_off) { set_err("out of memory"); goto fail; }
    for (int p = 0; p < s->n_pops; ++p) {
        if (s->pops[p].instance < 0 || s->pops[p].instance >= s->n_instances ||
            (p > 0 && s->pops[p].instance < s->pops[p - 1].instance) || s->pops[p].size < 1) {
            set_err("populations must be grouped by instance, sizes >= 1"); goto fail;
        }
        pop_off[p + 1] = pop_off[p] + s->pops[p].size;
    }
    n->N = pop_off[s->n_pops];
    for (int b = 0, p = 0; b < s->n_instances; ++b) {
        n->inst_off[b] = (p < s->n_pops) ? pop_off[p] : n->N;
        while (p < s->n_pops && s->pops[p].instance == b) ++p;
    }
    n->inst_off[s->n_instances] = n->N;
    for (int p = 0; p < s->n_pops; ++p)
        pop_local[p] = pop_off[p] - n->inst_off[s->pops[p].instance];
    if (n->N > 2147483647LL) { set_err("too many neurons for the oracle"); goto fail; }
    n->inst_of = (int32_t*)malloc((size_t)n->N * sizeof(int32_t));
    if (!n->inst_of) { set_err("out of memory"); goto fail; }
    for (int b = 0; b < s->n_instances; ++b)
        for (int64_t i = n->inst_off[b]; i < n->inst_off[b + 1]; ++i) n->inst_of[i] = b;

    for (int q = 0; q < s->n_projs; ++q) {
        const orc_proj* pr = &s->projs[q];
        if (pr->src_pop < 0 || pr->src_pop >= s->n_pops || pr->tgt_pop < 0 || pr->tgt_pop >= s->n_pops ||
            s->pops[pr->src_pop].instance != s->pops[pr->tgt_pop].instance) {
            set_err("projection must connect populations of one instance"); goto fail;
        }
        if (pr->rule == ORC_FIXED_INDEGREE && pr->k < 0) { set_err("negative in-degree"); goto fail; }
        if (pr->rule == ORC_PAIRWISE && !(pr->p >= 0.0 && pr->p <= 1.0)) { set_err("p outside [0, 1]"); goto fail; }
        if (pr->rule == ORC_FIXED_INDEGREE && !pr->autapses && pr->src_pop == pr->tgt_pop &&
            s->pops[pr->src_pop].size < 2 && pr->k > 0) { set_err("no source left without autapses"); goto fail; }
        if (pr->delay_kind == ORC_DELAY_UNIFORM_INT && (pr->d0 < 1 || pr->d1 < pr->d0)) {
            set_err("uniform delay needs 1 <= lo <= hi steps"); goto fail;
        }
    }

    /* selection */
    n->n_sel = s->sel ? s->n_sel : 0;
    n->col_of = (int64_t*)malloc((size_t)n->N * sizeof(int64_t));
    if (!n->col_of) { set_err("out of memory"); goto fail; }
    if (s->sel) {
        n->sel = (int64_t*)malloc((size_t)(s->n_sel > 0 ? s->n_sel : 1) * sizeof(int64_t));
        if (!n->sel) { set_err("out of memory"); goto fail; }
        for (int64_t i = 0; i < n->N; ++i) n->col_of[i] = -1;
        for (int64_t c = 0; c < s->n_sel; ++c) {
            if (s->sel[c] < 0 || s->sel[c] >= n->N || (c > 0 && s->sel[c] <= s->sel[c - 1])) {
                set_err("selection must be sorted distinct ids"); goto fail;
            }
            n->sel[c] = s->sel[c];
            n->col_of[s->sel[c]] = c;
        }
        n->n_rec = s->n_sel;
    } else {
        for (int64_t i = 0; i < n->N; ++i) n->col_of[i] = i;
        n->n_rec = n->N;
    }

    /* canonical in-edges: per target, projections in order, slots in order */
    n->inptr = (int64_t*)calloc((size_t)n->N + 1, sizeof(int64_t));
    if (!n->inptr) { set_err("out of memory"); goto fail; }
    {
        edgebuf eb = {0};
        int64_t cursor = 0;
        n->dmin = 1 << 30;
        n->dmax = 0;
        for (int64_t i = 0; i < n->N; ++i) {
            int b = n->inst_of[i];
            int64_t tl = i - n->inst_off[b];
            if (is_selected(s, i, &cursor)) {
                int64_t pl = -1;
                for (int q = 0; q < s->n_projs; ++q) {
                    const orc_proj* pr = &s->projs[q];
                    if (s->pops[pr->tgt_pop].instance != b) continue;
                    pl++;     /* projection index within the instance */
                    int64_t tp0 = pop_off[pr->tgt_pop];
                    if (i < tp0 || i >= tp0 + s->pops[pr->tgt_pop].size) continue;
                    int64_t t_in_pop = i - tp0;
                    int64_t ns = s->pops[pr->src_pop].size;
                    int same = (pr->src_pop == pr->tgt_pop) && !pr->autapses;
                    int64_t sbase = pop_local[pr->src_pop];
                    if (pr->rule == ORC_FIXED_INDEGREE) {
                        for (int64_t slot = 0; slot < pr->k; ++slot) {
                            uint64_t wd[4]; double z0, z1;
                            edge_draws(seed, (uint64_t)b, tl, slot, pl, wd, &z0, &z1);
                            int64_t sl;
                            if (same) {
                                sl = (int64_t)range64(wd[0], (uint64_t)(ns - 1));
                                if (sl >= t_in_pop) sl += 1;
                            } else {
                                sl = (int64_t)range64(wd[0], (uint64_t)ns);
                            }
                            int32_t dd = edge_delay(pr, wd[1], z1, s->dt);
                            double ww = edge_weight(pr, z0, k.conv);
                            if (eb_push(&eb, (int32_t)(n->inst_off[b] + sbase + sl), ww, dd)) {
                                set_err("out of memory"); free(eb.src); free(eb.w); free(eb.d); goto fail;
                            }
                            if (dd < n->dmin) n->dmin = dd;
                            if (dd > n->dmax) n->dmax = dd;
                        }
                    } else {
                        /* pairwise Bernoulli: pair (target, j) connects iff the
                           64-bit word (tl, j>>2, pl, 5)[j&3] is below p 2^64 */
                        uint64_t thr_p = (pr->p >= 1.0) ? UINT64_MAX : (uint64_t)ldexp(pr->p, 64);
                        int all = pr->p >= 1.0;
                        int64_t slot = 0;
                        uint64_t wb[4];
                        for (int64_t j = 0; j < ns; ++j) {
                            if ((j & 3) == 0) philox((uint64_t)tl, (uint64_t)(j >> 2), (uint64_t)pl, 5, seed, (uint64_t)b, wb);
                            if (same && j == t_in_pop) continue;
                            if (!(all || wb[j & 3] < thr_p)) continue;
                            uint64_t wd[4]; double z0, z1;
                            edge_draws(seed, (uint64_t)b, tl, slot, pl, wd, &z0, &z1);
                            int32_t dd = edge_delay(pr, wd[1], z1, s->dt);
                            double ww = edge_weight(pr, z0, k.conv);
                            if (eb_push(&eb, (int32_t)(n->inst_off[b] + sbase + j), ww, dd)) {
                                set_err("out of memory"); free(eb.src); free(eb.w); free(eb.d); goto fail;
                            }
                            if (dd < n->dmin) n->dmin = dd;
                            if (dd > n->dmax) n->dmax = dd;
                            slot++;
                        }
                    }
                }
            }
            n->inptr[i + 1] = eb.n;
        }
        n->E = eb.n;
        n->src = eb.src; n->w = eb.w; n->d = eb.d;
        if (n->E == 0) { n->dmin = 1; n->dmax = 1; }
    }
    if (n->E >= 4294967296LL) { set_err("too many edges for the oracle"); goto fail; }
    n->D = n->dmax + 1;

    n->tgt = (int32_t*)malloc((size_t)(n->E > 0 ? n->E : 1) * sizeof(int32_t));
    if (!n->tgt) { set_err("out of memory"); goto fail; }
    for (int64_t i = 0; i < n->N; ++i)
        for (int64_t e = n->inptr[i]; e < n->inptr[i + 1]; ++e) n->tgt[e] = (int32_t)i;

    /* out-edges: stable counting sort of canonical edge ids by source */
    n->outptr = (int64_t*)calloc((size_t)n->N + 1, sizeof(int64_t));
    n->outidx = (uint32_t*)malloc((size_t)(n->E > 0 ? n->E : 1) * sizeof(uint32_t));
    if (!n->outptr || !n->outidx) { set_err("out of memory"); goto fail; }
    for (int64_t e = 0; e < n->E; ++e) n->outptr[n->src[e] + 1]++;
    for (int64_t i = 0; i < n->N; ++i) n->outptr[i + 1] += n->outptr[i];
    {
        int64_t* fill = (int64_t*)malloc((size_t)n->N * sizeof(int64_t));
        if (!fill) { set_err("out of memory"); goto fail; }
        memcpy(fill, n->outptr, (size_t)n->N * sizeof(int64_t));
        for (int64_t e = 0; e < n->E; ++e) n->outidx[fill[n->src[e]]++] = (uint32_t)e;
        free(fill);
    }

    /* state */
    n->U = (double*)calloc((size_t)n->N, sizeof(double));
    n->y1 = (double*)calloc((size_t)n->N, sizeof(double));
    n->y2 = (double*)calloc((size_t)n->N, sizeof(double));
    n->r = (int32_t*)calloc((size_t)n->N, sizeof(int32_t));
    n->U0 = (double*)calloc((size_t)n->N, sizeof(double));
    n->y10 = (double*)calloc((size_t)n->N, sizeof(double));
    n->y20 = (double*)calloc((size_t)n->N, sizeof(double));
    n->r0 = (int32_t*)calloc((size_t)n->N, sizeof(int32_t));
    n->ring = (double*)calloc((size_t)n->N * (size_t)n->D, sizeof(double));
    if (!n->U || !n->y1 || !n->y2 || !n->r || !n->U0 || !n->y10 || !n->y20 || !n->r0 || !n->ring) {
        set_err("out of memory"); goto fail;
    }
    if (s->model == ORC_COND) {
        n->ring_in = (double*)calloc((size_t)n->N * (size_t)n->D, sizeof(double));
        if (!n->ring_in) { set_err("out of memory"); goto fail; }
        n->gL = s->C_m / s->tau_m;
        n->dt_C = s->dt / s->C_m;
        n->Eex = s->E_ex - s->E_L;
        n->Ein = s->E_in - s->E_L;
        n->I_e = s->I_e;
    }
    /* initial membrane potential uniform on [v0_lo, v0_hi): word 0 of the
       block (neuron, 0, 0, 3) */
    for (int64_t i = 0; i < n->N; ++i) {
        int b = n->inst_of[i];
        uint64_t wv[4];
        philox((uint64_t)(i - n->inst_off[b]), 0, 0, 3, seed, (uint64_t)b, wv);
        double u = unit53(wv[0]);
        double span = s->v0_hi - s->v0_lo;
        double t = span * u;
        double v = s->v0_lo + t;
        n->U[i] = v - s->E_L;
        n->U0[i] = n->U[i];
    }
    /* plasticity: the synapses inside population stdp_pop */
    if (s->stdp_pop >= 0) {
        if (s->stdp_pop >= s->n_pops) { set_err("stdp_pop out of range"); goto fail; }
        if (!(s->stdp_lambda >= 0.0 && s->stdp_alpha >= 0.0 && s->stdp_tau_plus > 0.0 &&
              s->stdp_tau_minus > 0.0 && s->stdp_w0 > 0.0 && s->stdp_wmax > 0.0)) {
            set_err("bad plasticity parameters"); goto fail;
        }
        double cw = (s->weight_unit == ORC_UNIT_PSP_MV) ? k.conv : 1.0;
        n->stdp = 1;
        n->dt = s->dt;
        n->stdp_lo = pop_off[s->stdp_pop];
        n->stdp_hi = pop_off[s->stdp_pop + 1];
        n->s_lambda = s->stdp_lambda;
        n->s_alpha = s->stdp_alpha;
        n->s_mu = s->stdp_mu;
        n->s_tp = s->stdp_tau_plus;
        n->s_tm = s->stdp_tau_minus;
        n->s_w0 = s->stdp_w0 * cw;
        n->s_wmax = s->stdp_wmax * cw;
        n->plastic = (unsigned char*)calloc((size_t)(n->E > 0 ? n->E : 1), 1);
        n->x_last = (double*)calloc((size_t)n->N, sizeof(double));
        n->q_last = (int64_t*)malloc((size_t)n->N * sizeof(int64_t));
        n->hp = (int64_t**)calloc((size_t)n->N, sizeof(int64_t*));
        n->hy = (double**)calloc((size_t)n->N, sizeof(double*));
        n->hn = (int64_t*)calloc((size_t)n->N, sizeof(int64_t));
        n->hcap = (int64_t*)calloc((size_t)n->N, sizeof(int64_t));
        if (!n->plastic || !n->x_last || !n->q_last || !n->hp || !n->hy || !n->hn || !n->hcap) {
            set_err("out of memory"); goto fail;
        }
        for (int64_t i = 0; i < n->N; ++i) n->q_last[i] = -1;
        for (int64_t e = 0; e < n->E; ++e)
            n->plastic[e] = n->src[e] >= n->stdp_lo && n->src[e] < n->stdp_hi &&
                            n->tgt[e] >= n->stdp_lo && n->tgt[e] < n->stdp_hi;
    }
    free(pop_off);
    free(pop_local);
    return n;
fail:
    free(pop_off);
    free(pop_local);
    orc_free(n);
    return NULL;
}

int64_t orc_num_neurons(const orc_net* n) { return n->N; }
int64_t orc_num_edges(const orc_net* n) { return n->E; }
int32_t orc_max_delay(const orc_net* n) { return n->dmax; }
int32_t orc_min_delay(const orc_net* n) { return n->dmin; }
int64_t orc_current_step(const orc_net* n) { return n->t; }
double orc_events(const orc_net* n) { return n->events; }

int orc_export_graph(const orc_net* n, int64_t* src, int64_t* tgt, double* w, int32_t* d) {
    for (int64_t i = 0; i < n->N; ++i)
        for (int64_t e = n->inptr[i]; e < n->inptr[i + 1]; ++e) {
            if (src) src[e] = n->src[e];
            if (tgt) tgt[e] = i;
            if (w) w[e] = n->w[e];
            if (d) d[e] = n->d[e];
        }
    return 0;
}

int orc_set_weight(orc_net* n, int64_t e, double w) {
    if (e < 0 || e >= n->E) { set_err("edge index out of range"); return -1; }
    n->w[e] = w;
    return 0;
}

int orc_set_weights(orc_net* n, const double* w) {
    memcpy(n->w, w, (size_t)n->E * sizeof(double));
    return 0;
}

int orc_reset(orc_net* n) {
    memcpy(n->U, n->U0, (size_t)n->N * sizeof(double));
    memcpy(n->y1, n->y10, (size_t)n->N * sizeof(double));
    memcpy(n->y2, n->y20, (size_t)n->N * sizeof(double));
    memcpy(n->r, n->r0, (size_t)n->N * sizeof(int32_t));
    memset(n->ring, 0, (size_t)n->N * (size_t)n->D * sizeof(double));
    if (n->ring_in) memset(n->ring_in, 0, (size_t)n->N * (size_t)n->D * sizeof(double));
    n->t = 0;
    n->events = 0.0;
    n->n_log = 0;
    if (n->stdp) {   /* traces and histories restart; the weights stay */
        for (int64_t i = 0; i < n->N; ++i) {
            n->x_last[i] = 0.0;
            n->q_last[i] = -1;
            n->hn[i] = 0;
        }
    }
    return 0;
}

int orc_get_state(const orc_net* n, double* V, int32_t* r, double* y1, double* y2) {
    for (int64_t i = 0; i < n->N; ++i) {
        if (V) V[i] = n->U[i] + n->E_L;
        if (r) r[i] = n->r[i];
        if (y1) y1[i] = n->y1[i];
        if (y2) y2[i] = n->y2[i];
    }
    return 0;
}

/* Poisson count of neuron i at step: 32-bit half (step & 1) of word
   (step & 7) >> 1 of the block (neuron, step >> 3, 0, 2). */
static int poisson_count(const orc_net* n, int64_t i, int64_t step) {
    if (n->n_thr == 0) return 0;
    int b = n->inst_of[i];
    uint64_t wp[4];
    philox((uint64_t)(i - n->inst_off[b]), (uint64_t)(step >> 3), 0, 2, n->seed, (uint64_t)b, wp);
    uint64_t word = wp[(step & 7) >> 1];
    uint32_t u = (step & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
    int c = 0;
    for (int m = 0; m < n->n_thr; ++m) c += (u >= n->thr[m]);
    return c;
}

/* One neuron update at step n with summed synaptic input x.
   Returns 1 if the neuron integrated (was not refractory). */
static int update_neuron(orc_net* n, int64_t i, double x, double xin, int k) {
    const consts_t* c = &n->k;
    double ext = n->w_ext * (double)k;
    int integ = 0;
    double U = n->U[i];
    if (n->model == ORC_COND) {
        /* y1 = g_ex, y2 = g_in (nS); x, xin: this step's arrivals */
        if (n->r[i] > 0) {
            n->r[i] -= 1;
            U = n->Ur;
        } else {
            integ = 1;
            double G = n->gL + n->y1[i];
            G = G + n->y2[i];
            double num = n->y1[i] * n->Eex;
            num = num + n->y2[i] * n->Ein;
            num = num + n->I_e;
            double Uinf = num / G;
            double e = exp(-n->dt_C * G);
            U = Uinf + (U - Uinf) * e;
        }
        double gex = c->P11 * n->y1[i];
        double gin = c->P11 * n->y2[i];
        if (ext >= 0.0) gex = gex + ext; else gin = gin - ext;
        n->y1[i] = gex + x;
        n->y2[i] = gin + xin;
        n->U[i] = U;
        return integ;
    }
    if (n->r[i] > 0) {
        n->r[i] -= 1;
        U = n->Ur;
    } else {
        integ = 1;
        U = c->P22 * U;
        if (n->model == ORC_EXP) {
            U = U + c->P21 * n->y1[i];
        } else if (n->model == ORC_ALPHA) {
            U = U + c->P31 * n->y1[i];
            U = U + c->P32 * n->y2[i];
        }
        U = U + n->P20Ie;
        if (n->model == ORC_DELTA) U = U + (x + ext);
    }
    if (n->model == ORC_EXP) {
        double I = c->P11 * n->y1[i];
        n->y1[i] = I + (x + ext);
    } else if (n->model == ORC_ALPHA) {
        double t1 = c->P21s * n->y1[i];
        double t2 = c->P22s * n->y2[i];
        n->y2[i] = t1 + t2;
        double a = c->P11 * n->y1[i];
        double j = c->jump * (x + ext);
        n->y1[i] = a + j;
    }
    n->U[i] = U;
    return integ;
}

static int log_spike(orc_net* n, int64_t step, int64_t id) {
    if (n->n_log == n->cap_log) {
        int64_t nc = n->cap_log ? 2 * n->cap_log : 4096;
        int64_t* a = (int64_t*)realloc(n->log_step, (size_t)nc * sizeof(int64_t));
        if (!a) return -1;
        n->log_step = a;
        int64_t* b = (int64_t*)realloc(n->log_id, (size_t)nc * sizeof(int64_t));
        if (!b) return -1;
        n->log_id = b;
        n->cap_log = nc;
    }
    n->log_step[n->n_log] = step;
    n->log_id[n->n_log] = id;
    n->n_log++;
    return 0;
}

/* Plasticity bookkeeping of a postsynaptic spike of i at step p: the
   trace y_i just after it, appended to i's history. */
static int stdp_post(orc_net* n, int64_t i, int64_t p) {
    if (!n->stdp) return 0;
    int64_t m = n->hn[i];
    double y = 1.0;
    if (m > 0) y += n->hy[i][m - 1] * exp(-(double)(p - n->hp[i][m - 1]) * n->dt / n->s_tm);
    if (m == n->hcap[i]) {
        int64_t nc = m ? 2 * m : 16;
        int64_t* a = (int64_t*)realloc(n->hp[i], (size_t)nc * sizeof(int64_t));
        if (!a) return -1;
        n->hp[i] = a;
        double* b = (double*)realloc(n->hy[i], (size_t)nc * sizeof(double));
        if (!b) return -1;
        n->hy[i] = b;
        n->hcap[i] = nc;
    }
    n->hp[i][m] = p;
    n->hy[i][m] = y;
    n->hn[i] = m + 1;
    return 0;
}

/* New weight of plastic synapse e (source j, target i, delay d) when the
   spike of j at step q is delivered (the rule of oracle.h). */
static double stdp_weight(const orc_net* n, int64_t e, int64_t j, int64_t q) {
    const double dt = n->dt;
    const int64_t i = n->tgt[e], d = n->d[e];
    const int64_t m = n->hn[i];
    const int64_t* hp = n->hp[i];
    double w = n->w[e];
    if (n->q_last[j] >= 0) {
        const int64_t ql = n->q_last[j];
        const double c = n->s_lambda * pow(n->s_w0, 1.0 - n->s_mu);
        for (int64_t k = 0; k < m; ++k) {
            const int64_t a = hp[k] + d;   /* arrival of the post spike at the synapse */
            if (a <= ql) continue;
            if (a > q) break;
            const double x = n->x_last[j] * exp(-(double)(a - ql) * dt / n->s_tp);
            w = w + c * pow(w, n->s_mu) * x;
            if (w > n->s_wmax) w = n->s_wmax;
        }
    }
    /* y_i at q - d: the latest post spike strictly before it */
    double y = 0.0;
    for (int64_t k = m - 1; k >= 0; --k) {
        if (hp[k] < q - d) {
            y = n->hy[i][k] * exp(-(double)(q - d - hp[k]) * dt / n->s_tm);
            break;
        }
    }
    w = w - n->s_lambda * n->s_alpha * w * y;
    if (w < 0.0) w = 0.0;
    return w;
}

static void push_spike(orc_net* n, int64_t step, int64_t j) {
    for (int64_t q = n->outptr[j]; q < n->outptr[j + 1]; ++q) {
        int64_t e = n->outidx[q];
        if (n->stdp && n->plastic[e]) n->w[e] = stdp_weight(n, e, j, step);
        int64_t slot = (step + n->d[e]) % n->D;
        int64_t tg = n->tgt[e];
        if (n->ring_in && n->w[e] < 0.0) n->ring_in[tg * n->D + slot] += -n->w[e];
        else n->ring[tg * n->D + slot] += n->w[e];
        n->events += 1.0;
    }
    if (n->stdp) {
        /* the presynaptic trace just after this spike */
        double x = 1.0;
        if (n->q_last[j] >= 0) x += n->x_last[j] * exp(-(double)(step - n->q_last[j]) * n->dt / n->s_tp);
        n->x_last[j] = x;
        n->q_last[j] = step;
    }
}

int orc_run(orc_net* n, int64_t n_steps) {
    int64_t* spk = (int64_t*)malloc((size_t)(n->N > 0 ? n->N : 1) * sizeof(int64_t));
    if (!spk) { set_err("out of memory"); return -1; }
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t step = n->t;
        int64_t slot = step % n->D;
        int64_t ns = 0;
        for (int64_t i = 0; i < n->N; ++i) {
            double x = n->ring[i * n->D + slot];
            n->ring[i * n->D + slot] = 0.0;
            double xin = 0.0;
            if (n->ring_in) {
                xin = n->ring_in[i * n->D + slot];
                n->ring_in[i * n->D + slot] = 0.0;
            }
            int kc = poisson_count(n, i, step);
            int integ = update_neuron(n, i, x, xin, kc);
            if (integ && n->U[i] >= n->theta) {
                n->U[i] = n->Ur;
                n->r[i] = n->k.n_ref;
                spk[ns++] = i;
                if (log_spike(n, step, i) || stdp_post(n, i, step)) {
                    free(spk); set_err("out of memory"); return -1;
                }
            }
        }
        for (int64_t q = 0; q < ns; ++q) push_spike(n, step, spk[q]);
        n->t++;
    }
    free(spk);
    return 0;
}

int64_t orc_spike_count(const orc_net* n) { return n->n_log; }
int orc_get_spikes(const orc_net* n, int64_t* steps, int64_t* ids) {
    memcpy(steps, n->log_step, (size_t)n->n_log * sizeof(int64_t));
    memcpy(ids, n->log_id, (size_t)n->n_log * sizeof(int64_t));
    return 0;
}

static int check_raster(const orc_net* n, const int64_t* st, const int64_t* id, int64_t ns) {
    for (int64_t q = 0; q < ns; ++q) {
        if (id[q] < 0 || id[q] >= n->N) { set_err("raster id out of range"); return -1; }
        if (q > 0 && (st[q] < st[q - 1] || (st[q] == st[q - 1] && id[q] <= id[q - 1]))) {
            set_err("raster must be sorted by (step, id) without duplicates"); return -1;
        }
    }
    return 0;
}

/* Frozen-raster forward; optional per-step records for the adjoint:
   Urec = U after each step, mrec = 1 iff the neuron integrated and did not
   spike (the step map depends on the previous state). */
static int frozen_core(orc_net* n, const int64_t* st, const int64_t* id, int64_t nspk,
                       int64_t n_steps, double* xt, double* vt, double* Urec, unsigned char* mrec,
                       double* vpre) {
    if (check_raster(n, st, id, nspk)) return -1;
    int64_t q = 0;
    while (q < nspk && st[q] < n->t) q++;
    for (int64_t s = 0; s < n_steps; ++s) {
        int64_t step = n->t;
        int64_t slot = step % n->D;
        int64_t q0 = q;
        while (q < nspk && st[q] == step) q++;
        int64_t qs = q0;
        for (int64_t i = 0; i < n->N; ++i) {
            /* with a target selection only the selected neurons are simulated;
               the others merely emit the raster's spikes */
            if (n->sel && n->col_of[i] < 0) continue;
            double x = n->ring[i * n->D + slot];
            n->ring[i * n->D + slot] = 0.0;
            double xin = 0.0;
            if (n->ring_in) {
                xin = n->ring_in[i * n->D + slot];
                n->ring_in[i * n->D + slot] = 0.0;
            }
            int kc = poisson_count(n, i, step);
            int integ = update_neuron(n, i, x, xin, kc);
            x = x - xin;   /* the trace records the signed sum of the arrivals */
            int spk = 0;
            while (qs < q && id[qs] < i) qs++;
            if (qs < q && id[qs] == i) spk = 1;
            int64_t c = n->col_of[i];
            /* the membrane potential the threshold test of a closed-loop run
               would see (NaN on refractory steps, which take no test) */
            if (vpre && c >= 0) vpre[s * n->n_rec + c] = integ ? n->U[i] + n->E_L : NAN;
            if (spk) {
                n->U[i] = n->Ur;
                n->r[i] = n->k.n_ref;
                if (stdp_post(n, i, step)) { set_err("out of memory"); return -1; }
            }
            if (c >= 0) {
                if (xt) xt[s * n->n_rec + c] = x;
                if (vt) vt[s * n->n_rec + c] = n->U[i] + n->E_L;
                if (Urec) Urec[s * n->n_rec + c] = n->U[i];
                if (mrec) mrec[s * n->n_rec + c] = (unsigned char)(integ && !spk);
            }
        }
        for (int64_t p = q0; p < q; ++p) push_spike(n, step, id[p]);
        n->t++;
    }
    return 0;
}

int orc_run_frozen(orc_net* n, const int64_t* st, const int64_t* id, int64_t nspk,
                   int64_t n_steps, double* xt, double* vt) {
    return frozen_core(n, st, id, nspk, n_steps, xt, vt, NULL, NULL, NULL);
}

int orc_run_frozen_pre(orc_net* n, const int64_t* st, const int64_t* id, int64_t nspk,
                       int64_t n_steps, double* vpre) {
    return frozen_core(n, st, id, nspk, n_steps, NULL, NULL, NULL, NULL, vpre);
}

/* Reverse-mode gradient with spikes frozen.  Per neuron, with m_n = 1 iff
   step n integrated and did not spike, l_n = dL/dU_n (direct term):
     delta: a_n = l_n + m_{n+1} P22 a_{n+1};                 g_n = m_n a_n
     exp:   aU_n = l_n + m_{n+1} P22 aU_{n+1}
            aI_n = m_{n+1} P21 aU_{n+1} + P11 aI_{n+1};      g_n = aI_n
     alpha: aU_n  = l_n + m_{n+1} P22 aU_{n+1}
            a2_n  = m_{n+1} P32 aU_{n+1} + P22s a2_{n+1}
            a1_n  = m_{n+1} P31 aU_{n+1} + P21s a2_{n+1} + P11 a1_{n+1}
            g_n = jump * a1_n
   where g_n = dL/dx_n is the sensitivity to the input consumed at step n.
   Then dL/dw_e = sum over raster spikes (m, src_e) with m + d_e < T of
   g_{tgt_e}(m + d_e). */
int orc_backward(orc_net* n, const int64_t* st, const int64_t* id, int64_t nspk,
                 int64_t T, const double* vstar, double* grad, double* loss) {
    if (T < 1) { set_err("need at least one step"); return -1; }
    if (n->model == ORC_COND) { set_err("no adjoint for conductance synapses"); return -1; }
    if (check_raster(n, st, id, nspk)) return -1;
    orc_reset(n);    /* restart from the build-time state */
    size_t cells = (size_t)T * (size_t)n->n_rec;
    double* Urec = (double*)malloc(cells * sizeof(double));
    unsigned char* mrec = (unsigned char*)malloc(cells);
    double* g = (double*)malloc(cells * sizeof(double));
    if (!Urec || !mrec || !g) { free(Urec); free(mrec); free(g); set_err("out of memory"); return -1; }
    if (frozen_core(n, st, id, nspk, T, NULL, NULL, Urec, mrec, NULL)) { free(Urec); free(mrec); free(g); return -1; }
    const consts_t* c = &n->k;
    double L = 0.0;
    for (int64_t i = 0; i < n->N; ++i) {
        int64_t col = n->col_of[i];
        if (col < 0) continue;
        int b = n->inst_of[i];
        double Nb = (double)(n->inst_off[b + 1] - n->inst_off[b]);
        double scale = 1.0 / (Nb * (double)T);
        double aU = 0.0, a1 = 0.0, a2 = 0.0;   /* adjoints at step n+1 */
        int m_next = 0;
        for (int64_t s = T - 1; s >= 0; --s) {
            size_t at = (size_t)s * (size_t)n->n_rec + (size_t)col;
            double diff = (Urec[at] + n->E_L) - vstar[at];
            L += scale * diff * diff;
            double l = 2.0 * scale * diff;
            double naU = l + (m_next ? c->P22 * aU : 0.0);
            double na1 = 0.0, na2 = 0.0;
            if (n->model == ORC_EXP) {
                na1 = (m_next ? c->P21 * aU : 0.0) + c->P11 * a1;
            } else if (n->model == ORC_ALPHA) {
                na2 = (m_next ? c->P32 * aU : 0.0) + c->P22s * a2;
                na1 = (m_next ? c->P31 * aU : 0.0) + c->P21s * a2 + c->P11 * a1;
            }
            aU = naU; a1 = na1; a2 = na2;
            m_next = mrec[at];
            if (n->model == ORC_DELTA) g[at] = mrec[at] ? aU : 0.0;
            else if (n->model == ORC_EXP) g[at] = a1;
            else g[at] = c->jump * a1;
        }
    }
    *loss = L;
    for (int64_t e = 0; e < n->E; ++e) grad[e] = 0.0;
    for (int64_t q = 0; q < nspk; ++q) {
        int64_t m = st[q], j = id[q];
        if (m < 0 || m >= T) continue;
        for (int64_t p = n->outptr[j]; p < n->outptr[j + 1]; ++p) {
            int64_t e = n->outidx[p];
            int64_t arr = m + n->d[e];
            if (arr >= T) continue;
            int64_t col = n->col_of[n->tgt[e]];
            if (col < 0) continue;
            grad[e] += g[(size_t)arr * (size_t)n->n_rec + (size_t)col];
        }
    }
    free(Urec); free(mrec); free(g);
    return 0;
}
