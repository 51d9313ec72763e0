/*
 * CPU oracle for the LIF + delayed spike delivery step (test infrastructure).
 *
 * This is a plain, slow, single-threaded FP64 event-driven simulator of the
 * per-time-step procedure the paper describes (Sec. II-B: spiking sources act
 * on their targets after each synapse's delay, then every neuron updates and
 * emits new spikes), with the LIF neuron of Sec. I-A (Eq. 1-2) and current
 * based synapses (the current form of Eq. 3).  It exists only to check the
 * HIP library: only tests, the smoke check and the benchmark's CPU baseline
 * may load it.  It shares no code with the library.
 *
 * Conventions
 *  - neurons are numbered globally, instance after instance, population
 *    after population; spikes are reported as (step, global id);
 *  - canonical edge order is (target, projection, slot) ascending;
 *  - all functions return 0 on success and a negative value on error
 *    (message from orc_last_error()).
 */
#ifndef CORTEX_ORACLE_H
#define CORTEX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_DELTA = 0, ORC_EXP = 1, ORC_ALPHA = 2, ORC_COND = 3 };
enum { ORC_FIXED_INDEGREE = 0, ORC_PAIRWISE = 1 };
enum { ORC_DELAY_CONST = 0, ORC_DELAY_UNIFORM_INT = 1, ORC_DELAY_NORMAL = 2 };
enum { ORC_UNIT_NATIVE = 0, ORC_UNIT_PSP_MV = 1 };

typedef struct {
    int32_t instance;   /* instance the population belongs to */
    int64_t size;
} orc_pop;

typedef struct {
    int32_t src_pop, tgt_pop;   /* indices into the global population list */
    int32_t rule;
    int64_t k;                  /* fixed in-degree */
    double p;                   /* pairwise probability */
    double w_mean, w_sd;
    int32_t delay_kind;
    double d0, d1;
    int32_t autapses;
} orc_proj;

typedef struct {
    int32_t model;
    double dt, tau_m, C_m, E_L, V_th, V_reset, t_ref, I_e, tau_syn;
    int32_t weight_unit;
    double poisson_lambda, w_ext, v0_lo, v0_hi;
    int32_t n_instances;
    int32_t n_pops;
    const orc_pop* pops;
    int32_t n_projs;
    const orc_proj* projs;
    /* optional: only these targets (sorted global ids) receive in-edges;
       traces and target voltages then have n_sel columns */
    int64_t n_sel;
    const int64_t* sel;
    /* optional spike-timing dependent plasticity (orc_stdp_* below) of the
       synapses whose source and target both belong to population stdp_pop
       (global index; -1: none) */
    int32_t stdp_pop;
    double stdp_lambda, stdp_alpha, stdp_mu;   /* step size, depression ratio, potentiation exponent */
    double stdp_tau_plus, stdp_tau_minus;      /* pre- and postsynaptic trace time constants (ms) */
    double stdp_w0, stdp_wmax;                 /* reference and largest weight (the weights' unit) */
    /* conductance-based synapses (model ORC_COND): reversal potentials (mV)
       of the excitatory channel (weights >= 0, in nS) and the inhibitory
       channel (weights < 0, |w| in nS) */
    double E_ex, E_in;
} orc_spec;

/* Model ORC_COND (the conductance form of the synaptic current, Sec. I-A
   Eq. 3, with an exponential conductance): a spike arriving through a
   synapse of weight w adds |w| to the target's excitatory (w >= 0) or
   inhibitory (w < 0) conductance, each decaying with tau_syn, and
     C dV/dt = -g_L (V - E_L) + g_ex (E_ex - V) + g_in (E_in - V) + I_e,
   g_L = C / tau_m.  A step holds the conductances at their values at its
   start, for which the membrane's solution is exact:
     G = g_L + g_ex + g_in,  V_inf = (g_L E_L + g_ex E_ex + g_in E_in + I_e) / G,
     V <- V_inf + (V - V_inf) exp(-dt G / C);
   then g <- g exp(-dt / tau_syn) + (the step's arrivals), so that V feels
   an input from the next step on (as with current-based exponential
   synapses).  External Poisson events of weight w_ext enter the channel of
   w_ext's sign.  Weights are in nS (native units only). */

/* Plasticity rule (read from the paper's verification network: E->E
   synapses with multiplicative depression and power-law potentiation).
   All of a synapse's delay d is dendritic: a presynaptic spike at step q is
   at the synapse at q, a postsynaptic spike at step p reaches it at p + d.
   Traces (all-to-all pairing, time in ms = steps x dt):
     x_j(t) = sum over spikes q' <= t of source j of exp(-(t - q') / tau_plus)
     y_i(t) = sum over spikes p < t of target i of exp(-(t - p) / tau_minus)
   When the spike of j at step q is delivered, each plastic synapse (j, i, d)
   first takes, in ascending p, the postsynaptic spikes p of i with
   q_last < p + d <= q (q_last: j's previous spike; none before j's first):
     w <- min(w_max, w + lambda w0^(1 - mu) w^mu x_j(p + d)),
   with x_j(p + d) counting the spikes up to q_last only; then
     w <- max(0, w - lambda alpha w y_i(q - d)),
   and the spike is delivered with the new w.  Weights are not restored by
   orc_reset. */

typedef struct orc_net orc_net;

const char* orc_last_error(void);

/* Philox4x64-10 block (Salmon et al., SC'11): out = philox(ctr, key). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Poisson inversion thresholds floor(F(m) * 2^32) for m = 0, 1, ... while
   below 2^32.  Returns the number of entries (<= cap) or < 0. */
int orc_poisson_table(double lambda, uint32_t* thr, int cap);

/* Propagators and derived constants of the spec's neuron model:
   out[0]=P22 out[1]=P20 out[2]=P11 out[3]=P21 out[4]=P31 out[5]=P32
   out[6]=P21s out[7]=P22s out[8]=jump scale out[9]=psp conversion (native
   weight per mV of PSP peak) out[10]=n_ref out[11]=psp peak time (ms). */
int orc_constants(const orc_spec* spec, double out[12]);

orc_net* orc_build(const orc_spec* spec, uint64_t seed);
void orc_free(orc_net* net);

int64_t orc_num_neurons(const orc_net* net);
int64_t orc_num_edges(const orc_net* net);
int32_t orc_max_delay(const orc_net* net);
int32_t orc_min_delay(const orc_net* net);
int64_t orc_current_step(const orc_net* net);
double orc_events(const orc_net* net);

/* Edges in canonical order; global neuron ids; delays in steps. */
int orc_export_graph(const orc_net* net, int64_t* src, int64_t* tgt, double* w, int32_t* d);

/* Overwrite the stored weight of canonical edge e. */
int orc_set_weight(orc_net* net, int64_t e, double w);
/* Overwrite every stored weight (w in canonical order, E entries). */
int orc_set_weights(orc_net* net, const double* w);
/* Back to the build-time state: step 0, empty rings, spike log cleared. */
int orc_reset(orc_net* net);

/* State (post-update membrane potential V, refractory counter, synaptic
   state: exp -> y1 = current; alpha -> y1 = auxiliary, y2 = current). */
int orc_get_state(const orc_net* net, double* V, int32_t* r, double* y1, double* y2);

/* Closed loop: advance n_steps, spikes from threshold crossings. */
int orc_run(orc_net* net, int64_t n_steps);
int64_t orc_spike_count(const orc_net* net);
int orc_get_spikes(const orc_net* net, int64_t* steps, int64_t* ids);

/* Frozen raster: advance n_steps; a neuron spikes (and resets) exactly at
   the raster's (step, id) pairs, thresholds are not evaluated, and
   deliveries come from the raster.  Raster sorted by (step, id), absolute
   steps.  Optional traces [n_steps][n_rec] (n_rec = N or n_sel): x = summed
   synaptic input consumed at each step, v = membrane potential after it. */
int orc_run_frozen(orc_net* net, const int64_t* r_steps, const int64_t* r_ids,
                   int64_t n_spk, int64_t n_steps, double* x_trace, double* v_trace);

/* Frozen raster as orc_run_frozen; vpre [n_steps][n_rec] receives the
   membrane potential after each step's update and before any reset, i.e.
   the value a closed-loop run compares with the threshold (NaN on
   refractory steps, which take no threshold test). */
int orc_run_frozen_pre(orc_net* net, const int64_t* r_steps, const int64_t* r_ids,
                       int64_t n_spk, int64_t n_steps, double* vpre);

/* Gradient of L = sum_b 1/(N_b T) sum_{i in b, n < T} (V_i(n) - V*_i(n))^2
   with respect to every stored weight (canonical order), spikes frozen to
   the raster, starting from the state at build time.  vstar is
   [n_steps][n_rec].  loss receives L (over the recorded columns). */
int orc_backward(orc_net* net, const int64_t* r_steps, const int64_t* r_ids,
                 int64_t n_spk, int64_t n_steps, const double* vstar,
                 double* grad, double* loss);

#ifdef __cplusplus
}
#endif
#endif
