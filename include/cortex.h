/*
 * cortex.h - C ABI of the MI355X (gfx950) LIF + delayed spike delivery
 * library.
 *
 * The library simulates spiking networks of leaky integrate-and-fire neurons
 * (Sec. I-A, Eq. 1-2 of Lyu et al., "CORTEX: Large-Scale Brain Simulator
 * Utilizing Indegree Sub-Graph Decomposition on Fugaku Supercomputer") with
 * current-based delta, exponential or alpha synapses (the current form of
 * Eq. 3).  One time step follows the procedure of Sec. II-B: the synapses of
 * neurons that spiked d steps ago act on their targets, then every neuron
 * updates and emits new spikes.  Work is organised by the indegree sub-graph
 * decomposition of Sec. II-A (Eq. 5, 9-14) and the thread ownership of
 * Sec. III-B: the neurons are cut into tiles of consecutive targets, each tile
 * owns all synapses into its targets, and exactly one GPU workgroup writes a
 * tile's input buffers, so delivery needs no global atomics.
 *
 * Conventions for every entry point:
 *  - return value: CORTEX_OK (0) or a negative cortex_status; the message of
 *    the last failure on the calling thread is cortex_last_error();
 *  - "device" pointers are GPU memory of the device current at
 *    cortex_build_network; "host" pointers are CPU memory;
 *  - pointers passed in stay owned by the caller; the network owns the device
 *    memory it obtained from cortex_device.alloc and returns it through
 *    cortex_device.free in cortex_destroy;
 *  - work is enqueued on cortex_device.stream; calls documented as
 *    "synchronising" wait for that stream;
 *  - neurons are numbered globally: instance after instance, population after
 *    population; spike times are step indices n (time (n+1)*dt);
 *  - canonical synapse order is (target, projection, slot) ascending, where a
 *    projection's slot is its draw index for that target.
 */
#ifndef CORTEX_H
#define CORTEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CORTEX_ABI_VERSION 4

typedef enum {
    CORTEX_OK = 0,
    CORTEX_EINVAL = -1,       /* invalid argument or specification */
    CORTEX_ENOMEM = -2,       /* allocation failed */
    CORTEX_EDEVICE = -3,      /* HIP runtime error */
    CORTEX_ESTATE = -4,       /* call not valid in the network's state */
    CORTEX_EUNSUPPORTED = -5, /* valid request the library cannot serve */
    CORTEX_ETIMEOUT = -6,     /* a device-side wait exceeded its spin limit */
    CORTEX_ETRUNC = -7        /* output truncated (buffer or log capacity) */
} cortex_status;

enum { CORTEX_MODEL_DELTA = 0, CORTEX_MODEL_EXP = 1, CORTEX_MODEL_ALPHA = 2, CORTEX_MODEL_COND = 3 };
enum { CORTEX_RULE_FIXED_INDEGREE = 0, CORTEX_RULE_PAIRWISE = 1 };
enum { CORTEX_DELAY_CONST = 0, CORTEX_DELAY_UNIFORM_INT = 1, CORTEX_DELAY_NORMAL = 2 };
enum { CORTEX_UNIT_NATIVE = 0, CORTEX_UNIT_PSP_MV = 1 };
enum { CORTEX_FP32 = 0, CORTEX_FP64_VERIFY = 1 };
enum { CORTEX_W_FP32 = 0, CORTEX_W_BF16 = 1 };
/* FP32 launch plans: RESIDENT keeps every tile's input ring in workgroup-local
   memory for a whole persistent launch; STREAMED launches one kernel per
   window of steps and stages each tile's ring through HBM (networks whose
   rings do not fit the chip's workgroup-local memory); AUTO takes RESIDENT
   when it fits. */
enum { CORTEX_PLAN_AUTO = 0, CORTEX_PLAN_RESIDENT = 1, CORTEX_PLAN_STREAMED = 2 };

/* A population: `size` consecutive neurons of instance `instance`.
   Populations must be listed grouped by instance, instances ascending. */
typedef struct {
    int32_t instance;
    int64_t size;
} cortex_pop;

/* All synapses from population src_pop onto population tgt_pop (indices into
   the population list, same instance).
   rule FIXED_INDEGREE: each target draws k sources uniformly with replacement
   (no self-connection unless `autapses`); rule PAIRWISE: each (source,
   target) pair connects with probability p.
   Weight ~ Normal(w_mean, w_sd^2) clipped at 0 to keep the sign of w_mean
   (constant if w_sd == 0), in the spec's weight unit.
   Delay CONST: d0 ms; UNIFORM_INT: integer steps uniform on [d0, d1];
   NORMAL: Normal(d0, d1^2) ms.  ms values round to the nearest step, at
   least 1. */
typedef struct {
    int32_t src_pop, tgt_pop;
    int32_t rule;
    int64_t k;
    double p;
    double w_mean, w_sd;
    int32_t delay_kind;
    double d0, d1;
    int32_t autapses;
} cortex_proj;

/* Network specification.  Units ms, mV, pF, pA.  Weights are mV jumps
   (delta) or pA current amplitudes (exp: jump of the current; alpha: peak of
   the current); with weight_unit PSP_MV they (and w_ext) are the PSP peak in
   mV and the library converts them.  Each neuron receives a Poisson count
   with mean poisson_lambda per step, each event of weight w_ext.  Initial
   V ~ Uniform[v0_lo, v0_hi). */
typedef struct {
    uint32_t abi_version;     /* CORTEX_ABI_VERSION */
    uint32_t struct_size;     /* sizeof(cortex_spec) */
    int32_t model;            /* CORTEX_MODEL_* */
    int32_t precision;        /* CORTEX_FP32 or CORTEX_FP64_VERIFY */
    int32_t weight_dtype;     /* CORTEX_W_* (FP32 mode only) */
    int32_t weight_unit;      /* CORTEX_UNIT_* */
    double dt, tau_m, C_m, E_L, V_th, V_reset, t_ref, I_e, tau_syn;
    double poisson_lambda, w_ext, v0_lo, v0_hi;
    int32_t n_instances;
    int32_t n_pops;
    const cortex_pop* pops;   /* host, n_pops */
    int32_t n_projs;
    const cortex_proj* projs; /* host, n_projs */
    int32_t tile_size;        /* targets per tile; 0 = automatic; at most 2 x block_size
                                 (4 x with block_size 512) */
    int32_t block_size;       /* threads per workgroup: 0 (auto), 256, 512, 1024 */
    int64_t record_steps;     /* steps of spike log kept (0 = none) */
    int32_t ckpt_every;       /* adjoint checkpoint interval in steps; 0 = no adjoint */
    int64_t adjoint_steps;    /* longest forward window the adjoint covers */
    int32_t spin_limit_log2;  /* device wait limit, 2^k polls (0 = default 22) */
    int32_t steps_per_sync;   /* FP32: time steps per exchange of spikes, 1..min(d_min, 8) (0 = auto) */
    int32_t plan_kind;        /* FP32: CORTEX_PLAN_* */
    int32_t wg_per_cu;        /* FP32 resident plan: workgroups per compute unit, 1, 2, 4, 8 (0 = auto) */
    /* Spike-timing dependent plasticity (the E->E plasticity of the paper's
       verification network, Sec. IV-A) of the synapses whose source and
       target both belong to population stdp_pop (global index), when
       stdp_enable != 0.  FP32 weights and the streamed plan only; the
       exchange window is cut to at most n_ref + 1 steps, so that a source
       spikes at most once per window.  Rule (all-to-all pairing, every delay
       dendritic: a presynaptic spike at step q is at the synapse at q, a
       postsynaptic spike at step p reaches it at p + d; times in ms):
         x_j(t) = sum over spikes q' <= t of source j of exp(-(t - q') / tau_plus)
         y_i(t) = sum over spikes p < t of target i of exp(-(t - p) / tau_minus)
       When the spike of j at step q is delivered, each plastic synapse
       (j, i, d) takes, in ascending p, the spikes p of i with
       q_last < p + d <= q (q_last: j's previous spike):
         w <- min(w_max, w + lambda w0^(1 - mu) w^mu x_j(p + d))
       (x_j counting j's spikes up to q_last), then
         w <- max(0, w - lambda alpha w y_i(q - d)),
       and the spike is delivered with the new w.  A neuron keeps its last
       32 spikes for this; a synapse that would need an older one makes the
       call fail with CORTEX_ETRUNC.  w0 and w_max are in the weights' unit.
       cortex_reset keeps the weights. */
    int32_t stdp_enable;
    int32_t stdp_pop;
    double stdp_lambda, stdp_alpha, stdp_mu, stdp_tau_plus, stdp_tau_minus, stdp_w0, stdp_wmax;
    /* CORTEX_MODEL_COND, the conductance form of the synaptic current (Sec.
       I-A Eq. 3) with exponential conductances: a spike through a synapse of
       weight w (nS, native units only) adds |w| to the target's excitatory
       (w >= 0, reversal potential E_ex) or inhibitory (w < 0, E_in)
       conductance, each decaying with tau_syn;
         C dV/dt = -(C / tau_m)(V - E_L) + g_ex (E_ex - V) + g_in (E_in - V) + I_e.
       A step holds the conductances at their values at its start, for which
       the membrane's solution is exact (V relaxes towards the conductance-
       weighted mean of the reversal potentials with rate G / C); the step's
       arrivals then join the conductances (V feels them from the next step).
       External Poisson events enter the channel of w_ext's sign.  Resident
       plan with 64-bit rings (the two channels in two 32-bit halves); no
       plasticity and no adjoint. */
    double E_ex, E_in;
    /* FP32 streamed plan of one instance whose sources reach a tile through
       a few synapses each (segments shorter than 16): records per tile that
       a window copies from the graph into a tile-major run before its
       delivery (every record line then read once, instead of a line per
       spike and tile).  0 = automatic (a window at 50 Hz, the buffer within
       4 GiB), < 0 = no staging; a requested count is rounded up to a
       multiple of 4.  A window with more records for a tile delivers the
       excess straight from the graph; the sums are the same. */
    int64_t stage_records;
} cortex_spec;

/* Device memory and stream supplied by the caller.  alloc returns device
   memory of at least `bytes` bytes aligned to 256 (NULL on failure); free
   releases it.  With alloc == NULL the library uses hipMalloc/hipFree.
   stream is a hipStream_t (NULL = the null stream). */
typedef struct {
    void* stream;
    void* (*alloc)(size_t bytes, void* user);
    void (*free)(void* ptr, void* user);
    void* user;
} cortex_device;

typedef struct cortex_net cortex_net;

/* Passage: the graph G = (V, E) of Sec. II-A with its indegree sub-graphs
   (Eq. 5) over a partition of the neurons (Eq. 9-10), bound to their owners
   as in Sec. III-B (Fig. v_e_map_thread) and balanced by edge count
   (Sec. III-A, load balance); the populations, projections and neuron
   parameters are the problem description of Sec. II-B.
   Build a network from `spec` with Philox key (seed, instance): generates
   every synapse on the device, lays the graph out in indegree tiles and sets
   the initial state (step 0).  Synchronising.  *out receives the handle.
   Errors: EINVAL (bad spec), ENOMEM, EDEVICE, EUNSUPPORTED (e.g. input rings
   larger than the workgroup-local memory). */
int cortex_build_network(const cortex_spec* spec, uint64_t seed, const cortex_device* dev,
                         cortex_net** out);

/* Passage: the partition of the neurons into parts, one per owner (Eq.
   9-10), balanced by edge count (Sec. III-A, load balance), with every owner's
   input buffers in workgroup-local memory (Sec. III-B).
   The FP32 launch plan cortex_build_network would choose for `spec` on a
   device with n_cu compute units, lds_per_cu bytes of workgroup-local memory
   and threads_per_cu resident threads per compute unit, made on the host
   alone (no device call; register limits are not known, so a plan that
   fits here may still be refused by the device; normal delays are planned
   for their widest possible range).  Every plan is checked: the indices the
   kernels derive from it stay inside their arrays.  plan (host, n_plan
   entries, fewer are cut): plan kind, tiles, tile stride T, workgroup size,
   neurons per thread, steps per exchange W, ring slots, history slots, chunk,
   largest tile count of an instance, LDS bytes, ring element bytes, d_min,
   d_max, XCD map, one-thread-per-segment delivery, records per tile staged
   per window (0: none).  Errors: EINVAL,
   EUNSUPPORTED (no plan fits, or a plan failed its check). */
int cortex_plan(const cortex_spec* spec, int32_t n_cu, int64_t lds_per_cu, int32_t threads_per_cu,
                int64_t* plan, int32_t n_plan);

/* Passage: the simulation step of Sec. II-B (Fig.
   brain_simulation_procedure (d)): synapses of spiking sources act on their
   targets after each synapse's delay, then every neuron advances by the LIF
   dynamics of Eq. 1 with threshold, reset and refractory period (Eq. 2);
   only the spiking sub-graph (Eq. 11) of each owner is read.  Spikes are
   exchanged once per window of steps no longer than the smallest delay, the
   buffered-spike overlap of Sec. III-C.
   Advance the simulation by n_steps (closed loop: spikes from threshold
   crossings).  Asynchronous on the network's stream.  FP32 networks run one
   persistent launch; the spike log keeps steps inside the record window.
   Errors: EINVAL (n_steps < 0), ESTATE (network failed earlier), EDEVICE,
   ETIMEOUT (reported by the next synchronising call). */
int cortex_step(cortex_net* net, int64_t n_steps);

/* Passage: the spike buffer of Sec. III-C (spikes broadcast and buffer),
   read back as (step, neuron) pairs.
   Spikes with step in [step0, step1) from the log, sorted by (step, id),
   into host arrays of `capacity` entries; *count = number of spikes in the
   range.  Returns ETRUNC if capacity < *count (the first `capacity` are
   written) or if the range leaves the record window.  Synchronising. */
int cortex_get_spikes(cortex_net* net, int64_t step0, int64_t step1, uint32_t* steps,
                      uint32_t* ids, int64_t capacity, int64_t* count);

/* Passage: the spike buffer of Sec. III-C.
   Restart the spike log window at the current step. */
int cortex_clear_spikes(cortex_net* net);

/* Passage: the step of Sec. II-B with the spiking set of each step given
   instead of computed (the spiking sub-graph of Eq. 11 taken from a
   raster), so that delivery is a linear function of the weights.
   Open loop with spikes frozen to a raster (host arrays, sorted by (step,
   id), absolute steps): advance n_steps; a neuron spikes and resets exactly at
   its raster entries, thresholds are not evaluated, and delivery uses the
   raster.  Optional device traces [n_steps][N] (float in FP32 mode, double in
   FP64 mode): x = synaptic input consumed at each step, v = membrane
   potential after the step.  Synchronising. */
int cortex_run_frozen(cortex_net* net, const uint32_t* r_steps, const uint32_t* r_ids,
                      int64_t n_spikes, int64_t n_steps, void* x_trace, void* v_trace);

/* Passage: the exact integration of Eq. 1 between spikes (linear in the
   synaptic input) and the delivery of Sec. II-B over the indegree
   sub-graphs of Eq. 5: with spikes frozen, V is affine in the weights, and
   the gradient is the transpose of delivery over the same spiking
   sub-graph (Eq. 11), one writer per synapse as in Sec. III-B.
   Gradient of L = sum_b 1/(N_b T) sum_{i in b, n < T} (V_i(n) - V*_i(n))^2
   over the T steps simulated since the build (or the last cortex_reset),
   with every neuron's spikes frozen to the ones it emitted, with respect to
   all stored synaptic weights (native units).  Requires spec.ckpt_every > 0
   and T <= spec.adjoint_steps.  vstar: device float [T][N]; grad_w: device
   float [E] in canonical synapse order (overwritten); *loss (host) gets L.
   Synchronising.  Errors: ESTATE (adjoint not enabled / window too long). */
int cortex_backward(cortex_net* net, const float* vstar, float* grad_w, double* loss);

/* Passage: the synaptic weights W of Eq. 3 (current form), one per edge of
   G (Sec. II-A), stored inside their target's indegree sub-graph (Eq. 5).
   Replace every stored synaptic weight (native units; FP32 networks with
   spec.ckpt_every > 0, at step 0, i.e. after the build or cortex_reset):
   w_canonical is a device float [E] in canonical synapse order (caller
   owned, read only).  Weights are stored in the network's weight format and
   the input rings' fixed-point scale is recomputed from the new weights, so
   the sums stay exact for any weights.  This and cortex_backward let a caller
   run the adjoint on weights it chooses (e.g. a training loop).  Errors:
   ESTATE (not at step 0, or no canonical order without ckpt_every),
   EUNSUPPORTED (FP64 networks), EINVAL (NULL). */
int cortex_set_weights(cortex_net* net, const float* w_canonical);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc):
   cortex_run_frozen without any device allocation.  Same arguments, results
   and errors as cortex_run_frozen, FP32 networks only (EUNSUPPORTED for
   FP64).  The raster and its per-step list offsets go to a fixed device
   array of 32 MiB held by the library on each GPU until the process ends;
   (n_steps x tiles + 1) x 8 + n_spikes x 8 bytes (each part rounded up to 256)
   must fit it, else EINVAL.  Every call on a GPU shares that GPU's array:
   calls that overlap on one GPU race.  Synchronising. */
int cortex_run_frozen_noalloc(cortex_net* net, const uint32_t* r_steps, const uint32_t* r_ids,
                              int64_t n_spikes, int64_t n_steps, void* x_trace, void* v_trace);

/* Passage: the initial state of the simulation of Sec. II-B.
   Back to the build-time state (step 0, empty input rings, empty log). */
int cortex_reset(cortex_net* net);

/* Passage: the state of the LIF neuron of Eq. 1-2 (membrane potential,
   refractory clock) and of its current synapse (Eq. 3, current form).
   Neuron state into host arrays of N entries (V in mV; r = refractory steps
   left; y1/y2 synaptic state as in the oracle: exp y1 = current; alpha y1 =
   auxiliary, y2 = current); NULL skips an array.  Synchronising. */
int cortex_get_state(cortex_net* net, double* V, int32_t* r, double* y1, double* y2);

/* Passage: the state of the simulation of Sec. II-B between two time steps
   (the neurons of Eq. 1-2, the delayed inputs of Sec. III-B not yet
   consumed, the spikes still to be delivered, Sec. III-C).
   Checkpoint and resume of a network: cortex_state_size gives the bytes of
   its complete dynamic state (neuron and synapse state, input rings,
   pending spikes, cached Poisson counts, spike log and counters, and with
   plasticity the synapse records with their weights, the traces and the
   spike histories; in FP64 verify mode the state, the recent spike bits and
   the record window; the rest of the graph is rebuilt from the spec and
   seed); cortex_save_state copies it into a caller-owned host buffer of at
   least that size; cortex_load_state restores it into a network built from
   the same spec and seed with the same plan, which then continues exactly
   as the saved one would have (same spikes, same state, bit for bit).
   Synchronising.  Errors: EUNSUPPORTED (networks with the adjoint enabled),
   EINVAL (NULL, a buffer too small, a state saved by a network of another
   spec, seed or plan). */
int cortex_state_size(cortex_net* net, int64_t* bytes);
int cortex_save_state(cortex_net* net, void* host, int64_t bytes);
int cortex_load_state(cortex_net* net, const void* host, int64_t bytes);

/* Passage: the edges E of Sec. II-A as triplets (source, target, weight)
   plus the delay, stored per source and per owning tile (the segments of
   the spiking sub-graph, Eq. 11; Sec. III-B, Fig. data_ins).
   All synapses into host arrays of E entries, in the library's storage
   order (grouped by source, then tile).  Global ids; delay in steps; weight
   as stored, widened to double.  Synchronising. */
int cortex_export_graph(cortex_net* net, int64_t* src, int64_t* tgt, double* w, int32_t* d);

/* Passage: the bijection between stored and canonical edges that makes
   the indegree sub-graphs a partition of E (Eq. 8).
   Canonical index of every stored synapse (host int64[E], storage order),
   so export order can be mapped to canonical order. Synchronising. */
int cortex_export_canonical(cortex_net* net, int64_t* canon);

/* Passage: the partition of V into disjoint parts V_1 ... V_n (Eq. 9-10),
   one per owner.
   Tile table into host arrays of n_tiles entries: first global target,
   number of targets, instance.  Synchronising. */
int cortex_export_tiles(cortex_net* net, int64_t* start, int32_t* size, int32_t* instance);

enum {
    CORTEX_Q_NEURONS = 0,
    CORTEX_Q_SYNAPSES = 1,
    CORTEX_Q_MIN_DELAY = 2,
    CORTEX_Q_MAX_DELAY = 3,
    CORTEX_Q_TILES = 4,
    CORTEX_Q_TILE_SIZE = 5,
    CORTEX_Q_RING_SLOTS = 6,
    CORTEX_Q_STEP = 7,            /* current step */
    CORTEX_Q_EVENTS = 8,          /* synaptic events delivered since build/reset */
    CORTEX_Q_SPIKES = 9,          /* spikes emitted since build/reset */
    CORTEX_Q_DEVICE_BYTES = 10,   /* device memory held */
    CORTEX_Q_EDGE_BYTES = 11,     /* bytes of one stored synapse record */
    CORTEX_Q_BLOCK_SIZE = 12,
    CORTEX_Q_LDS_BYTES = 13,      /* workgroup-local memory per workgroup */
    CORTEX_Q_OFFSET_BYTES = 14,   /* bytes of the per-(source, tile) offset table */
    CORTEX_Q_STEPS_PER_SYNC = 15, /* FP32: time steps per spike exchange chosen at build */
    CORTEX_Q_RING_BYTES = 16,     /* FP32: bytes of one input-ring element (8: 64-bit, 4: 32-bit sums) */
    CORTEX_Q_PLAN = 17,           /* FP32: CORTEX_PLAN_RESIDENT or CORTEX_PLAN_STREAMED */
    CORTEX_Q_NPT = 18,            /* FP32: neurons per thread */
    CORTEX_Q_STAGE_RECORDS = 19,  /* FP32 streamed: records per tile staged per window (0: none) */
    CORTEX_Q_STAGE_GROUP = 20     /* FP32 streamed with staging: tiles per copy work item (0: no staging) */
};
/* Passage: the sizes of G (Sec. II-A) and of its decomposition (Eq. 9-10);
   EVENTS counts the edges of the spiking sub-graphs (Eq. 11) delivered.
   Scalar facts about the network into *value.  EVENTS and SPIKES
   synchronise. */
int cortex_query(cortex_net* net, int what, int64_t* value);

/* Passage: none (measurement of the kernels of Sec. III-B's delivery).
   FP32 streamed plan: live timing of the window launches.  on != 0 clears
   the sums and makes the staging copy (if the plan stages) and the delivery
   launch of every window stamp the device clock as they start (one thread
   each); the interval from a launch's stamp to the next launch's is its
   duration plus the gap before the next one.  on == 0 stops it.
   cortex_kernel_times synchronises and writes the mean interval in
   milliseconds since the last cortex_kernel_timing(net, 1) of the staging
   copy (0 without staging) into ms[0] and of the delivery launch into ms[1]
   (which includes a plasticity pass, if any); *n_windows = the delivery
   launches counted.  Errors: EUNSUPPORTED (not a streamed FP32 network),
   EINVAL (NULL). */
int cortex_kernel_timing(cortex_net* net, int on);
int cortex_kernel_times(cortex_net* net, double* ms, int32_t* n_windows);

/* Passage: none (resource management).
   Release the network and its device memory.  NULL is ignored. */
void cortex_destroy(cortex_net* net);

/* Passage: none (error reporting).
   Message of the last failure on the calling thread (never NULL). */
const char* cortex_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
