// Internal declarations shared by the translation units of libcortex.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cortex.h"

namespace cortex {

// Error reporting -----------------------------------------------------------
void set_error(const std::string& msg);

struct Error {
    int status;
    std::string msg;
};

#define CX_HIP(expr)                                                                \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            throw ::cortex::Error{CORTEX_EDEVICE, std::string(#expr) + ": " +       \
                                                      hipGetErrorString(e_)};       \
    } while (0)

inline void require(bool ok, int status, const std::string& msg) {
    if (!ok) throw Error{status, msg};
}

// Model constants (host, FP64) ----------------------------------------------
struct Consts {
    double P22, P20, P11, P21, P31, P32, P21s, P22s, jump, conv;
    int n_ref;
};
Consts model_constants(const cortex_spec& s);
int poisson_thresholds(double lambda, uint32_t* thr, int cap);

// Generation tables ----------------------------------------------------------
// One "block" is a (target population, projection) pair: every target of the
// population draws the projection's synapses.  Blocks are listed in
// canonical order inside a population: projections ascending.
struct GenBlock {
    int64_t tgt0;        // first global target of the population
    int64_t n_tgt;       // population size
    int64_t inst_n0;     // first global neuron of the instance
    int64_t src0_local;  // first source (instance-local id)
    int64_t n_src;
    int64_t k;           // fixed in-degree
    uint64_t thr_p;      // pairwise threshold p*2^64
    double w_mean, w_sd;
    double d0, d1;
    int32_t rule, delay_kind;
    int32_t same_pop_no_autapse;
    int32_t proj_local;  // projection index within the instance
    int32_t instance;
    int32_t all_pairs;   // pairwise with p >= 1
    int64_t tgt0_in_pop; // offset of tgt0 inside its population (0)
    int32_t slot_base;   // canonical offset of this projection within a target (fixed-k only)
    int32_t pad;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Live timing of the window launches by the launches themselves (constant-
// rate device clock): thread 0 of workgroup 0 of each timed launch (the
// first dispatched) reads the clock at its start, which closes the previous
// timed launch's interval on the same stream; launches on one stream run one
// after another, so an interval is the launch's duration and the gap to the
// next launch.  One thread per launch: no contention.
struct KernelTime {
    unsigned long long last_t;     // start of the last timed launch (0: none yet)
    unsigned long long sum[2];     // summed intervals: [0] staging copy, [1] delivery launch
    unsigned long long count[2];
    int last_kind, pad;
};
// What the planner needs to know of the device: compute units, LDS bytes and
// resident threads per compute unit, and whether kernel occupancy can be
// asked of the runtime (a live device) or must be estimated from LDS and
// threads alone (host-only planning).
struct DeviceDesc {
    int n_cu = 256;
    size_t lds_cu = 163840;
    int thr_cu = 2048;
    bool live = false;
};

}  // namespace cortex

// Network object ----------------------------------------------------------------
struct cortex_net {
    cortex_spec spec{};
    std::vector<cortex_pop> pops;
    std::vector<cortex_proj> projs;
    cortex_device dev{};
    hipStream_t stream = nullptr;
    int device = 0;
    uint64_t seed = 0;
    bool failed = false;
    cortex::Consts k{};
    uint32_t thr[64] = {};
    int n_thr = 0;
    double w_ext_native = 0;

    // sizes
    int64_t N = 0, E = 0;
    int n_inst = 0;
    std::vector<int64_t> inst_n0, inst_N;
    std::vector<int32_t> inst_tile0, inst_ntiles;
    std::vector<uint64_t> inst_offbase;     // start of the instance's off_rel block
    int n_tiles = 0, T = 0, BS = 512, NPT = 1;   // T: largest tile (LDS and buffer stride)
    std::vector<int32_t> inst_T;                 // tile size of each instance
    std::vector<int64_t> tile_start;
    std::vector<int32_t> tile_size, tile_inst;
    int dmin = 1, dmax = 1, R = 1, H = 64;
    int W = 1, chunk = 1024, ntb_max = 1;   // steps per spike exchange, staged spikes, tiles per instance
    int meta_bytes = 2, w_bytes = 4;    // record: (delay - dmin) T + target in tile
    size_t lds_bytes = 0;
    int xcd_map = 0;
    int plan_kind = CORTEX_PLAN_RESIDENT;   // resolved plan (never AUTO)
    int64_t step = 0;
    std::vector<cortex::GenBlock> blocks;

    // record window
    int64_t log_step0 = 0, log_steps = 0;

    // device memory
    std::vector<cortex::DevBuf> bufs;
    std::vector<cortex::DevBuf> scratch;
    size_t dev_bytes = 0;
    // tables
    int64_t* d_tile_start = nullptr;
    int32_t* d_tile_size = nullptr;
    int32_t* d_tile_inst = nullptr;
    int32_t* d_inst_tile0 = nullptr;
    int32_t* d_inst_ntiles = nullptr;
    int32_t* d_inst_T = nullptr;
    int64_t* d_inst_n0 = nullptr;
    uint64_t* d_inst_offbase = nullptr;
    // production graph
    uint64_t* d_row_start = nullptr;   // [N+1]
    uint32_t* d_off_rel = nullptr;     // [sum_b N_b (nt_b + 1)]
    uint64_t* d_seg = nullptr;         // same index: (first synapse << 24) | length of segment (source, tile)
    void* d_meta = nullptr;            // u16/u32 [E]
    void* d_w = nullptr;               // f32/bf16 [E]
    uint32_t* d_canon = nullptr;       // [E] canonical index of each stored synapse (adjoint)
    uint64_t* d_cin = nullptr;         // [N + 1] first canonical synapse of each target (adjoint)
    uint32_t* d_csrc = nullptr;        // [E] source of each canonical synapse (adjoint)
    uint16_t* d_cdel = nullptr;        // [E] delay in steps of each canonical synapse (adjoint)
    // FP32 state
    float *d_U = nullptr, *d_y1 = nullptr, *d_y2 = nullptr;
    int32_t* d_r = nullptr;
    void* d_ring = nullptr;            // [n_tiles][R][T] fixed-point input sums (ring_bytes each)
    int ring_bytes = 8;                // 8: 64-bit sums; 4: 32-bit sums when 64-bit rings do not fit
    int fx = 32;                       // fixed-point fraction bits of the rings
    int fx_shift = 0;                  // weights are rounded at 2^(fx - fx_shift), then shifted
    uint64_t* d_pub = nullptr;         // [H][n_tiles][T + 1] tagged spike records
    uint32_t* d_log_cnt = nullptr;     // [log_steps][n_tiles]
    uint32_t* d_log_ids = nullptr;
    uint64_t* d_log_base = nullptr;    // [n_tiles + 1]
    uint64_t* d_log_pos = nullptr;     // [n_tiles]
    uint64_t* d_events = nullptr;      // [n_tiles]
    uint64_t* d_spikes = nullptr;      // [n_tiles]
    int32_t* d_err = nullptr;          // [4]
    // streamed plan: per-step spike lists, device clock, workgroup order
    uint32_t* d_spk_cnt = nullptr;     // [H][n_inst]
    uint32_t* d_spk_ids = nullptr;     // [H][N]
    int64_t* d_clock = nullptr;        // [2]
    int32_t* d_order = nullptr;        // [n_tiles]
    std::vector<int32_t> order;        // streamed plan: tile of each workgroup
    cortex::DeviceDesc dd;
    int clock_parity = 0;
    int thread_segments = 0;           // streamed delivery with one thread per (short) segment
    // tile-major staging of each window's records (streamed plan, short
    // segments, one instance): records per tile (0: no staging)
    uint32_t stage_cap = 0;
    int stage_group = 16;                    // tiles per copy work item (a power of two, at most 16)
    void* d_stage = nullptr;                 // [n_tiles][stage_cap] records
    unsigned long long* d_cursor = nullptr;  // [n_tiles] records staged for the coming delivery
    unsigned long long* d_kcache = nullptr;  // streamed plan, [N]: Poisson counts of one 8-step block
    bool use_graph = true;
    // plasticity (streamed plan): per (source, tile) segment the presynaptic
    // trace just after the source's last spike and that spike's step + 1
    // (0: none); per neuron the steps and traces of its last kHistLen
    // spikes; per tile the first step not yet in its targets' histories
    bool stdp = false;
    int64_t stdp_lo = 0, stdp_hi = 0;     // plastic population, global ids [lo, hi)
    double stdp_c = 0, stdp_lam_alpha = 0, stdp_mu = 0, stdp_tp = 0, stdp_tm = 0, stdp_wmax = 0;
    uint64_t n_seg = 0;                   // entries of d_seg
    uint64_t* d_seg_state = nullptr;      // [n_seg] float x | (q + 1) << 32
    int32_t* d_hist_step = nullptr;       // [N][kHistLen]
    float* d_hist_y = nullptr;            // [N][kHistLen]
    uint32_t* d_hist_cnt = nullptr;       // [N] spikes recorded so far
    int64_t* d_hist_upto = nullptr;       // [n_tiles]
    hipGraphExec_t graph_exec = nullptr;   // kGraphWindows window launches
    hipStream_t graph_stream = nullptr;    // library stream the graph is captured on and replayed on
    hipEvent_t fence_in = nullptr, fence_out = nullptr;   // order it after / before the caller's stream
    // per-kernel timing of the window launches (cortex_kernel_timing):
    // [0] staging copy, [1] delivery launch
    bool ktiming = false;
    cortex::KernelTime* d_ktime = nullptr;
    int64_t graph_log_step0 = -1, graph_log_steps = -1;
    bool graph_ktiming = false;
    // initial state copy (reset / adjoint)
    float *d_U0 = nullptr;
    // FP64 verify graph and state
    uint64_t* d_in_ptr = nullptr;      // [N+1]
    uint32_t* d_in_src = nullptr;
    double* d_in_w = nullptr;
    uint16_t* d_in_d = nullptr;
    uint32_t* d_in_canon = nullptr;
    double *d_Ud = nullptr, *d_y1d = nullptr, *d_y2d = nullptr;
    double* d_Ud0 = nullptr;
    uint64_t* d_raster = nullptr;      // [log_steps][W] spike bits of the record window
    uint64_t* d_hist = nullptr;        // [H][W] spike bits of the last H steps
    int64_t raster_steps = 0;
    int64_t W64 = 0;
    double events_fp64 = 0;

    // adjoint: checkpoints of (U, y1, y2, r) and the rings every ckpt steps
    int ckpt = 0;
    int64_t adj_steps = 0;
    int n_ckpt = 0;
    float* d_ck_U = nullptr;           // [n_ckpt][N]
    float* d_ck_y1 = nullptr;
    float* d_ck_y2 = nullptr;
    int32_t* d_ck_r = nullptr;
    unsigned char* d_ck_ring = nullptr;   // [n_ckpt][n_tiles][R][T] ring elements
};

namespace cortex {
void* dev_alloc(cortex_net* n, size_t bytes, bool scratch = false);
void free_scratch(cortex_net* n);
// Release the scratch buffers allocated after the first `mark` ones (waits
// for the stream first).
void free_scratch_from(cortex_net* n, size_t mark);
void dev_zero(cortex_net* n, void* p, size_t bytes);
template <class T>
T* dev_alloc_t(cortex_net* n, size_t count, bool scratch = false) {
    return static_cast<T*>(dev_alloc(n, count * sizeof(T) + (count == 0 ? 16 : 0), scratch));
}

// Kernel launchers (graph.hip) -----------------------------------------------
void delay_range(cortex_net* n, int* dmin, int* dmax);
void build_graph_fp32(cortex_net* n);
// Largest sum of |w| over the stored in-synapses of any neuron (after
// build_graph_fp32); *wmax (if not NULL) gets the largest single |w|.
double max_abs_input(cortex_net* n, double* wmax = nullptr);
// Stored weights from a device array in canonical synapse order.
void set_weights_fp32(cortex_net* n, const float* w_canonical);
void build_graph_fp64(cortex_net* n);
void init_state(cortex_net* n);
// step.hip
// Frozen runs pass the per-(step, tile) id lists (frz_ptr into frz_ids,
// frz_n ids in all); the kernel clamps every list to [0, frz_n).
// out[k] = in[0] + ... + in[k - 1] for k <= count (graph.hip; one workgroup,
// on n->stream; setup-sized counts).
void scan_counts(cortex_net* n, const uint32_t* in, uint64_t* out, int64_t count);
// Offsets of a raster sorted by (step, id) (noalloc.hip): ptr[s * n_keys + k]
// = first entry with (step, id) >= (step0 + s, keys[k]), and ptr[n_steps *
// n_keys] = first entry past step0 + n_steps; on n->stream.
void raster_index(cortex_net* n, const uint32_t* steps, const uint32_t* ids, int64_t n_spk, int64_t step0,
                  int64_t n_steps, const int64_t* keys, int n_keys, uint64_t* ptr);
// Rejects (EINVAL) a frozen raster in which a plastic neuron spikes twice
// within its refractory period (api.hip).
void check_plastic_raster(const cortex_net* n, const uint32_t* st, const uint32_t* id, int64_t ns);
// Plasticity pass of one window of the streamed plan (stdp.hip): on `stream`,
// before the window's delivery launch with the same clock parity and length.
void launch_stdp(cortex_net* n, int parity, int wn, hipStream_t stream);
void launch_gather(cortex_net* n, int parity, int wn, hipStream_t stream);
void gather_prepare(cortex_net* n);
// records of rec_bytes each that one copy work item can hold in workgroup-local memory
int gather_out_records(int rec_bytes);
void launch_step_fp32(cortex_net* n, int64_t n_steps, const uint32_t* frz_ids,
                      const uint64_t* frz_ptr, uint64_t frz_n, float* x_trace, float* v_trace,
                      uint8_t* m_trace = nullptr);
// adjoint.hip
void adjoint_backward(cortex_net* n, const float* vstar, float* grad_w, double* loss);
void republish(cortex_net* n, int64_t q0, int64_t q1, const uint32_t* ids, const uint64_t* ptr,
               uint64_t n_ids);
size_t step_lds_bytes(int R, int T, int W, int ntiles_max, int chunk, int ring_bytes);
// stream.hip: window launches of the streamed plan
constexpr int kGraphWindows = 32;


__device__ inline void ktime_mark(KernelTime* kt, int kind) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const unsigned long long t = wall_clock64();
    const unsigned long long p = kt->last_t;
    if (p != 0) {
        kt->sum[kt->last_kind] += t - p;
        kt->count[kt->last_kind] += 1;
    }
    kt->last_t = t;
    kt->last_kind = kind;
}
constexpr int kHistLen = 32;   // postsynaptic spikes a neuron keeps for plasticity   // window launches per captured graph (even)
size_t stream_lds_bytes(int R, int T, int W, int chunk);
int stream_occupancy(int model, int meta_bytes, int w_bytes, int npt, int bs, size_t lds);
void launch_stream_fp32(cortex_net* n, int64_t n_steps, const uint32_t* frz_ids, const uint64_t* frz_ptr,
                        uint64_t frz_n, float* x_trace, float* v_trace, uint8_t* m_trace = nullptr);
int step_max_blocks_per_cu(cortex_net* n);
// Resident workgroups per CU of the step kernel variant for a model, record
// format, neurons per thread, workgroup size and LDS bytes (0 if none fit).
int step_occupancy(int model, int meta_bytes, int w_bytes, int npt, int bs, size_t lds, int ring_bytes);
// api.hip: advance an FP32 network by n_steps (frozen lists and traces
// indexed from its current step; launches split at adjoint checkpoints), and
// raise CORTEX_ETIMEOUT if a device-side wait failed (synchronising)
void advance_fp32(cortex_net* n, int64_t n_steps, const uint32_t* frz_ids, const uint64_t* frz_ptr,
                  uint64_t frz_n, float* x_trace, float* v_trace);
void check_device_flag(cortex_net* n);
// verify.hip
void launch_step_fp64(cortex_net* n, int64_t n_steps, const uint64_t* frz_bits,
                      double* x_trace, double* v_trace);
}  // namespace cortex
