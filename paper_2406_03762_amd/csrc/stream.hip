// Streamed FP32 step: one kernel launch per window of W <= d_min steps over
// all tiles, for networks whose input rings do not all fit the workgroup-local
// memory of the chip at once (e.g. two million neurons with 26 delay values:
// 240 MB of rings against 40 MB of LDS).
//
// Each workgroup takes one tile for one window: it stages the tile's input
// ring (R slots x T targets, 32-bit fixed point) and neuron state from HBM,
// delivers the spikes of steps [t0 - d_min, t0 - d_min + W) of its instance
// into the ring (the same segment layout as the persistent kernel: the
// spiking part, Eq. 11, of the tile's indegree sub-graph, Eq. 5), advances
// its neurons through the W steps, appends their spikes to the per-step
// spike lists and writes ring and state back.  The tile is still the only
// writer of its targets' input (Sec. III-B), so delivery needs no global
// atomic; the kernel boundary replaces the persistent kernel's spin waits
// (every spike a window delivers was emitted by an earlier launch, as
// W <= d_min), and a run is a sequence of window launches that a captured
// HIP graph replays.
//
// Per step and instance, the spike list has one counter (spikes appended so
// far, one atomic reservation per tile and step) and room for every neuron of
// the instance; H >= d_min + 2 W list slots cycle.  The first workgroup of a
// launch clears the counters of the next window's slots, which no workgroup
// of the launch reads or writes.
//
// The window start t0 lives in device memory (clock[parity]); the first
// workgroup writes the next window's start into clock[1 - parity], so a
// captured sequence of launches can be replayed without new arguments.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "deliver.hpp"
#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

constexpr int kMaxThr = 32;   // Poisson table entries in kernel arguments
constexpr int kMaxW = 8;      // steps per window

struct StreamArgs {
    const int32_t* order;          // [n_tiles] tile of each workgroup
    const int32_t* tile_inst;
    const int32_t* tile_size;
    const int32_t* inst_tile0;
    const int32_t* inst_ntiles;
    const int32_t* inst_T;
    const int64_t* inst_n0;
    const uint64_t* inst_offbase;
    const uint64_t* seg;           // (first synapse << 24) | length per (source, tile)
    const void* meta;
    const void* w;
    float* U;
    float* y1;
    float* y2;
    int32_t* r;
    unsigned long long* kcache;    // per neuron: Poisson counts of one 8-step block (see block_counts)
    int32_t* ring;                 // [n_tiles][R][T] 32-bit fixed-point sums
    uint32_t* spk_cnt;             // [H][n_inst] spikes per step and instance
    uint32_t* spk_ids;             // [H][N] their ids (instance b at offset inst_n0[b])
    int64_t* clock;                // [2] window starts
    uint32_t* log_cnt;
    uint32_t* log_ids;
    const uint64_t* log_base;
    uint64_t* log_pos;
    uint64_t* events;
    uint64_t* spikes;
    const uint32_t* frz_ids;
    const uint64_t* frz_ptr;       // [(step - frz_step0) * n_tiles + tile]
    uint64_t frz_n;
    int64_t frz_step0;
    float* x_trace;                // [(step - trace_step0) * N + neuron]
    float* v_trace;
    uint8_t* m_trace;
    int64_t trace_step0;
    const void* stage;             // staged records [n_tiles][stage_cap] (null: no staging)
    unsigned long long* cursor;    // [n_tiles] records staged for this window (reset here)
    KernelTime* ktime;             // launch timing (null: off)
    uint32_t stage_cap;
    int64_t log_step0, log_steps, N;
    int parity, wn;
    int thread_segments;           // segments of a few synapses: one thread per segment
    int n_tiles, n_inst, T, R, dmin, H, W, chunk, n_ref, n_thr;
    float P22, P20Ie, P11, P21, P31, P32, P21s, P22s, jump, theta, Ur, w_ext, E_L;
    float fxw_scale;
    double fx_inv;
    uint64_t seed;
    uint32_t thr[kMaxThr];
};

}  // namespace

// Bytes of workgroup-local memory of the streamed kernel; the kernel carves
// its arrays in this order.
size_t stream_lds_bytes(int R, int T, int W, int chunk) {
    size_t b = (size_t)chunk * 16;                 // s_sg: segment descriptors
    b += (size_t)R * T * 4;                        // ring
    b += (size_t)(chunk + 1) * 4;                  // s_len: segment prefix
    b += ((size_t)W * T * 2 + 3) & ~(size_t)3;     // s_spk: local ids of each step's spikes
    b += (size_t)T * 4;                            // s_frz: frozen-spike bits
    b += (size_t)kDeliverBlk * 4;                  // s_blk
    b += (size_t)kMaxThr * 4;                      // s_thr
    b += (size_t)(kMaxW + 1) * 4;                  // s_pc: spikes per delivered step (prefix)
    b += (size_t)kMaxW * 4;                        // s_cnt: spikes per updated step
    b += (size_t)20 * 4 + 20 * 4 + 8 * 4;          // s_wsum, s_kw, s_misc
    return (b + 15) & ~(size_t)15;
}

namespace {

// Poisson counts of one 8-step block (neuron nl, steps 8 blk .. 8 blk + 7):
// step 8 blk + sub takes the 32-bit half (sub & 1) of word sub >> 1 of the
// Philox block (nl, blk, 0, Poisson tag); its count is the number of the
// (increasing) thresholds at or below it, found by a binary search of the
// table in workgroup-local memory.  6 bits per step, step sub at bit 6 sub.
// A cache entry holds such a block's counts (48 bits) and, in its top 16
// bits, the block's index + 1 modulo 2^16 (0: empty); the entry is rewritten
// at least every second window, so a stale entry never matches.
constexpr unsigned long long kCountsMask = (1ull << 48) - 1;

__device__ __forceinline__ uint64_t block_counts(uint64_t nl, uint64_t blk, const uint32_t* s_thr, int n_thr,
                                                 uint64_t seed, uint64_t inst) {
    const Philox4 p = philox(nl, blk, 0, kTagPoisson, seed, inst);
    uint64_t packed = 0;
#pragma unroll
    for (int sub = 0; sub < 8; ++sub) {
        const uint64_t word = p.v[sub >> 1];
        const uint32_t u = (sub & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
        int kc = 0;
#pragma unroll
        for (int h = kMaxThr; h > 0; h >>= 1) {
            // (no branch: the 8 searches of a block interleave)
            const uint32_t t = s_thr[min(kc + h, kMaxThr) - 1];
            kc += (kc + h <= n_thr && t <= u) ? h : 0;
        }
        packed |= (uint64_t)kc << (6 * sub);
    }
    return packed;
}

__device__ __forceinline__ bool kcache_holds(unsigned long long e, uint64_t blk) {
    return (e >> 48) == ((blk + 1) & 0xFFFFull);
}

__device__ __forceinline__ unsigned long long kcache_entry(uint64_t blk, uint64_t counts) {
    return (((blk + 1) & 0xFFFFull) << 48) | (counts & kCountsMask);
}

// Data a launch touches once, in streams (the staged run, the ring rows
// staged in and written back, the neurons' state), are loaded and stored
// with the non-temporal hint (the instructions' nt bit), so that they do not
// push more reused lines out of the caches.  Measured on the two-million-
// neuron net: the delivery launch 0.203 -> 0.183 ms, the next staging copy
// 0.189 -> 0.181 ms.
typedef int32_t i32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 load_stream(const int4* p) {
    const i32x4_t q = __builtin_nontemporal_load(reinterpret_cast<const i32x4_t*>(p));
    return make_int4(q.x, q.y, q.z, q.w);
}
__device__ __forceinline__ uint4 load_stream(const uint4* p) {
    const int4 q = load_stream(reinterpret_cast<const int4*>(p));
    return make_uint4((uint32_t)q.x, (uint32_t)q.y, (uint32_t)q.z, (uint32_t)q.w);
}
__device__ __forceinline__ void store_stream(int4* p, int4 v) {
    i32x4_t q;
    q.x = v.x;
    q.y = v.y;
    q.z = v.z;
    q.w = v.w;
    __builtin_nontemporal_store(q, reinterpret_cast<i32x4_t*>(p));
}

// Staged records (gather.hip): u32 words (16-bit record with the bf16
// weight in the high half) or {record, fp32 weight bits}.
template <bool WBF16>
using StagedRec = typename std::conditional<WBF16, uint32_t, uint2>::type;

template <bool WBF16>
__device__ __forceinline__ void staged_add(const StreamArgs& a, int32_t* ring, StagedRec<WBF16> r, bool use,
                                           uint32_t row0, uint32_t RT) {
    uint32_t m;
    float wv;
    if constexpr (WBF16) {
        m = r & 0xFFFFu;
        wv = __uint_as_float(r & 0xFFFF0000u);
    } else {
        m = r.x;
        wv = __uint_as_float(r.y);
    }
    uint32_t x = m + row0;
    x = min(x, x - RT);
    if (use) ring_add(ring, x, __float2int_rn(wv * a.fxw_scale));
}

// The tile's n_st staged records, in any order, each with its ring row
// relative to the window's first delivered step, read as 16-byte pieces (4
// bf16 records or 2 fp32 records; the run starts 16-byte aligned because the
// capacity per tile is a multiple of 4 records): every thread takes pieces
// tid, tid + bs, ..., kStageU at a time, so that a workgroup has kStageU x 16
// bytes per thread in flight.  Clamped indices keep the loads free of
// branches; the records of a clamped piece, and those past n_st in the last
// piece (which lies inside the tile's capacity), are not added.
constexpr int kStageU = 12;   // 48K records per 1024-thread pass: a tile's run (44K on average at 7 Hz) in one

template <bool WBF16>
__device__ __forceinline__ void deliver_staged(const StreamArgs& a, int32_t* ring, uint32_t n_st, int tile,
                                               int base_slot, uint32_t T, uint32_t RT, int tid, int bs) {
    constexpr uint32_t PER = WBF16 ? 4u : 2u;
    const uint4* run =
        reinterpret_cast<const uint4*>(static_cast<const StagedRec<WBF16>*>(a.stage) + (size_t)tile * a.stage_cap);
    const uint32_t row0 = (uint32_t)base_slot * T;
    const uint32_t np = (n_st + PER - 1) / PER;
    for (uint32_t i0 = (uint32_t)tid; i0 < np; i0 += kStageU * (uint32_t)bs) {
        uint4 r[kStageU];
#pragma unroll
        for (int u = 0; u < kStageU; ++u) r[u] = load_stream(&run[min(i0 + (uint32_t)(u * bs), np - 1)]);
#pragma unroll
        for (int u = 0; u < kStageU; ++u) {
            const uint32_t first = (i0 + (uint32_t)(u * bs)) * PER;
            if constexpr (WBF16) {
                staged_add<true>(a, ring, r[u].x, first < n_st, row0, RT);
                staged_add<true>(a, ring, r[u].y, first + 1 < n_st, row0, RT);
                staged_add<true>(a, ring, r[u].z, first + 2 < n_st, row0, RT);
                staged_add<true>(a, ring, r[u].w, first + 3 < n_st, row0, RT);
            } else {
                staged_add<false>(a, ring, make_uint2(r[u].x, r[u].y), first < n_st, row0, RT);
                staged_add<false>(a, ring, make_uint2(r[u].z, r[u].w), first + 1 < n_st, row0, RT);
            }
        }
    }
}

// Short segments (a few synapses each, e.g. two million neurons in tiles of
// about a thousand) without workgroup-wide staging: every wave takes 64
// spikes at a time, one per lane.  A lane loads its spike's segment
// descriptor (one 64-bit word), a DPP scan over the wave gives the segments'
// offsets in the wave's flattened synapse range, the lanes publish (first
// synapse, offset, ring row) in the wave's own LDS slots, and then lane l
// takes synapses l, l + 64, ... of the range (contiguous loads within each
// segment), finding its segment by binary search over the 64 offsets.  No
// workgroup barrier.  Returns the wave's synaptic events (in every lane).
template <typename META, bool WBF16>
__device__ __forceinline__ uint32_t deliver_waves(const StreamArgs& a, int32_t* ring, const uint32_t* s_pc, int nq,
                                                  int64_t q_lo, int64_t n0b, uint64_t offb, int ntb, int tl,
                                                  int base_slot, uint32_t RT, int lane, int wave, int n_waves,
                                                  uint4* s_wv, uint32_t k_begin) {
    const uint32_t S = s_pc[nq];
    const uint32_t T = (uint32_t)a.T;
    uint4* my = s_wv + 64 * wave;   // this wave's 64 segment slots
    uint32_t ev = 0;
    // D rounds of 64 spikes per wave: their ids and descriptors are loaded
    // together before the first round's synapses
    constexpr int D = 4;
    const uint32_t stride = (uint32_t)n_waves * 64u;
    for (uint32_t kd = k_begin + (uint32_t)wave * 64u; kd < S; kd += D * stride) {
        uint32_t len[D], roff[D];
        uint64_t beg[D];
        uint32_t j[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            const uint32_t k = kd + (uint32_t)r * stride + (uint32_t)lane;
            j[r] = 0xFFFFFFFFu;
            roff[r] = 0;
            if (k < S) {
                int qi = 0;
                while (qi + 1 < nq && s_pc[qi + 1] <= k) ++qi;
                j[r] = a.spk_ids[(size_t)((q_lo + qi) & (a.H - 1)) * a.N + n0b + (k - s_pc[qi])];
                roff[r] = (uint32_t)(base_slot + qi) * T;
            }
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            len[r] = 0;
            beg[r] = 0;
            if (j[r] != 0xFFFFFFFFu) {
                const uint64_t d = a.seg[offb + (uint64_t)(j[r] - n0b) * (uint64_t)(ntb + 1) + tl];
                len[r] = (uint32_t)(d & 0xFFFFFFu);
                beg[r] = d >> 24;
            }
        }
#pragma unroll
        for (int r = 0; r < D; ++r) {
            const uint32_t incl = wave_incl_scan(len[r]);
            const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            if (total == 0) continue;   // wave-uniform
            ev += total;
            // the slots are rewritten only after every lane has read the
            // previous round's (the wave executes in lockstep; the barriers
            // and fences keep the LDS accesses of this wave in order)
            __builtin_amdgcn_wave_barrier();
            my[lane] = make_uint4(incl - len[r], roff[r], (uint32_t)beg[r], (uint32_t)(beg[r] >> 32));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            constexpr int U = 4;
            for (uint32_t f0 = (uint32_t)lane; f0 < total; f0 += 64u * U) {
                uint32_t m[U], x0[U];
                float wv[U];
                bool ok[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint32_t f = f0 + 64u * u;
                    ok[u] = f < total;
                    m[u] = 0;
                    wv[u] = 0.f;
                    x0[u] = 0;
                    if (ok[u]) {
                        // last slot whose offset is <= f
                        int lo = 0, hi = 64;
                        while (hi - lo > 1) {
                            const int mid = (lo + hi) >> 1;
                            if (my[mid].x <= f) lo = mid; else hi = mid;
                        }
                        const uint4 g = my[lo];
                        x0[u] = g.y;
                        load_rec<META, WBF16>(a.meta, a.w, (((uint64_t)g.w << 32) | g.z) + (f - g.x), m[u], wv[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (ok[u]) {
                        uint32_t x = m[u] + x0[u];
                        x = min(x, x - RT);
                        ring_add(ring, x, __float2int_rn(wv[u] * a.fxw_scale));
                    }
                }
            }
        }
    }
    return ev;
}

template <int MODEL, typename META, bool WBF16, int NPT>
// At most 4 waves per SIMD (1024 threads, or 2 x 512, per compute unit and
// its whole workgroup-local memory): registers for loads in flight are free.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4))) stream_kernel(StreamArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    if (a.ktime) ktime_mark(a.ktime, 1);
    const int tid = threadIdx.x, bs = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, n_waves = bs >> 6;
    const int tile = a.order[blockIdx.x];
    const int b = a.tile_inst[tile];
    const int ntb = a.inst_ntiles[b];
    const int tl = tile - a.inst_tile0[b];
    const int64_t n0b = a.inst_n0[b];
    const int64_t g0 = n0b + (int64_t)tl * a.inst_T[b];
    const int tsz = a.tile_size[tile];
    const uint64_t offb = a.inst_offbase[b];
    const int T = a.T, R = a.R, H = a.H, CH = a.chunk;
    const uint32_t RT = (uint32_t)R * (uint32_t)T;
    const int64_t t0 = a.clock[a.parity];
    const int wn = a.wn;

    uint4* s_sg = reinterpret_cast<uint4*>(lds_raw);                        // CH
    int32_t* ring = reinterpret_cast<int32_t*>(s_sg + CH);                  // R * T
    uint32_t* s_len = reinterpret_cast<uint32_t*>(ring + (size_t)R * T);    // CH + 1
    uint16_t* s_spk = reinterpret_cast<uint16_t*>(s_len + CH + 1);          // W * T
    uint32_t* s_frz = reinterpret_cast<uint32_t*>(s_spk + (size_t)a.W * T + ((a.W * T) & 1));   // T
    uint32_t* s_blk = s_frz + T;                                            // kDeliverBlk
    uint32_t* s_thr = s_blk + kDeliverBlk;                                  // kMaxThr
    uint32_t* s_pc = s_thr + kMaxThr;                                       // kMaxW + 1
    int* s_cnt = reinterpret_cast<int*>(s_pc + kMaxW + 1);                  // kMaxW
    uint32_t* s_wsum = reinterpret_cast<uint32_t*>(s_cnt + kMaxW);          // 20
    int* s_kw = reinterpret_cast<int*>(s_wsum + 20);                        // 20
    int* s_misc = s_kw + 20;                                                // 8

    if (blockIdx.x == 0) {
        // the next window's start, and its spike-list counters cleared
        if (tid == 0) a.clock[1 - a.parity] = t0 + wn;
        for (int i = tid; i < a.W * a.n_inst; i += bs) {
            const int64_t n = t0 + wn + i / a.n_inst;
            a.spk_cnt[(size_t)(n & (H - 1)) * a.n_inst + (i % a.n_inst)] = 0u;
        }
    }
    // The delivered steps' spike counts and the staged run's length (wave
    // 0) are requested first and used after the input ring is staged.
    const int64_t q_hi = t0 - a.dmin + wn;
    const int64_t q_lo = max((int64_t)0, t0 - a.dmin);
    const int nq = (int)max((int64_t)0, q_hi - q_lo);
    uint32_t c_q = 0;
    unsigned long long c_run = 0;
    if (wave == 0) {
        c_q = lane < nq ? a.spk_cnt[(size_t)((q_lo + lane) & (H - 1)) * a.n_inst + b] : 0u;
        if (lane == 0 && a.stage) c_run = a.cursor[tile];
        if (lane < kMaxThr) s_thr[lane] = lane < a.n_thr ? a.thr[lane] : 0xFFFFFFFFu;
    }
    float U[NPT], Y1[NPT], Y2[NPT];
    int RF[NPT];
    unsigned long long KC[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        // (a thread past the tile's end reads its last neuron and never uses it)
        const int64_t gi = g0 + min(tid + k * bs, tsz - 1);
        U[k] = __builtin_nontemporal_load(&a.U[gi]);
        RF[k] = __builtin_nontemporal_load(&a.r[gi]);
        Y1[k] = MODEL != CORTEX_MODEL_DELTA ? __builtin_nontemporal_load(&a.y1[gi]) : 0.f;
        Y2[k] = MODEL == CORTEX_MODEL_ALPHA ? __builtin_nontemporal_load(&a.y2[gi]) : 0.f;
        KC[k] = __builtin_nontemporal_load(&a.kcache[gi]);
    }
    __syncthreads();   // s_thr
    // ------------------------------------------------------------ stage in
    // Only the rows that can hold sums: the spikes delivered before this
    // window were emitted before t0 - dmin and arrive before
    // t0 + dmax - dmin, so the rows of arrival steps t0 .. t0 + nin - 1
    // (nin = dmax - dmin = R - W) are loaded and the other W rows start at
    // zero (their stored contents are stale: consumed rows are not written
    // back).  The first kStageIn pieces per thread are requested before the
    // Poisson draws below and stored after them, so that the draws run while
    // the loads are in flight; the loads carry no branches: an index past the
    // end is clamped to the last piece, which is then read and written again
    // with its own value.
    const int T4 = T / 4, RT4 = R * T4;   // 16-byte pieces (T is a multiple of 4)
    const int nin4 = (R - a.W) * T4;
    constexpr int kStageIn = 8;
    const int4* ring_src = reinterpret_cast<const int4*>(a.ring + (size_t)tile * R * T);
    int4* ring_dst = reinterpret_cast<int4*>(ring);
    const int p_in = (int)(t0 % R) * T4;
    int4 v_in[kStageIn];
    int at_in[kStageIn];
    // (equal delays leave no row to load: then the piece at p_in is read
    // and zero is stored, as the zero rows below do)
    const int last_in = max(nin4 - 1, 0);
#pragma unroll
    for (int u = 0; u < kStageIn; ++u) {
        const int p = p_in + min(tid + u * bs, last_in);
        at_in[u] = p >= RT4 ? p - RT4 : p;
        v_in[u] = load_stream(&ring_src[at_in[u]]);
    }
    {
        const int z0 = (int)((t0 + (R - a.W)) % R) * T4;
        for (int i = tid; i < RT4 - nin4; i += bs) {
            const int p = z0 + i;
            ring_dst[p >= RT4 ? p - RT4 : p] = make_int4(0, 0, 0, 0);
        }
    }
    // Poisson counts of the window's steps, 6 bits per step, before the
    // delivery (the update below is then only the ring and the membrane).  A
    // window of at most 8 steps touches at most two 8-step blocks; the block
    // of a neuron's last step is kept in kcache for the next window, so a
    // block is drawn once.
    uint64_t kcs[NPT];
    {
        const uint64_t blk_lo = (uint64_t)(t0 >> 3), blk_hi = (uint64_t)((t0 + wn - 1) >> 3);
        const int s0 = (int)(t0 & 7);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int li = tid + k * bs;
            const uint64_t nl = (uint64_t)(g0 - n0b + min(li, tsz - 1));   // instance-local neuron
            const uint64_t cl = kcache_holds(KC[k], blk_lo)
                                    ? KC[k] & kCountsMask
                                    : block_counts(nl, blk_lo, s_thr, a.n_thr, a.seed, (uint64_t)b);
            const uint64_t ch = blk_hi != blk_lo ? block_counts(nl, blk_hi, s_thr, a.n_thr, a.seed, (uint64_t)b) : cl;
            // steps s0.. of the first block, then the second block's
            const uint64_t w = (cl >> (6 * s0)) | (s0 ? ch << (6 * (8 - s0)) : 0ull);
            kcs[k] = w & ((1ull << (6 * wn)) - 1);
            const unsigned long long kn = kcache_entry(blk_hi, ch);
            if (li < tsz && kn != KC[k]) __builtin_nontemporal_store(kn, &a.kcache[g0 + li]);
        }
    }
#pragma unroll
    for (int u = 0; u < kStageIn; ++u) ring_dst[at_in[u]] = nin4 > 0 ? v_in[u] : make_int4(0, 0, 0, 0);
    for (int i0 = tid + kStageIn * bs; i0 < nin4; i0 += kStageIn * bs) {
        int4 v[kStageIn];
        int at[kStageIn];
#pragma unroll
        for (int u = 0; u < kStageIn; ++u) {
            const int p = p_in + min(i0 + u * bs, nin4 - 1);
            at[u] = p >= RT4 ? p - RT4 : p;
            v[u] = ring_src[at[u]];
        }
#pragma unroll
        for (int u = 0; u < kStageIn; ++u) ring_dst[at[u]] = v[u];
    }
    if (wave == 0) {
        // exclusive prefix s_pc[0..nq] of the delivered steps' spike counts;
        // the run staged for this window, and its cursor reset for the next
        const uint32_t incl = wave_incl_scan(c_q);
        if (lane <= nq) s_pc[lane] = incl - c_q;
        if (lane == 0 && a.stage) {
            s_misc[5] = (int)min(c_run, 0xFFFFFFFFull);
            a.cursor[tile] = 0ull;
        }
    }
    for (int i = tid; i < T; i += bs) s_frz[i] = 0;
    if (tid < kMaxW) s_cnt[tid] = 0;
    if (tid == 0) s_misc[7] = 0;
    // frozen spikes of the updated steps (replay); the bits are set only
    // once every thread has cleared its share of them
    if (a.frz_ptr) {
        __syncthreads();
        for (int si = 0; si < wn; ++si) {
            const int64_t n = t0 + si;
            const size_t at = (size_t)(n - a.frz_step0) * a.n_tiles + tile;
            const uint64_t f0 = min(a.frz_ptr[at], a.frz_n), f1 = min(a.frz_ptr[at + 1], a.frz_n);
            for (uint64_t q = f0 + tid; q < f1; q += bs) {
                const int64_t li = (int64_t)a.frz_ids[q] - g0;
                if (li >= 0 && li < tsz) atomicOr(&s_frz[li], 1u << si);
            }
        }
    }
    __syncthreads();
    // ------------------------------------------------------------ deliver
    const uint32_t S = s_pc[nq];
    const int base_slot = (int)((q_lo + a.dmin) % R);
    uint64_t ev = 0;
    if (a.thread_segments) {
        uint32_t k_begin = 0, n_staged = 0;
        if (a.stage) {
            // a complete run replaces the window's spikes; an incomplete one
            // (more records than the capacity) is ignored
            const uint32_t c = (uint32_t)s_misc[5];
            if (c <= a.stage_cap) {
                deliver_staged<WBF16>(a, ring, c, tile, base_slot, (uint32_t)T, RT, tid, bs);
                n_staged = c;
                k_begin = S;
            }
        }
        // the descriptor area holds the waves' segment slots (16 x 64 x 16 B)
        const uint32_t wev = deliver_waves<META, WBF16>(a, ring, s_pc, nq, q_lo, n0b, offb, ntb, tl, base_slot, RT,
                                                        lane, wave, n_waves, s_sg, k_begin);
        if (lane == 0) atomicAdd(reinterpret_cast<unsigned int*>(&s_misc[7]), wev);
        __syncthreads();
        ev = (uint64_t)(uint32_t)s_misc[7] + n_staged;
    }
    for (uint32_t c0 = 0; c0 < (a.thread_segments ? 0u : S); c0 += CH) {
        const int cn = (int)min((uint32_t)CH, S - c0);
        for (int k = tid; k < cn; k += bs) {
            const uint32_t kk = c0 + k;
            int qi = 0;
            while (qi + 1 < nq && s_pc[qi + 1] <= kk) ++qi;
            const uint32_t j = a.spk_ids[(size_t)((q_lo + qi) & (H - 1)) * a.N + n0b + (kk - s_pc[qi])];
            const uint64_t d = a.seg[offb + (uint64_t)(j - n0b) * (uint64_t)(ntb + 1) + tl];
            const uint32_t len = (uint32_t)(d & 0xFFFFFFu);
            const uint64_t beg = d >> 24;
            s_sg[k] = make_uint4(len, (uint32_t)qi, (uint32_t)beg, (uint32_t)(beg >> 32));
            s_len[k] = len;
        }
        __syncthreads();
        const uint32_t EL = block_excl_scan(s_len, cn, s_wsum);
        wave_runs(s_len, s_kw, cn, EL, n_waves, tid, bs);
        __syncthreads();
        if (EL >= 32u * (uint32_t)cn)
            deliver_long<META, WBF16, int32_t>(s_sg, ring, s_kw[wave], s_kw[wave + 1], lane, a.meta, a.w,
                                               base_slot, (uint32_t)T, RT, a.fxw_scale);
        else
            deliver_short<META, WBF16, int32_t>(s_sg, s_len, s_blk, ring, cn, EL, tid, bs, lane, wave, n_waves,
                                                a.meta, a.w, base_slot, (uint32_t)T, RT, a.fxw_scale);
        ev += EL;
        __syncthreads();
    }
    // ------------------------------------------------------------ update
    const int slot0 = (int)(t0 % R);
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int li = tid + k * bs;
        if (li < tsz) {
            const uint32_t frz = s_frz[li];
            int slot = slot0;
            for (int si = 0; si < wn; ++si, slot = (slot + 1 == R) ? 0 : slot + 1) {
                const int64_t n = t0 + si;
                const float x = (float)((double)ring[slot * T + li] * a.fx_inv);
                ring[slot * T + li] = 0;
                const int kc = (int)((kcs[k] >> (6 * si)) & 63u);
                const float inp = x + a.w_ext * (float)kc;
                const bool integ = RF[k] == 0;
                float u_new;
                if (!integ) {
                    RF[k] -= 1;
                    u_new = a.Ur;
                } else if (MODEL == CORTEX_MODEL_DELTA) {
                    u_new = a.P22 * U[k] + a.P20Ie + inp;
                } else if (MODEL == CORTEX_MODEL_EXP) {
                    u_new = a.P22 * U[k] + a.P21 * Y1[k] + a.P20Ie;
                } else {
                    u_new = a.P22 * U[k] + a.P31 * Y1[k] + a.P32 * Y2[k] + a.P20Ie;
                }
                if (MODEL == CORTEX_MODEL_EXP) {
                    Y1[k] = a.P11 * Y1[k] + inp;
                } else if (MODEL == CORTEX_MODEL_ALPHA) {
                    Y2[k] = a.P21s * Y1[k] + a.P22s * Y2[k];
                    Y1[k] = a.P11 * Y1[k] + a.jump * inp;
                }
                const bool spk = a.frz_ptr ? ((frz >> si) & 1u) != 0 : (integ && u_new >= a.theta);
                if (spk) {
                    u_new = a.Ur;
                    RF[k] = a.n_ref;
                    const int p = atomicAdd(&s_cnt[si], 1);
                    s_spk[si * T + p] = (uint16_t)li;
                }
                U[k] = u_new;
                if (a.x_trace || a.v_trace || a.m_trace) {
                    const size_t ti = (size_t)(n - a.trace_step0) * a.N + g0 + li;
                    if (a.x_trace) a.x_trace[ti] = x;
                    if (a.v_trace) a.v_trace[ti] = u_new + a.E_L;
                    if (a.m_trace) a.m_trace[ti] = (integ && !spk) ? 1 : 0;
                }
            }
            __builtin_nontemporal_store(U[k], &a.U[g0 + li]);
            __builtin_nontemporal_store(RF[k], &a.r[g0 + li]);
            if (MODEL != CORTEX_MODEL_DELTA) __builtin_nontemporal_store(Y1[k], &a.y1[g0 + li]);
            if (MODEL == CORTEX_MODEL_ALPHA) __builtin_nontemporal_store(Y2[k], &a.y2[g0 + li]);
        }
    }
    __syncthreads();
    // ------------------------------------------------------------ publish
    // one reservation per step in the instance's list of that step; the
    // reservations are requested first and the ring rows the next window
    // loads (arrival steps t0 + wn .. t0 + wn + nin - 1) are written back
    // while they are in flight
    uint32_t res_c = 0, res_at = 0;
    if (tid < wn) {
        const int64_t n = t0 + tid;
        res_c = (uint32_t)s_cnt[tid];
        if (res_c) res_at = atomicAdd(&a.spk_cnt[(size_t)(n & (H - 1)) * a.n_inst + b], res_c);
    }
    {
        int4* dst = reinterpret_cast<int4*>(a.ring + (size_t)tile * R * T);
        const int4* src = reinterpret_cast<const int4*>(ring);
        const int p0 = (int)((t0 + wn) % R) * T4;
        for (int i = tid; i < nin4; i += bs) {
            const int p = p0 + i;
            const int q = p >= RT4 ? p - RT4 : p;
            store_stream(&dst[q], src[q]);
        }
    }
    if (tid < wn) s_misc[tid] = res_c ? (int)res_at : 0;
    uint64_t log_pos = a.log_pos[tile];
    const uint64_t log_b = a.log_base[tile], log_cap = a.log_base[tile + 1] - log_b;
    __syncthreads();
    uint64_t nspk = 0;
    for (int si = 0; si < wn; ++si) {
        const int64_t n = t0 + si;
        const int c = s_cnt[si];
        uint32_t* dst = a.spk_ids + (size_t)(n & (H - 1)) * a.N + n0b + (uint32_t)s_misc[si];
        const uint16_t* ls = s_spk + (size_t)si * T;
        for (int i = tid; i < c; i += bs) dst[i] = (uint32_t)(g0 + ls[i]);
        if (n >= a.log_step0 && n < a.log_step0 + a.log_steps) {
            if (log_pos + c <= log_cap) {
                for (int i = tid; i < c; i += bs) a.log_ids[log_b + log_pos + i] = (uint32_t)(g0 + ls[i]);
                if (tid == 0) a.log_cnt[(n - a.log_step0) * a.n_tiles + tile] = (uint32_t)c;
                log_pos += c;
            } else if (tid == 0) {
                a.log_cnt[(n - a.log_step0) * a.n_tiles + tile] = 0xFFFFFFFFu;   // overflow mark
            }
        }
        nspk += c;
    }
    if (tid == 0) {
        a.events[tile] += ev;
        a.spikes[tile] += nspk;
        a.log_pos[tile] = log_pos;
    }
}

using StreamFn = void (*)(StreamArgs);

template <int MODEL, typename META, bool WBF16>
StreamFn pick_npt(int npt) {
    if (npt == 1) return stream_kernel<MODEL, META, WBF16, 1>;
    if (npt == 2) return stream_kernel<MODEL, META, WBF16, 2>;
    return stream_kernel<MODEL, META, WBF16, 4>;
}

// bf16 weights come packed with 16-bit records (see deliver.hpp)
template <int MODEL>
StreamFn pick_fmt(int meta_bytes, int w_bytes, int npt) {
    if (w_bytes == 2) return meta_bytes == 2 ? pick_npt<MODEL, uint16_t, true>(npt) : nullptr;
    return meta_bytes == 2 ? pick_npt<MODEL, uint16_t, false>(npt) : pick_npt<MODEL, uint32_t, false>(npt);
}

StreamFn pick_stream(int model, int meta_bytes, int w_bytes, int npt) {
    switch (model) {
        case CORTEX_MODEL_DELTA: return pick_fmt<CORTEX_MODEL_DELTA>(meta_bytes, w_bytes, npt);
        case CORTEX_MODEL_EXP: return pick_fmt<CORTEX_MODEL_EXP>(meta_bytes, w_bytes, npt);
        case CORTEX_MODEL_ALPHA: return pick_fmt<CORTEX_MODEL_ALPHA>(meta_bytes, w_bytes, npt);
        default: return nullptr;   // conductances need 64-bit rings
    }
}

}  // namespace

int stream_occupancy(int model, int meta_bytes, int w_bytes, int npt, int bs, size_t lds) {
    StreamFn f = pick_stream(model, meta_bytes, w_bytes, npt);
    if (!f) return 0;
    if (hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, bs, lds) != hipSuccess) return 0;
    return nb;
}

// Arguments of the window launches of a network (everything but the clock
// parity and window length).
static StreamArgs stream_args(cortex_net* n, const uint32_t* frz_ids, const uint64_t* frz_ptr, uint64_t frz_n,
                              int64_t frz_step0, float* x_trace, float* v_trace, uint8_t* m_trace,
                              int64_t trace_step0) {
    require(n->n_thr <= kMaxThr, CORTEX_EUNSUPPORTED, "Poisson mean too large for the FP32 kernel");
    StreamArgs a{};
    a.order = n->d_order;
    a.tile_inst = n->d_tile_inst;
    a.tile_size = n->d_tile_size;
    a.inst_tile0 = n->d_inst_tile0;
    a.inst_ntiles = n->d_inst_ntiles;
    a.inst_T = n->d_inst_T;
    a.inst_n0 = n->d_inst_n0;
    a.inst_offbase = n->d_inst_offbase;
    a.seg = n->d_seg;
    a.meta = n->d_meta;
    a.w = n->d_w;
    a.U = n->d_U;
    a.y1 = n->d_y1;
    a.y2 = n->d_y2;
    a.kcache = n->d_kcache;
    a.r = n->d_r;
    a.ring = static_cast<int32_t*>(n->d_ring);
    a.spk_cnt = n->d_spk_cnt;
    a.spk_ids = n->d_spk_ids;
    a.clock = n->d_clock;
    a.log_cnt = n->d_log_cnt;
    a.log_ids = n->d_log_ids;
    a.log_base = n->d_log_base;
    a.log_pos = n->d_log_pos;
    a.events = n->d_events;
    a.spikes = n->d_spikes;
    a.frz_ids = frz_ids;
    a.frz_ptr = frz_ptr;
    a.frz_n = frz_n;
    a.frz_step0 = frz_step0;
    a.x_trace = x_trace;
    a.v_trace = v_trace;
    a.m_trace = m_trace;
    a.trace_step0 = trace_step0;
    a.stage = n->stage_cap ? n->d_stage : nullptr;
    a.cursor = n->d_cursor;
    a.stage_cap = n->stage_cap;
    a.ktime = n->ktiming ? n->d_ktime : nullptr;
    a.log_step0 = n->log_step0;
    a.log_steps = n->log_steps;
    a.N = n->N;
    a.n_tiles = n->n_tiles;
    a.n_inst = n->n_inst;
    a.T = n->T;
    a.R = n->R;
    a.dmin = n->dmin;
    a.H = n->H;
    a.W = n->W;
    a.chunk = n->chunk;
    a.n_ref = n->k.n_ref;
    a.n_thr = n->n_thr;
    a.thread_segments = n->thread_segments;
    a.P22 = (float)n->k.P22;
    a.P20Ie = (float)(n->k.P20 * n->spec.I_e);
    a.P11 = (float)n->k.P11;
    a.P21 = (float)n->k.P21;
    a.P31 = (float)n->k.P31;
    a.P32 = (float)n->k.P32;
    a.P21s = (float)n->k.P21s;
    a.P22s = (float)n->k.P22s;
    a.jump = (float)n->k.jump;
    a.theta = (float)(n->spec.V_th - n->spec.E_L);
    a.Ur = (float)(n->spec.V_reset - n->spec.E_L);
    a.w_ext = (float)n->w_ext_native;
    a.E_L = (float)n->spec.E_L;
    a.fxw_scale = std::ldexp(1.0f, n->fx - n->fx_shift);
    a.fx_inv = std::ldexp(1.0, n->fx_shift - n->fx);
    a.seed = n->seed;
    for (int m = 0; m < n->n_thr; ++m) a.thr[m] = n->thr[m];
    return a;
}

// One window: plasticity, staging copy, delivery launch.
static void launch_window(cortex_net* n, StreamFn f, StreamArgs& a, int wn, hipStream_t stream) {
    if (n->stdp) launch_stdp(n, n->clock_parity, wn, stream);   // weights first, then their delivery
    if (n->stage_cap) launch_gather(n, n->clock_parity, wn, stream);
    a.parity = n->clock_parity;
    a.wn = wn;
    hipLaunchKernelGGL(f, dim3(n->n_tiles), dim3(n->BS), n->lds_bytes, stream, a);
    CX_HIP(hipGetLastError());
    n->clock_parity ^= 1;
}

void launch_stream_fp32(cortex_net* n, int64_t n_steps, const uint32_t* frz_ids, const uint64_t* frz_ptr,
                        uint64_t frz_n, float* x_trace, float* v_trace, uint8_t* m_trace) {
    if (n_steps <= 0) return;
    StreamFn f = pick_stream(n->spec.model, n->meta_bytes, n->w_bytes, n->NPT);
    require(f != nullptr, CORTEX_EUNSUPPORTED, "no streamed kernel for this record format");
    CX_HIP(hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)n->lds_bytes));
    if (n->stage_cap) gather_prepare(n);
    const int64_t first = n->step;
    StreamArgs a = stream_args(n, frz_ids, frz_ptr, frz_n, first, x_trace, v_trace, m_trace, first);
    int64_t left = n_steps;
    // Full windows of plain closed-loop runs replay a captured graph of
    // kGraphWindows launches (the clock advances on the device; the parity
    // alternates inside the graph, so it starts even).
    // The graph lives on a stream of the library's own (the caller's may be
    // the legacy null stream, which cannot be captured), ordered after the
    // caller's earlier work and before its later work by two events.
    const bool plain = !frz_ptr && !x_trace && !v_trace && !m_trace;
    if (plain && n->use_graph) {
        const int64_t per = (int64_t)kGraphWindows * n->W;
        if (left >= per && n->clock_parity != 0) {
            launch_window(n, f, a, n->W, n->stream);
            left -= n->W;
            n->step += n->W;
        }
        if (left >= per) {
            if (!n->graph_stream) {
                CX_HIP(hipStreamCreate(&n->graph_stream));
                CX_HIP(hipEventCreateWithFlags(&n->fence_in, hipEventDisableTiming));
                CX_HIP(hipEventCreateWithFlags(&n->fence_out, hipEventDisableTiming));
            }
            if (!n->graph_exec || n->graph_log_step0 != n->log_step0 || n->graph_log_steps != n->log_steps ||
                n->graph_ktiming != n->ktiming) {
                if (n->graph_exec) {
                    CX_HIP(hipStreamSynchronize(n->graph_stream));
                    CX_HIP(hipGraphExecDestroy(n->graph_exec));
                    n->graph_exec = nullptr;
                }
                hipGraph_t g = nullptr;
                CX_HIP(hipStreamBeginCapture(n->graph_stream, hipStreamCaptureModeThreadLocal));
                const int saved = n->clock_parity;
                for (int k = 0; k < kGraphWindows; ++k) launch_window(n, f, a, n->W, n->graph_stream);
                n->clock_parity = saved;
                CX_HIP(hipStreamEndCapture(n->graph_stream, &g));
                CX_HIP(hipGraphInstantiate(&n->graph_exec, g, nullptr, nullptr, 0));
                CX_HIP(hipGraphDestroy(g));
                n->graph_log_step0 = n->log_step0;
                n->graph_log_steps = n->log_steps;
                n->graph_ktiming = n->ktiming;
            }
            CX_HIP(hipEventRecord(n->fence_in, n->stream));
            CX_HIP(hipStreamWaitEvent(n->graph_stream, n->fence_in, 0));
            while (left >= per) {
                CX_HIP(hipGraphLaunch(n->graph_exec, n->graph_stream));
                left -= per;
                n->step += per;
            }
            CX_HIP(hipEventRecord(n->fence_out, n->graph_stream));
            CX_HIP(hipStreamWaitEvent(n->stream, n->fence_out, 0));
        }
    }
    while (left > 0) {
        const int wn = (int)std::min<int64_t>(n->W, left);
        launch_window(n, f, a, wn, n->stream);
        left -= wn;
        n->step += wn;
    }
}

}  // namespace cortex
