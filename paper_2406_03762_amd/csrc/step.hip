// Persistent FP32 step kernel: LIF update, spike publication and delivery
// into workgroup-local input rings.
//
// Mapping of the paper's scheme onto the GPU:
//  - a tile of T consecutive targets and all synapses into them (the
//    indegree sub-graph of Eq. 5 for that vertex set, one per part of the
//    partition of Eq. 9-10) belongs to exactly one workgroup for the whole
//    run, as each post-neuron and its in-edges belong to one thread in
//    Sec. III-B; the tile's pending input lives in that workgroup's LDS, so
//    every write of the delivery is local and no global atomic is needed
//    (the shared part of two indegree sub-graphs holds only read-only
//    pre-vertices, Eq. 14);
//  - a spike emitted at step q acts no earlier than q + d_min, so the
//    workgroups exchange spikes once per W <= d_min steps: a "window"
//    [t0, t0 + W) first delivers the spikes of steps [t0 - d_min,
//    t0 - d_min + W) (all published by every tile before the window began:
//    the buffered spikes of Sec. III-C), then updates its neurons W times,
//    publishing each step's spikes.  Steps stay strictly sequential per
//    neuron (Sec. III-B, "Varied Synaptic Delays");
//  - delivery reads, for every spike of the window, the one segment of the
//    source's synapses that lands in this tile (the spiking sub-graph,
//    Eq. 11) and adds each weight into ring slot (step + delay) mod R.
//    Pending arrivals span R = d_max - d_min + W steps.
// The rings hold 64-bit fixed-point sums (scale 2^fx, chosen so that no
// target's total in-weight can overflow): integer LDS atomics are several
// times faster than float ones, and an integer sum does not depend on the
// order in which the spikes of a window are added.
// Spikes are published as 64-bit words tagged with the step (coherent
// device-scope stores, no cache flushes); a reader accepts a word only when
// its tag matches the step it waits for.
#include <algorithm>
#include <cmath>

#include "deliver.hpp"
#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

constexpr int kMaxThr = 32;       // Poisson table entries in kernel arguments
constexpr int kInline = 1;        // spike ids fetched together with a tile's step record

struct StepArgs {
    const int32_t* inst_tile0;
    const int32_t* inst_ntiles;
    const int32_t* inst_T;
    const int64_t* inst_n0;
    const uint64_t* inst_offbase;
    const int32_t* tile_inst;
    const int32_t* tile_size;
    const uint64_t* seg;        // (first synapse << 24) | length per (source, tile)
    const void* meta;
    const void* w;
    float* U;
    float* y1;
    float* y2;
    int32_t* r;
    void* ring;                 // [n_tiles][R][T] of RING
    uint64_t* pub;              // [H][n_tiles][T + 1] tagged step records and spike ids
    uint32_t* log_cnt;
    uint32_t* log_ids;
    const uint64_t* log_base;
    uint64_t* log_pos;
    uint64_t* events;
    uint64_t* spikes;
    int32_t* err;
    const uint32_t* frz_ids;
    const uint64_t* frz_ptr;
    uint64_t frz_n;             // ids in frz_ids
    float* x_trace;
    float* v_trace;
    uint8_t* m_trace;           // 1 where a neuron integrated and did not spike (adjoint)
    int64_t n0, n1, log_step0, log_steps, N;
    int n_tiles, T, R, dmin, H, W, chunk, n_ref, n_thr, xcd, spin_log2, ntb_max;
    float P22, P20Ie, P11, P21, P31, P32, P21s, P22s, jump, theta, Ur, w_ext, E_L;
    float fxw_scale;            // 2^fw: synaptic weight to its 32-bit fixed-point value
    double fx_inv;              // 2^-fw: ring sum to input
    float gL, Eex, Ein, Ie, dt_C;   // conductance model (reversal potentials relative to E_L)
    uint64_t seed;
    uint32_t thr[kMaxThr];
};

__device__ __forceinline__ uint64_t coherent_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Re-read a published word until it carries `tag` (bounded).  A wait that
// gives up returns 0, whose tag (0) no published word carries; the status
// travels in the return value, not through a pointer, so the caller's flag
// stays in a register.
__device__ __noinline__ uint64_t wait_tag(const uint64_t* p, uint64_t v, uint32_t tag, int64_t spin_max,
                                          int32_t* err) {
    int64_t spins = 0;
    int32_t e = 0;
    while ((uint32_t)(v >> 32) != tag) {
        if (++spins > spin_max || e != 0) return 0;
        __builtin_amdgcn_s_sleep(1);
        // the error flag is read with the word, so one round trip per try
        e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = coherent_load(p);
    }
    return v;
}

// Up to 1024 threads per workgroup with one or two neurons per thread; four
// neurons per thread (large tiles) need the registers of a 512-thread limit.
template <int MODEL, typename META, bool WBF16, int NPT, typename RING>
__global__ void __launch_bounds__(NPT == 4 ? 512 : 1024) step_kernel(StepArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int tid = threadIdx.x, bs = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, n_waves = bs >> 6;
    const int bid = blockIdx.x;
    const int tile = a.xcd ? ((bid & 7) * (a.n_tiles >> 3) + (bid >> 3)) : bid;
    const int b = a.tile_inst[tile];
    const int tile0b = a.inst_tile0[b];
    const int ntb = a.inst_ntiles[b];
    const int tl = tile - tile0b;
    const int64_t n0b = a.inst_n0[b];
    const int64_t g0 = n0b + (int64_t)tl * a.inst_T[b];
    const int tsz = a.tile_size[tile];
    const uint64_t offb = a.inst_offbase[b];
    const int T = a.T, R = a.R, H = a.H, CH = a.chunk;
    const uint32_t RT = (uint32_t)R * (uint32_t)T;
    const size_t pub_tile = (size_t)T + 1;
    const size_t pub_slot = (size_t)a.n_tiles * pub_tile;
    const int pairs_max = a.W * a.ntb_max;

    // s_sg[k] describes segment k of a delivery chunk: x = its number of
    // synapses, y = step offset of the spike within the delivered steps,
    // (z, w) = index of its first synapse (64-bit)
    uint4* s_sg = reinterpret_cast<uint4*>(lds_raw);                // CH
    RING* ring = reinterpret_cast<RING*>(s_sg + CH);                // R * T
    uint32_t* s_len = reinterpret_cast<uint32_t*>(ring + (size_t)R * T);   // CH + 1
    uint32_t* s_spk = s_len + CH + 1;                               // W * T (spikes per step of a window)
    uint32_t* s_pc = s_spk + (size_t)a.W * T;                       // pairs_max + 1
    uint32_t* s_pid = s_pc + pairs_max + 1;                         // pairs_max * kInline
    uint32_t* s_wsum = s_pid + (size_t)pairs_max * kInline;         // 20
    int* s_misc = reinterpret_cast<int*>(s_wsum + 20);              // 4
    int* s_cnt = s_misc + 4;                                        // 8 (spike count per step of a window)
    int* s_kw = s_cnt + 8;                                          // 20 (first segment of each wave's run)
    uint32_t* s_frz = reinterpret_cast<uint32_t*>(s_kw + 20);      // T (bit si: frozen spike at step si)
    uint32_t* s_thr = s_frz + T;                                    // kMaxThr Poisson thresholds
    unsigned char* s_kcb = reinterpret_cast<unsigned char*>(s_thr + kMaxThr);  // 2 x 8 x T Poisson counts
    uint32_t* s_blk = reinterpret_cast<uint32_t*>(s_kcb + (size_t)16 * T);        // kDeliverBlk

    float U[NPT], Y1[NPT], Y2[NPT];
    int RF[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int li = tid + k * bs;
        U[k] = Y1[k] = Y2[k] = 0.f;
        RF[k] = 0;
        if (li < tsz) {
            U[k] = a.U[g0 + li];
            RF[k] = a.r[g0 + li];
            if (MODEL != CORTEX_MODEL_DELTA) Y1[k] = a.y1[g0 + li];
            if (MODEL == CORTEX_MODEL_ALPHA || MODEL == CORTEX_MODEL_COND) Y2[k] = a.y2[g0 + li];
        }
    }
    const RING* g_ring = static_cast<const RING*>(a.ring) + (size_t)tile * R * T;
    for (int i = tid; i < R * T; i += bs) ring[i] = g_ring[i];
    for (int i = tid; i < T; i += bs) s_frz[i] = 0;
    if (tid == 0) { s_misc[0] = 0; s_misc[1] = 0; }
    if (tid < 8) s_cnt[tid] = 0;
    if (tid < kMaxThr) s_thr[tid] = tid < a.n_thr ? a.thr[tid] : 0xFFFFFFFFu;
    uint64_t log_pos = a.log_pos[tile];
    const uint64_t log_b = a.log_base[tile], log_cap = a.log_base[tile + 1] - log_b;
    uint64_t ev = 0, nspk = 0;
    const int64_t spin_max = (int64_t)1 << a.spin_log2;
    bool bail = false;
    // 8-step blocks held in the two halves of s_kcb (same in every thread;
    // two scalars, not an indexed array, which would live in scratch memory)
    int64_t kc_blk0 = -1, kc_blk1 = -1;
    __syncthreads();

    for (int64_t t0 = a.n0; t0 < a.n1; t0 += a.W) {
        const int wn = (int)min((int64_t)a.W, a.n1 - t0);
        // Per-window work that does not depend on the network state (frozen
        // spike marks, Poisson counts) runs while the step records are in
        // flight.  Readers are separated from it by a workgroup barrier.
        bool marked = false, prepared = false;
        auto mark_frozen = [&]() {
            if (a.frz_ptr) {
                for (int si = 0; si < wn; ++si) {
                    const int64_t n = t0 + si;
                    const uint64_t f0 = min(a.frz_ptr[(n - a.n0) * a.n_tiles + tile], a.frz_n);
                    const uint64_t f1 = min(a.frz_ptr[(n - a.n0) * a.n_tiles + tile + 1], a.frz_n);
                    for (uint64_t q = f0 + tid; q < f1; q += bs) {
                        const int64_t li = (int64_t)a.frz_ids[q] - g0;
                        if (li >= 0 && li < tsz) atomicOr(&s_frz[li], 1u << si);
                    }
                }
            }
            marked = true;
        };
        // Poisson counts, 8 steps of one neuron per Philox call, for the 8-step
        // blocks the window touches; the two most recent blocks stay in
        // workgroup-local memory, so each block is generated once
        auto prepare = [&]() {
            const int64_t blk0 = t0 >> 3, blk1 = (t0 + wn - 1) >> 3;
            for (int64_t blk = blk0; blk <= blk1; ++blk) {
                if (((blk & 1) ? kc_blk1 : kc_blk0) == blk) continue;
                unsigned char* dst = s_kcb + (size_t)(blk & 1) * 8 * T;
                for (int li = tid; li < tsz; li += bs) {
                    const Philox4 p = philox((uint64_t)(g0 - n0b + li), (uint64_t)blk, 0, kTagPoisson, a.seed,
                                             (uint64_t)b);
#pragma unroll
                    for (int sub = 0; sub < 8; ++sub) {
                        const uint64_t word = p.v[sub >> 1];
                        const uint32_t u = (sub & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
                        // inversion: the count is the number of the n_thr
                        // (increasing) thresholds at or below u, found by a
                        // binary search over the table
                        int kc = 0;
#pragma unroll
                        for (int h = kMaxThr; h > 0; h >>= 1)
                            if (kc + h <= a.n_thr && s_thr[kc + h - 1] <= u) kc += h;
                        dst[sub * T + li] = (unsigned char)kc;
                    }
                }
                if (blk & 1) kc_blk1 = blk; else kc_blk0 = blk;
            }
            prepared = true;
        };
        // ------------------------------------------------------------ deliver
        const int64_t q_hi = t0 - a.dmin + wn;
        const int64_t q_lo = max((int64_t)0, t0 - a.dmin);
        if (q_hi > q_lo) {
            const int nq = (int)(q_hi - q_lo);
            const int pairs = nq * ntb;
            // step records of every tile of the instance, with their first
            // ids: all loads of a thread's pairs are issued before any wait
            constexpr int kP = 2;
            for (int p0 = 0; p0 < pairs; p0 += kP * bs) {
                uint64_t rec[kP], idw[kP][kInline];
                const uint64_t* base[kP];
#pragma unroll
                for (int u = 0; u < kP; ++u) {
                    const int p = p0 + tid + u * bs;
                    base[u] = nullptr;
                    if (p < pairs) {
                        const int qi = p / ntb, tt = p - qi * ntb;
                        const int64_t q = q_lo + qi;
                        base[u] = a.pub + (size_t)(q & (H - 1)) * pub_slot + (size_t)(tile0b + tt) * pub_tile;
                        rec[u] = coherent_load(base[u]);
#pragma unroll
                        for (int k = 0; k < kInline; ++k) idw[u][k] = coherent_load(base[u] + 1 + k);
                    }
                }
                if (!marked) mark_frozen();
                if (!prepared) prepare();
                // every stale word of the thread's pairs is re-read in the
                // same round (one round trip per try, the error flag with
                // them) until all carry their step's tag
                uint32_t tag[kP];
#pragma unroll
                for (int u = 0; u < kP; ++u) tag[u] = (uint32_t)(q_lo + (p0 + tid + u * bs) / ntb + 1);
                int64_t spins = 0;
                int32_t e = 0;
                while (!bail) {
                    bool stale[kP], pending = false;
#pragma unroll
                    for (int u = 0; u < kP; ++u) {
                        stale[u] = false;
                        if (base[u]) {
                            bool st = (uint32_t)(rec[u] >> 32) != tag[u];
#pragma unroll
                            for (int k = 0; k < kInline; ++k)
                                st |= (uint32_t)k < (uint32_t)rec[u] && (uint32_t)(idw[u][k] >> 32) != tag[u];
                            stale[u] = st;
                            pending |= st;
                        }
                    }
                    if (!pending) break;
                    if (++spins > spin_max || e != 0) {
                        bail = true;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    e = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                    for (int u = 0; u < kP; ++u) {
                        if (stale[u]) {
                            rec[u] = coherent_load(base[u]);
#pragma unroll
                            for (int k = 0; k < kInline; ++k) idw[u][k] = coherent_load(base[u] + 1 + k);
                        }
                    }
                }
                if (!bail) {
#pragma unroll
                    for (int u = 0; u < kP; ++u) {
                        const int p = p0 + tid + u * bs;
                        if (base[u]) {
                            const uint32_t c = (uint32_t)rec[u];
                            s_pc[p] = c;
#pragma unroll
                            for (int k = 0; k < kInline; ++k)
                                if ((uint32_t)k < c) s_pid[p * kInline + k] = (uint32_t)idw[u][k];
                        }
                    }
                }
            }
            if (bail) {
                s_misc[1] = 1;
                __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();
            if (s_misc[1]) break;
            const uint32_t S = block_excl_scan(s_pc, pairs, s_wsum);
            const int base_slot = (int)((q_lo + a.dmin) % R);
            for (uint32_t c0 = 0; c0 < S; c0 += CH) {
                const int cn = (int)min((uint32_t)CH, S - c0);
                // spike kk of the window belongs to the (step, tile) pair p
                // with s_pc[p] <= kk < s_pc[p + 1]: each pair writes its
                // spikes' pair index (s_len is reused, each entry is read and
                // then overwritten by the same thread below)
                for (int p = tid; p < pairs; p += bs) {
                    const uint32_t lo = max(s_pc[p], c0);
                    const uint32_t hi = min(p + 1 < pairs ? s_pc[p + 1] : S, c0 + (uint32_t)cn);
                    for (uint32_t kk = lo; kk < hi; ++kk) s_len[kk - c0] = (uint32_t)p;
                }
                __syncthreads();
                for (int k = tid; k < cn; k += bs) {
                    const uint32_t kk = c0 + k;
                    const int p = (int)s_len[k];
                    const uint32_t rnk = kk - s_pc[p];
                    const int qi = p / ntb, tt = p - qi * ntb;
                    uint32_t j;
                    if (rnk < (uint32_t)kInline) {
                        j = s_pid[p * kInline + rnk];
                    } else {
                        const int64_t q = q_lo + qi;
                        const uint64_t* w = a.pub + (size_t)(q & (H - 1)) * pub_slot +
                                            (size_t)(tile0b + tt) * pub_tile + 1 + rnk;
                        const uint64_t v = wait_tag(w, coherent_load(w), (uint32_t)(q + 1), spin_max, a.err);
                        if ((uint32_t)(v >> 32) != (uint32_t)(q + 1)) bail = true;
                        j = (uint32_t)v;
                    }
                    if (bail) {
                        // the id never arrived: the kernel stops after this
                        // chunk, so the entry is only kept in range
                        s_sg[k] = make_uint4(0u, 0u, 0u, 0u);
                        s_len[k] = 0;
                        continue;
                    }
                    const uint64_t d = a.seg[offb + (uint64_t)(j - n0b) * (uint64_t)(ntb + 1) + tl];
                    const uint32_t len = (uint32_t)(d & 0xFFFFFFu);
                    const uint64_t beg = d >> 24;
                    s_sg[k] = make_uint4(len, (uint32_t)qi, (uint32_t)beg, (uint32_t)(beg >> 32));
                    s_len[k] = len;
                }
                if (bail) {
                    s_misc[1] = 1;
                    __hip_atomic_store(a.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
                if (s_misc[1]) break;
                const uint32_t EL = block_excl_scan(s_len, cn, s_wsum);
                wave_runs(s_len, s_kw, cn, EL, n_waves, tid, bs);
                __syncthreads();
                if (EL >= 32u * (uint32_t)cn)
                    deliver_long<META, WBF16, RING>(s_sg, ring, s_kw[wave], s_kw[wave + 1], lane, a.meta, a.w,
                                                    base_slot, (uint32_t)T, RT, a.fxw_scale);
                else
                    deliver_short<META, WBF16, RING>(s_sg, s_len, s_blk, ring, cn, EL, tid, bs, lane, wave,
                                                     n_waves, a.meta, a.w, base_slot, (uint32_t)T, RT,
                                                     a.fxw_scale);
                ev += EL;
                __syncthreads();
            }
            if (s_misc[1]) break;
        }
        // ------------------------------------------------------------ update
        // Every input of the window's steps has been delivered (W <= d_min),
        // so each thread advances its neurons through all wn steps without
        // workgroup barriers; spikes go to per-step lists.
        // threads whose waves had no synapses to load (or a window without
        // deliveries) finish the per-window work here; the barrier is taken
        // by every thread
        if (!marked) mark_frozen();
        if (!prepared) prepare();
        __syncthreads();
        const int slot0 = (int)(t0 % R);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int li = tid + k * bs;
            if (li < tsz) {
                const uint32_t frz = a.frz_ptr ? s_frz[li] : 0u;
                int slot = slot0;
                for (int si = 0; si < wn; ++si, slot = (slot + 1 == R) ? 0 : slot + 1) {
                    const int64_t n = t0 + si;
                    float x, x_in = 0.f;
                    if (MODEL == CORTEX_MODEL_COND) {
                        // the two channels of the cell: excitatory low, inhibitory high
                        const unsigned long long c = (unsigned long long)ring[slot * T + li];
                        x = (float)((double)(uint32_t)c * a.fx_inv);
                        x_in = (float)((double)(uint32_t)(c >> 32) * a.fx_inv);
                    } else {
                        x = (float)((double)ring[slot * T + li] * a.fx_inv);
                    }
                    ring[slot * T + li] = 0;
                    const int kc = s_kcb[(size_t)((n >> 3) & 1) * 8 * T + (size_t)(n & 7) * T + li];
                    const float inp = x + a.w_ext * (float)kc;
                    const bool integ = RF[k] == 0;
                    float u_new;
                    if (!integ) {
                        RF[k] -= 1;
                        u_new = a.Ur;
                    } else if (MODEL == CORTEX_MODEL_COND) {
                        // the exact solution for conductances held over the step
                        const float G = a.gL + Y1[k] + Y2[k];
                        const float u_inf = (Y1[k] * a.Eex + Y2[k] * a.Ein + a.Ie) / G;
                        u_new = u_inf + (U[k] - u_inf) * expf(-a.dt_C * G);
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
                    } else if (MODEL == CORTEX_MODEL_COND) {
                        const float ext = a.w_ext * (float)kc;   // into the channel of its sign
                        Y1[k] = a.P11 * Y1[k] + x + (ext >= 0.f ? ext : 0.f);
                        Y2[k] = a.P11 * Y2[k] + x_in + (ext < 0.f ? -ext : 0.f);
                        x = x - x_in;   // the trace records the signed sum of the arrivals
                    }
                    const bool spk = a.frz_ptr ? ((frz >> si) & 1u) != 0 : (integ && u_new >= a.theta);
                    if (spk) {
                        u_new = a.Ur;
                        RF[k] = a.n_ref;
                        const int p = atomicAdd(&s_cnt[si], 1);
                        s_spk[si * T + p] = (uint32_t)(g0 + li);
                    }
                    U[k] = u_new;
                    const size_t ti = (size_t)(n - a.n0) * a.N + g0 + li;
                    if (a.x_trace) a.x_trace[ti] = x;
                    if (a.v_trace) a.v_trace[ti] = u_new + a.E_L;
                    if (a.m_trace) a.m_trace[ti] = (integ && !spk) ? 1 : 0;
                }
                if (a.frz_ptr) s_frz[li] = 0;
            }
        }
        __syncthreads();
        // -------------------------------------------------------- publish
        // id words first, then the step's count word; a reader validates the
        // step tag of every word it uses, so no ordering between them is needed
        for (int si = 0; si < wn; ++si) {
            const int64_t n = t0 + si;
            const int c = s_cnt[si];
            const uint64_t tag = (uint64_t)(uint32_t)(n + 1) << 32;
            uint64_t* base = a.pub + (size_t)(n & (H - 1)) * pub_slot + (size_t)tile * pub_tile;
            const uint32_t* ls = s_spk + (size_t)si * T;
            for (int i = tid; i < c; i += bs) coherent_store(base + 1 + i, tag | ls[i]);
            if (tid == si) coherent_store(base, tag | (uint32_t)c);
            if (n >= a.log_step0 && n < a.log_step0 + a.log_steps) {
                if (log_pos + c <= log_cap) {
                    for (int i = tid; i < c; i += bs) a.log_ids[log_b + log_pos + i] = ls[i];
                    if (tid == 0) a.log_cnt[(n - a.log_step0) * a.n_tiles + tile] = (uint32_t)c;
                    log_pos += c;
                } else if (tid == 0) {
                    a.log_cnt[(n - a.log_step0) * a.n_tiles + tile] = 0xFFFFFFFFu;   // overflow mark
                }
            }
            nspk += c;
        }
        __syncthreads();
        if (tid < wn) s_cnt[tid] = 0;
    }
    // ---------------------------------------------------------------- save
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int li = tid + k * bs;
        if (li < tsz) {
            a.U[g0 + li] = U[k];
            a.r[g0 + li] = RF[k];
            if (MODEL != CORTEX_MODEL_DELTA) a.y1[g0 + li] = Y1[k];
            if (MODEL == CORTEX_MODEL_ALPHA || MODEL == CORTEX_MODEL_COND) a.y2[g0 + li] = Y2[k];
        }
    }
    RING* g_ring_out = static_cast<RING*>(a.ring) + (size_t)tile * R * T;
    for (int i = tid; i < R * T; i += bs) g_ring_out[i] = ring[i];
    if (tid == 0) {
        a.events[tile] += ev;
        a.spikes[tile] += nspk;
        a.log_pos[tile] = log_pos;
    }
}

using KernelFn = void (*)(StepArgs);

template <int MODEL, typename META, bool WBF16, typename RING>
KernelFn pick_npt(int npt) {
    if (npt == 1) return step_kernel<MODEL, META, WBF16, 1, RING>;
    if (npt == 2) return step_kernel<MODEL, META, WBF16, 2, RING>;
    return step_kernel<MODEL, META, WBF16, 4, RING>;
}

// Record formats: 16- or 32-bit records with fp32 weights, or packed 32-bit
// words (16-bit record, bf16 weight); bf16 weights need 16-bit records.
template <int MODEL, typename RING>
KernelFn pick_fmt(int meta_bytes, int w_bytes, int npt) {
    if (w_bytes == 2) return meta_bytes == 2 ? pick_npt<MODEL, uint16_t, true, RING>(npt) : nullptr;
    return meta_bytes == 2 ? pick_npt<MODEL, uint16_t, false, RING>(npt) : pick_npt<MODEL, uint32_t, false, RING>(npt);
}

template <typename RING>
KernelFn pick_model(int model, int meta_bytes, int w_bytes, int npt) {
    switch (model) {
        case CORTEX_MODEL_DELTA: return pick_fmt<CORTEX_MODEL_DELTA, RING>(meta_bytes, w_bytes, npt);
        case CORTEX_MODEL_EXP: return pick_fmt<CORTEX_MODEL_EXP, RING>(meta_bytes, w_bytes, npt);
        case CORTEX_MODEL_ALPHA: return pick_fmt<CORTEX_MODEL_ALPHA, RING>(meta_bytes, w_bytes, npt);
        default: return nullptr;
    }
}

// Conductances: two 32-bit channels per 64-bit cell, FP32 weights.
KernelFn pick_cond(int meta_bytes, int w_bytes, int npt) {
    if (w_bytes != 4) return nullptr;
    return meta_bytes == 2 ? pick_npt<CORTEX_MODEL_COND, uint16_t, false, unsigned long long>(npt)
                           : pick_npt<CORTEX_MODEL_COND, uint32_t, false, unsigned long long>(npt);
}

KernelFn pick_variant(int model, int meta_bytes, int w_bytes, int npt, int ring_bytes) {
    if (model == CORTEX_MODEL_COND) return ring_bytes == 8 ? pick_cond(meta_bytes, w_bytes, npt) : nullptr;
    return ring_bytes == 8 ? pick_model<long long>(model, meta_bytes, w_bytes, npt)
                           : pick_model<int>(model, meta_bytes, w_bytes, npt);
}

KernelFn pick_kernel(const cortex_net* n) {
    KernelFn f = pick_variant(n->spec.model, n->meta_bytes, n->w_bytes, n->NPT, n->ring_bytes);
    require(f != nullptr, CORTEX_EUNSUPPORTED, "no step kernel for this record format");
    return f;
}

}  // namespace

size_t step_lds_bytes(int R, int T, int W, int ntiles_max, int chunk, int ring_bytes) {
    size_t b = (size_t)chunk * 16;                // s_sg
    b += (size_t)R * T * ring_bytes;              // ring
    b += (size_t)(chunk + 1) * 4;                 // s_len
    b += (size_t)W * T * 4;                       // s_spk
    const size_t pairs = (size_t)W * ntiles_max;
    b += (pairs + 1) * 4;                         // s_pc
    b += pairs * kInline * 4;                     // s_pid
    b += 20 * 4 + 4 * 4 + 8 * 4 + 20 * 4;         // s_wsum, s_misc, s_cnt, s_kw
    b += (size_t)T * 4;                           // s_frz
    b += (size_t)kMaxThr * 4;                     // s_thr
    b += (size_t)16 * T;                          // s_kcb
    b += (size_t)kDeliverBlk * 4;                 // s_blk
    return (b + 15) & ~(size_t)15;
}

int step_occupancy(int model, int meta_bytes, int w_bytes, int npt, int bs, size_t lds, int ring_bytes) {
    KernelFn f = pick_variant(model, meta_bytes, w_bytes, npt, ring_bytes);
    if (!f) return 0;
    if (hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, bs, lds) != hipSuccess) return 0;
    return nb;
}

int step_max_blocks_per_cu(cortex_net* n) {
    KernelFn f = pick_kernel(n);
    CX_HIP(hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)n->lds_bytes));
    int nb = 0;
    CX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, n->BS, n->lds_bytes));
    return nb;
}

void launch_step_fp32(cortex_net* n, int64_t n_steps, const uint32_t* frz_ids,
                      const uint64_t* frz_ptr, uint64_t frz_n, float* x_trace, float* v_trace,
                      uint8_t* m_trace) {
    if (n_steps <= 0) return;
    require(n->n_thr <= kMaxThr, CORTEX_EUNSUPPORTED, "Poisson mean too large for the FP32 kernel");
    StepArgs a{};
    a.inst_tile0 = n->d_inst_tile0;
    a.inst_ntiles = n->d_inst_ntiles;
    a.inst_T = n->d_inst_T;
    a.inst_n0 = n->d_inst_n0;
    a.inst_offbase = n->d_inst_offbase;
    a.tile_inst = n->d_tile_inst;
    a.tile_size = n->d_tile_size;
    a.seg = n->d_seg;
    a.meta = n->d_meta;
    a.w = n->d_w;
    a.U = n->d_U;
    a.y1 = n->d_y1;
    a.y2 = n->d_y2;
    a.r = n->d_r;
    a.ring = n->d_ring;
    a.pub = n->d_pub;
    a.log_cnt = n->d_log_cnt;
    a.log_ids = n->d_log_ids;
    a.log_base = n->d_log_base;
    a.log_pos = n->d_log_pos;
    a.events = n->d_events;
    a.spikes = n->d_spikes;
    a.err = n->d_err;
    a.frz_ids = frz_ids;
    a.frz_ptr = frz_ptr;
    a.frz_n = frz_n;
    a.x_trace = x_trace;
    a.v_trace = v_trace;
    a.m_trace = m_trace;
    a.n0 = n->step;
    a.n1 = n->step + n_steps;
    a.log_step0 = n->log_step0;
    a.log_steps = n->log_steps;
    a.N = n->N;
    a.n_tiles = n->n_tiles;
    a.T = n->T;
    a.R = n->R;
    a.dmin = n->dmin;
    a.H = n->H;
    a.W = n->W;
    a.chunk = n->chunk;
    a.n_ref = n->k.n_ref;
    a.n_thr = n->n_thr;
    a.xcd = n->xcd_map;
    a.spin_log2 = n->spec.spin_limit_log2 > 0 ? n->spec.spin_limit_log2 : 22;
    a.ntb_max = n->ntb_max;
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
    // weights are rounded at 2^(fx - fx_shift) and summed in those units
    a.fxw_scale = std::ldexp(1.0f, n->fx - n->fx_shift);
    a.fx_inv = std::ldexp(1.0, n->fx_shift - n->fx);
    a.gL = (float)(n->spec.C_m / n->spec.tau_m);
    a.Eex = (float)(n->spec.E_ex - n->spec.E_L);
    a.Ein = (float)(n->spec.E_in - n->spec.E_L);
    a.Ie = (float)n->spec.I_e;
    a.dt_C = (float)(n->spec.dt / n->spec.C_m);
    a.seed = n->seed;
    for (int m = 0; m < n->n_thr; ++m) a.thr[m] = n->thr[m];
    KernelFn f = pick_kernel(n);
    CX_HIP(hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)n->lds_bytes));
    void* params[] = {&a};
    CX_HIP(hipLaunchCooperativeKernel((const void*)f, dim3(n->n_tiles), dim3(n->BS), params,
                                      (unsigned)n->lds_bytes, n->stream));
    n->step += n_steps;
}

}  // namespace cortex
