// On-device network generation and indegree-tile layout.
//
// Every synapse is a pure function of its canonical position (target,
// projection, slot) and the Philox key, so the device regenerates the graph
// instead of reading it from the host.  The production layout stores, for
// each source j, its out-synapses grouped by destination tile: the tile that
// owns a target owns every synapse into it (the indegree sub-graph of Eq. 5,
// one per tile as in Eq. 9-10), and the segment (j, tile) is exactly the part
// of the spiking sub-graph (Eq. 11) that tile must read when j spikes
// (Sec. III-B, Fig. data_ins (c)).  The records of one segment are contiguous
// and segments of neighbouring tiles are adjacent, so a spike's synapses are
// read as one contiguous stream across the tiles.
//
// Build: (1) count synapses per (source, tile); (2) scan rows into segment
// offsets and sources into row starts; (3) regenerate and scatter every
// synapse into its segment.  The FP64 verification layout instead keeps, per
// target, its in-synapses sorted by (delay descending, source, canonical
// index), the order in which a pull reproduces the push summation order.
//
// This file is compiled with -ffp-contract=off: weights and delays are
// produced by the same unfused FP64 operations as the CPU reference recipe.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

enum GenMode : int {
    kCountTiles = 0,   // count per (source, tile) [+ per item]
    kFillTiles = 1,    // scatter into the tile layout
    kCountItems = 2,   // count per (target, projection) only
    kFillCanon = 3     // write canonical in-edge arrays (FP64 verify)
};

struct GenArgs {
    const GenBlock* blocks;
    const int64_t* blk_item0;   // [n_blocks + 1]
    int n_blocks;
    int64_t n_items;
    uint64_t seed;
    double dt;
    // tile layout
    uint32_t* cnt;              // [sum N_b (nt_b + 1)] counts, then cursors
    const uint64_t* inst_offbase;
    const int32_t* inst_ntiles;
    const int32_t* inst_T;      // tile size per instance
    const uint64_t* row_start;
    const uint32_t* off_rel;
    void* meta;
    void* w;
    int T;          // ring row stride: a record is (delay - dmin) T + target in tile
    int dmin;
    int meta16;
    int wbf16;
    // canonical positions
    uint32_t* cnt_item;         // [n_items]
    const uint32_t* item_rel;   // [n_items] offset of the item inside its target
    const uint64_t* cin;        // [N + 1] canonical start of each target
    uint32_t* canon_out;        // [E] canonical index of each stored synapse
    uint32_t* csrc_out;         // [E] source of each canonical synapse
    uint16_t* cdel_out;         // [E] delay (steps) of each canonical synapse
    // FP64 verify arrays (canonical order)
    uint32_t* in_src;
    double* in_w;
    uint16_t* in_d;
    int32_t* dminmax;           // [2]
};

__device__ __forceinline__ int32_t steps_of(double ms, double dt) {
    const double x = ms / dt + 0.5;
    const double f = floor(x);
    if (f < 1.0) return 1;
    if (f > 1e9) return 1000000000;
    return (int32_t)f;
}

struct Draw {
    int64_t src_in_pop;
    int32_t d;
    double w;
};

// Draws of synapse (target tl, projection, slot): counter (tl, slot, proj,
// edge tag); word 0 -> source, word 1 -> integer delay, words 2, 3 ->
// Box-Muller pair (first normal: weight, second normal: normal delay).
__device__ __forceinline__ Draw draw_edge(const GenBlock& B, uint64_t seed, int64_t tl,
                                          int64_t slot, int64_t t_in_pop, double dt,
                                          int64_t given_src) {
    const Philox4 p = philox((uint64_t)tl, (uint64_t)slot, (uint64_t)B.proj_local, kTagEdge,
                             seed, (uint64_t)B.instance);
    Draw r;
    if (given_src >= 0) {
        r.src_in_pop = given_src;
    } else if (B.same_pop_no_autapse) {
        int64_t s = (int64_t)uniform_below(p.v[0], (uint64_t)(B.n_src - 1));
        r.src_in_pop = s + (s >= t_in_pop ? 1 : 0);
    } else {
        r.src_in_pop = (int64_t)uniform_below(p.v[0], (uint64_t)B.n_src);
    }
    double z0 = 0.0, z1 = 0.0;
    if (B.w_sd != 0.0 || B.delay_kind == CORTEX_DELAY_NORMAL) {
        const double u1 = unit_open0(p.v[2]);
        const double u2 = unit_closed0(p.v[3]);
        const double rad = sqrt(-2.0 * log(u1));
        const double ang = 6.283185307179586 * u2;
        z0 = rad * cos(ang);
        z1 = rad * sin(ang);
    }
    double w;
    if (B.w_sd == 0.0) {
        w = B.w_mean;
    } else {
        const double t = B.w_sd * z0;
        w = B.w_mean + t;
        if (B.w_mean > 0.0 && w < 0.0) w = 0.0;
        if (B.w_mean < 0.0 && w > 0.0) w = 0.0;
    }
    r.w = w;   // unit conversion applied by the caller
    if (B.delay_kind == CORTEX_DELAY_CONST) {
        r.d = steps_of(B.d0, dt);
    } else if (B.delay_kind == CORTEX_DELAY_UNIFORM_INT) {
        const int64_t lo = (int64_t)B.d0, hi = (int64_t)B.d1;
        r.d = (int32_t)(lo + (int64_t)uniform_below(p.v[1], (uint64_t)(hi - lo + 1)));
    } else {
        const double t = B.d1 * z1;
        r.d = steps_of(B.d0 + t, dt);
    }
    return r;
}

// bf16 with round-to-nearest-even from a double: round to float toward zero
// with a sticky bit (round-to-odd), then to nearest-even at 8 mantissa bits.
__device__ __forceinline__ uint16_t to_bf16(double x) {
    float f = __double2float_rz(x);
    uint32_t u = __float_as_uint(f);
    if ((double)f != x) u |= 1u;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <int MODE>
__device__ __forceinline__ void emit(const GenArgs& a, const GenBlock& B, int64_t tgt_global,
                                     int64_t tl, int64_t item, int64_t slot, const Draw& dr,
                                     double conv, int& dlo, int& dhi) {
    const int64_t src_global = B.inst_n0 + B.src0_local + dr.src_in_pop;
    const double w = (conv != 1.0) ? dr.w * conv : dr.w;
    if (MODE == kCountTiles || MODE == kCountItems) {
        dlo = min(dlo, dr.d);
        dhi = max(dhi, dr.d);
    }
    if (MODE == kCountTiles || MODE == kFillTiles) {
        const int ntb = a.inst_ntiles[B.instance];
        const int Tb = a.inst_T[B.instance];
        const int64_t tile_local = tl / Tb;
        const uint64_t key = a.inst_offbase[B.instance] +
                             (uint64_t)(B.src0_local + dr.src_in_pop) * (uint64_t)(ntb + 1) +
                             (uint64_t)tile_local;
        if (MODE == kCountTiles) {
            atomicAdd(&a.cnt[key], 1u);
        } else {
            const uint32_t k = atomicAdd(&a.cnt[key], 1u);
            const uint64_t pos = a.row_start[src_global] + a.off_rel[key] + k;
            const uint32_t m = (uint32_t)(tl - tile_local * Tb) + (uint32_t)(dr.d - a.dmin) * (uint32_t)a.T;
            if (a.wbf16) {
                // packed record: bf16 weight in the high half, 16-bit record below
                static_cast<uint32_t*>(a.meta)[pos] = ((uint32_t)to_bf16(w) << 16) | m;
            } else {
                if (a.meta16) static_cast<uint16_t*>(a.meta)[pos] = (uint16_t)m;
                else static_cast<uint32_t*>(a.meta)[pos] = m;
                static_cast<float*>(a.w)[pos] = (float)w;
            }
            if (a.canon_out) {
                const uint64_t c = a.cin[tgt_global] + a.item_rel[item] + slot;
                a.canon_out[pos] = (uint32_t)c;
                a.csrc_out[c] = (uint32_t)src_global;
                a.cdel_out[c] = (uint16_t)dr.d;
            }
        }
    }
    if (MODE == kFillCanon) {
        const uint64_t pos = a.cin[tgt_global] + a.item_rel[item] + slot;
        a.in_src[pos] = (uint32_t)src_global;
        a.in_w[pos] = w;
        a.in_d[pos] = (uint16_t)dr.d;
    }
}

// One wave per (target, projection) item.
template <int MODE>
__global__ void __launch_bounds__(256) gen_kernel(GenArgs a, double conv) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t item = wave; item < a.n_items; item += n_waves) {
        int lo = 0, hi = a.n_blocks;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.blk_item0[mid] <= item) lo = mid; else hi = mid;
        }
        const GenBlock B = a.blocks[lo];
        const int64_t t_in_pop = item - a.blk_item0[lo];
        const int64_t tgt = B.tgt0 + t_in_pop;
        const int64_t tl = tgt - B.inst_n0;
        // delay range of the item's synapses (count passes): kept per lane,
        // reduced over the wave, one atomic per item
        int dlo = 0x7FFFFFFF, dhi = 0;
        if (B.rule == CORTEX_RULE_FIXED_INDEGREE) {
            for (int64_t s = lane; s < B.k; s += 64) {
                const Draw dr = draw_edge(B, a.seed, tl, s, t_in_pop, a.dt, -1);
                emit<MODE>(a, B, tgt, tl, item, s, dr, conv, dlo, dhi);
            }
            if ((MODE == kCountTiles || MODE == kCountItems) && a.cnt_item && lane == 0)
                a.cnt_item[item] = (uint32_t)B.k;
        } else {
            uint32_t run = 0;
            for (int64_t j0 = 0; j0 < B.n_src; j0 += 64) {
                const int64_t j = j0 + lane;
                bool conn = false;
                if (j < B.n_src) {
                    const Philox4 p = philox((uint64_t)tl, (uint64_t)(j >> 2), (uint64_t)B.proj_local,
                                             kTagPair, a.seed, (uint64_t)B.instance);
                    conn = (B.all_pairs || philox_word(p, (uint32_t)(j & 3)) < B.thr_p) &&
                           !(B.same_pop_no_autapse && j == t_in_pop);
                }
                const uint64_t mask = __ballot(conn);
                if (conn) {
                    const uint64_t below = mask & ((1ull << lane) - 1ull);
                    const int64_t slot = run + (uint32_t)__popcll(below);
                    const Draw dr = draw_edge(B, a.seed, tl, slot, t_in_pop, a.dt, j);
                    emit<MODE>(a, B, tgt, tl, item, slot, dr, conv, dlo, dhi);
                }
                run += (uint32_t)__popcll(mask);
            }
            if ((MODE == kCountTiles || MODE == kCountItems) && a.cnt_item && lane == 0)
                a.cnt_item[item] = run;
        }
        if (MODE == kCountTiles || MODE == kCountItems) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                dlo = min(dlo, __shfl_xor(dlo, off, 64));
                dhi = max(dhi, __shfl_xor(dhi, off, 64));
            }
            if (lane == 0 && dhi > 0) {
                atomicMin(&a.dminmax[0], dlo);
                atomicMax(&a.dminmax[1], dhi);
            }
        }
    }
}

// Per source row: exclusive scan of its per-tile counts into segment offsets
// (last entry = out-degree).  One wave per row.
__global__ void __launch_bounds__(256) row_scan_kernel(const uint32_t* cnt, uint32_t* off_rel,
                                                       uint32_t* outdeg, const int64_t* inst_n0,
                                                       const uint64_t* inst_offbase,
                                                       const int32_t* inst_ntiles, int n_inst,
                                                       int64_t N) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < N; j += n_waves) {
        int lo = 0, hi = n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (inst_n0[mid] <= j) lo = mid; else hi = mid;
        }
        const int nt = inst_ntiles[lo];
        const uint64_t base = inst_offbase[lo] + (uint64_t)(j - inst_n0[lo]) * (uint64_t)(nt + 1);
        uint32_t carry = 0;
        for (int t0 = 0; t0 < nt; t0 += 64) {
            const int t = t0 + lane;
            const uint32_t c = (t < nt) ? cnt[base + t] : 0u;
            const uint32_t inc = wave_incl_scan(c);
            if (t < nt) off_rel[base + t] = carry + inc - c;
            carry += __shfl(inc, 63, 64);
        }
        if (lane == 0) {
            off_rel[base + nt] = carry;
            outdeg[j] = carry;
        }
    }
}

// Segment descriptors: seg[j][t] = (first synapse << 24) | length of the
// synapses of source j into tile t, one 64-bit word per segment, so that a
// kernel finds a segment with a single load (the entry after a row's last
// tile is 0).  One wave per source row; *bad is set if a first synapse or a
// length does not fit its field.
__global__ void __launch_bounds__(256) seg_kernel(const uint64_t* row_start, const uint32_t* off_rel, uint64_t* seg,
                                                  const int64_t* inst_n0, const uint64_t* inst_offbase,
                                                  const int32_t* inst_ntiles, int n_inst, int64_t N, int32_t* bad) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t j = wave; j < N; j += n_waves) {
        int lo = 0, hi = n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (inst_n0[mid] <= j) lo = mid; else hi = mid;
        }
        const int nt = inst_ntiles[lo];
        const uint64_t base = inst_offbase[lo] + (uint64_t)(j - inst_n0[lo]) * (uint64_t)(nt + 1);
        const uint64_t rs = row_start[j];
        for (int t = lane; t <= nt; t += 64) {
            uint64_t v = 0;
            if (t < nt) {
                const uint64_t first = rs + off_rel[base + t];
                const uint64_t len = off_rel[base + t + 1] - off_rel[base + t];
                if (first >= (1ull << 40) || len >= (1ull << 24)) atomicOr(bad, 1);
                v = (first << 24) | len;
            }
            seg[base + t] = v;
        }
    }
}

// Exclusive scan of n 32-bit counts into n + 1 64-bit prefixes by one
// workgroup of 1024 threads (setup only).
__global__ void __launch_bounds__(1024) scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n) {
    __shared__ uint64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t beg = min(n, (int64_t)tid * per), end = min(n, beg + per);
    uint64_t s = 0;
    for (int64_t i = beg; i < end; ++i) s += in[i];
    part[tid] = s;
    __syncthreads();
    if (tid == 0) {
        uint64_t acc = 0;
        for (int i = 0; i < 1024; ++i) { uint64_t t = part[i]; part[i] = acc; acc += t; }
        out[n] = acc;
    }
    __syncthreads();
    uint64_t run = part[tid];
    for (int64_t i = beg; i < end; ++i) { out[i] = run; run += in[i]; }
}

// Canonical offsets: per target, the start of each of its items inside the
// target (projections in order) and the in-degree.
__global__ void item_offsets_kernel(const uint32_t* cnt_item, uint32_t* item_rel, uint32_t* indeg,
                                    const int64_t* pop_t0, const int32_t* pop_blk0,
                                    const int32_t* pop_blk1, int n_pops, const int64_t* blk_item0,
                                    const GenBlock* blocks, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int lo = 0, hi = n_pops;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pop_t0[mid] <= i) lo = mid; else hi = mid;
    }
    uint32_t run = 0;
    for (int b = pop_blk0[lo]; b < pop_blk1[lo]; ++b) {
        const int64_t item = blk_item0[b] + (i - blocks[b].tgt0);
        item_rel[item] = run;
        run += cnt_item[item];
    }
    indeg[i] = run;
}

// Per target, stable merge sort of its canonical in-edges by
// (delay descending, source ascending).  Setup of the FP64 verify layout.
__global__ void sort_in_edges_kernel(const uint64_t* in_ptr, uint32_t* src, double* w, uint16_t* d,
                                     uint32_t* canon, uint64_t* key_a, uint64_t* key_b,
                                     uint32_t* idx_a, uint32_t* idx_b, uint32_t* src_tmp,
                                     double* w_tmp, uint16_t* d_tmp, int64_t N) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const uint64_t b = in_ptr[i], n = in_ptr[i + 1] - b;
    if (n < 2) {
        if (n == 1) canon[b] = (uint32_t)b;
        return;
    }
    for (uint64_t q = 0; q < n; ++q) {
        key_a[b + q] = ((uint64_t)(0xFFFFu - d[b + q]) << 32) | src[b + q];
        idx_a[b + q] = (uint32_t)q;
    }
    uint64_t* kin = key_a + b; uint64_t* kout = key_b + b;
    uint32_t* iin = idx_a + b; uint32_t* iout = idx_b + b;
    for (uint64_t width = 1; width < n; width *= 2) {
        for (uint64_t lo = 0; lo < n; lo += 2 * width) {
            const uint64_t mid = min(lo + width, n), hi = min(lo + 2 * width, n);
            uint64_t x = lo, y = mid, o = lo;
            while (x < mid && y < hi) {
                if (kin[y] < kin[x]) { kout[o] = kin[y]; iout[o++] = iin[y++]; }
                else { kout[o] = kin[x]; iout[o++] = iin[x++]; }
            }
            while (x < mid) { kout[o] = kin[x]; iout[o++] = iin[x++]; }
            while (y < hi) { kout[o] = kin[y]; iout[o++] = iin[y++]; }
        }
        uint64_t* tk = kin; kin = kout; kout = tk;
        uint32_t* ti = iin; iin = iout; iout = ti;
    }
    for (uint64_t q = 0; q < n; ++q) {
        const uint32_t from = iin[q];
        src_tmp[b + q] = src[b + from];
        w_tmp[b + q] = w[b + from];
        d_tmp[b + q] = d[b + from];
        canon[b + q] = (uint32_t)(b + from);
    }
    for (uint64_t q = 0; q < n; ++q) {
        src[b + q] = src_tmp[b + q];
        w[b + q] = w_tmp[b + q];
        d[b + q] = d_tmp[b + q];
    }
}

// Initial state: V0 uniform on [v0_lo, v0_hi) from word 0 of the block
// (neuron, 0, 0, V0 tag); refractory counters and synaptic state zero.
__global__ void init_state_kernel(const int64_t* inst_n0, int n_inst, int64_t N, uint64_t seed,
                                  double v0_lo, double v0_hi, double E_L, float* U32,
                                  double* U64, float* U32copy, double* U64copy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (inst_n0[mid] <= i) lo = mid; else hi = mid;
    }
    const Philox4 p = philox((uint64_t)(i - inst_n0[lo]), 0, 0, kTagV0, seed, (uint64_t)lo);
    const double u = unit_closed0(p.v[0]);
    const double span = v0_hi - v0_lo;
    const double t = span * u;
    const double v = v0_lo + t;
    const double U = v - E_L;
    if (U32) { U32[i] = (float)U; U32copy[i] = (float)U; }
    if (U64) { U64[i] = U; U64copy[i] = U; }
}

int grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (int)g;
}

struct Tables {
    GenBlock* blocks = nullptr;
    int64_t* blk_item0 = nullptr;
    int n_blocks = 0;
    int64_t n_items = 0;
    std::vector<int64_t> h_blk_item0;
    int64_t* pop_t0 = nullptr;
    int32_t* pop_blk0 = nullptr;
    int32_t* pop_blk1 = nullptr;
    int n_pops = 0;
};

Tables upload_tables(cortex_net* n) {
    Tables t;
    t.n_blocks = (int)n->blocks.size();
    t.h_blk_item0.resize(t.n_blocks + 1, 0);
    for (int b = 0; b < t.n_blocks; ++b) t.h_blk_item0[b + 1] = t.h_blk_item0[b] + n->blocks[b].n_tgt;
    t.n_items = t.h_blk_item0[t.n_blocks];
    t.blocks = dev_alloc_t<GenBlock>(n, std::max(1, t.n_blocks), true);
    t.blk_item0 = dev_alloc_t<int64_t>(n, t.n_blocks + 1, true);
    if (t.n_blocks)
        CX_HIP(hipMemcpyAsync(t.blocks, n->blocks.data(), t.n_blocks * sizeof(GenBlock),
                              hipMemcpyHostToDevice, n->stream));
    CX_HIP(hipMemcpyAsync(t.blk_item0, t.h_blk_item0.data(), (t.n_blocks + 1) * sizeof(int64_t),
                          hipMemcpyHostToDevice, n->stream));
    // population table (global populations, in order)
    std::vector<int64_t> pt0;
    std::vector<int32_t> pb0, pb1;
    int64_t g = 0;
    int bi = 0;
    for (size_t p = 0; p < n->pops.size(); ++p) {
        pt0.push_back(g);
        pb0.push_back(bi);
        while (bi < t.n_blocks && n->blocks[bi].tgt0 == g) ++bi;
        pb1.push_back(bi);
        g += n->pops[p].size;
    }
    t.n_pops = (int)pt0.size();
    t.pop_t0 = dev_alloc_t<int64_t>(n, t.n_pops, true);
    t.pop_blk0 = dev_alloc_t<int32_t>(n, t.n_pops, true);
    t.pop_blk1 = dev_alloc_t<int32_t>(n, t.n_pops, true);
    CX_HIP(hipMemcpyAsync(t.pop_t0, pt0.data(), t.n_pops * sizeof(int64_t), hipMemcpyHostToDevice, n->stream));
    CX_HIP(hipMemcpyAsync(t.pop_blk0, pb0.data(), t.n_pops * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
    CX_HIP(hipMemcpyAsync(t.pop_blk1, pb1.data(), t.n_pops * sizeof(int32_t), hipMemcpyHostToDevice, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));   // the host tables above go out of scope
    return t;
}

GenArgs base_args(cortex_net* n, const Tables& t) {
    GenArgs a{};
    a.blocks = t.blocks;
    a.blk_item0 = t.blk_item0;
    a.n_blocks = t.n_blocks;
    a.n_items = t.n_items;
    a.seed = n->seed;
    a.dt = n->spec.dt;
    a.inst_offbase = n->d_inst_offbase;
    a.inst_ntiles = n->d_inst_ntiles;
    a.inst_T = n->d_inst_T;
    return a;
}

template <int MODE>
void run_gen(cortex_net* n, const GenArgs& a) {
    if (a.n_items == 0) return;
    const int grid = grid_for(a.n_items * 64, 256);
    hipLaunchKernelGGL(gen_kernel<MODE>, dim3(grid), dim3(256), 0, n->stream, a, n->k.conv);
    CX_HIP(hipGetLastError());
}

// Canonical offsets (cnt_item -> item_rel, cin); returns the edge count.
int64_t canonical_offsets(cortex_net* n, const Tables& t, uint32_t* cnt_item, uint32_t* item_rel,
                          uint64_t* cin) {
    uint32_t* indeg = dev_alloc_t<uint32_t>(n, n->N, true);
    hipLaunchKernelGGL(item_offsets_kernel, dim3(grid_for(n->N, 256)), dim3(256), 0, n->stream,
                       cnt_item, item_rel, indeg, t.pop_t0, t.pop_blk0, t.pop_blk1, t.n_pops,
                       t.blk_item0, t.blocks, n->N);
    CX_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_u32_to_u64, dim3(1), dim3(1024), 0, n->stream, indeg, cin, n->N);
    CX_HIP(hipGetLastError());
    uint64_t E = 0;
    CX_HIP(hipMemcpyAsync(&E, cin + n->N, sizeof(uint64_t), hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    return (int64_t)E;
}

}  // namespace

void delay_range(cortex_net* n, int* dmin, int* dmax) {
    Tables t = upload_tables(n);
    int32_t* dmm = dev_alloc_t<int32_t>(n, 2, true);
    const int32_t dinit[2] = {1 << 30, 0};
    CX_HIP(hipMemcpyAsync(dmm, dinit, sizeof dinit, hipMemcpyHostToDevice, n->stream));
    GenArgs a = base_args(n, t);
    a.dminmax = dmm;
    run_gen<kCountItems>(n, a);
    int32_t dm[2];
    CX_HIP(hipMemcpyAsync(dm, dmm, sizeof dm, hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    *dmin = dm[1] == 0 ? 1 : dm[0];
    *dmax = dm[1] == 0 ? 1 : dm[1];
}

namespace {

// Per target, the sum of |w| over its stored in-synapses (the largest value
// any of its input sums can reach), and the largest |w|.  One workgroup per
// tile (the tile owns its targets' in-synapses, so the sums stay in LDS):
// lanes take the instance's sources, each walks its segment into the tile
// through the one-load segment descriptors; LDS FP64 atomics per synapse,
// one global maximum per workgroup.  Setup only.
__global__ void __launch_bounds__(1024) abs_input_kernel(const uint64_t* seg, const void* meta, int meta16,
                                                         const void* w, int wbf16, int T,
                                                         const int32_t* tile_inst, const int32_t* tile_size,
                                                         const int32_t* inst_tile0, const int32_t* inst_ntiles,
                                                         const int32_t* inst_T, const int64_t* inst_n0,
                                                         const int64_t* inst_N, const uint64_t* inst_offbase,
                                                         int64_t plo, int64_t phi, float w_plastic,
                                                         double* tile_max, unsigned int* wmax_bits) {
    extern __shared__ double s_sum[];   // [T]
    __shared__ unsigned int s_wmax;
    const int tile = blockIdx.x;
    const int b = tile_inst[tile];
    const int tl = tile - inst_tile0[b];
    const int ntb = inst_ntiles[b];
    const int tsz = tile_size[tile];
    const int64_t n0b = inst_n0[b], Nb = inst_N[b];
    const uint64_t offb = inst_offbase[b];
    const int64_t g0 = n0b + (int64_t)tl * inst_T[b];
    for (int i = threadIdx.x; i < T; i += blockDim.x) s_sum[i] = 0.0;
    if (threadIdx.x == 0) s_wmax = 0u;
    __syncthreads();
    unsigned int my_max = 0u;
    for (int64_t j = threadIdx.x; j < Nb; j += blockDim.x) {
        const uint64_t d = seg[offb + (uint64_t)j * (uint64_t)(ntb + 1) + (uint64_t)tl];
        const uint64_t e0 = d >> 24, e1 = e0 + (d & 0xFFFFFFu);
        for (uint64_t e = e0; e < e1; ++e) {
            uint32_t m;
            float wv;
            if (wbf16) {
                const uint32_t r = static_cast<const uint32_t*>(meta)[e];
                m = r & 0xFFFFu;
                wv = __uint_as_float(r & 0xFFFF0000u);
            } else {
                m = meta16 ? static_cast<const uint16_t*>(meta)[e] : static_cast<const uint32_t*>(meta)[e];
                wv = static_cast<const float*>(w)[e];
            }
            // a plastic synapse (source and target in [plo, phi)) may grow to w_plastic
            const int64_t tg = g0 + (int64_t)(m % (uint32_t)T);
            const bool plastic = n0b + j >= plo && n0b + j < phi && tg >= plo && tg < phi;
            const float aw = plastic ? fmaxf(w_plastic, fabsf(wv)) : fabsf(wv);
            atomicAdd(&s_sum[m % (uint32_t)T], (double)aw);
            my_max = max(my_max, __float_as_uint(aw));   // non-negative floats order as integers
        }
    }
    atomicMax(&s_wmax, my_max);
    __syncthreads();
    // the tile's largest sum: per thread, per wave, then over the waves
    __shared__ double s_wave[16];
    double mx = 0.0;
    for (int i = threadIdx.x; i < tsz; i += blockDim.x) mx = fmax(mx, s_sum[i]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t = fmax(t, s_wave[k]);
        tile_max[tile] = t;
        atomicMax(wmax_bits, s_wmax);
    }
}

}  // namespace

double max_abs_input(cortex_net* n, double* wmax) {
    double* tmax = dev_alloc_t<double>(n, std::max(1, n->n_tiles), true);
    unsigned int* wbits = dev_alloc_t<unsigned int>(n, 1, true);
    int64_t* inst_N = dev_alloc_t<int64_t>(n, n->n_inst, true);
    dev_zero(n, wbits, sizeof(unsigned int));
    CX_HIP(hipMemcpyAsync(inst_N, n->inst_N.data(), n->n_inst * sizeof(int64_t), hipMemcpyHostToDevice, n->stream));
    const size_t lds = (size_t)n->T * sizeof(double);
    require(lds <= n->dd.lds_cu, CORTEX_EUNSUPPORTED, "tile too large for the input-bound pass");
    CX_HIP(hipFuncSetAttribute((const void*)abs_input_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(abs_input_kernel, dim3(n->n_tiles), dim3(1024), lds, n->stream, n->d_seg, n->d_meta,
                       n->meta_bytes == 2 ? 1 : 0, n->d_w, n->w_bytes == 2 ? 1 : 0, n->T, n->d_tile_inst,
                       n->d_tile_size, n->d_inst_tile0, n->d_inst_ntiles, n->d_inst_T, n->d_inst_n0, inst_N,
                       n->d_inst_offbase, n->stdp ? n->stdp_lo : (int64_t)0, n->stdp ? n->stdp_hi : (int64_t)0,
                       (float)n->stdp_wmax, tmax, wbits);
    CX_HIP(hipGetLastError());
    std::vector<double> h((size_t)n->n_tiles);
    unsigned int wb = 0;
    CX_HIP(hipMemcpyAsync(h.data(), tmax, h.size() * sizeof(double), hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipMemcpyAsync(&wb, wbits, sizeof wb, hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    double m = 0.0;
    for (double v : h) m = std::max(m, v);
    if (wmax) {
        float wf;
        std::memcpy(&wf, &wb, sizeof wf);
        *wmax = wf;
    }
    return m;
}

namespace {
// Stored weight of every synapse from a canonical-order array (setup).
__global__ void set_weights_kernel(const float* w_canon, const uint32_t* canon, void* w, void* meta, int wbf16,
                                   int64_t E) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const float v = w_canon[canon[e]];
        if (wbf16) {
            uint32_t* r = static_cast<uint32_t*>(meta) + e;
            *r = (*r & 0xFFFFu) | ((uint32_t)to_bf16((double)v) << 16);
        } else {
            static_cast<float*>(w)[e] = v;
        }
    }
}
}  // namespace

void scan_counts(cortex_net* n, const uint32_t* in, uint64_t* out, int64_t count) {
    hipLaunchKernelGGL(scan_u32_to_u64, dim3(1), dim3(1024), 0, n->stream, in, out, count);
    CX_HIP(hipGetLastError());
}

void set_weights_fp32(cortex_net* n, const float* w_canonical) {
    if (n->E == 0) return;
    hipLaunchKernelGGL(set_weights_kernel, dim3(grid_for(n->E, 256)), dim3(256), 0, n->stream, w_canonical,
                       n->d_canon, n->d_w, n->d_meta, n->w_bytes == 2 ? 1 : 0, n->E);
    CX_HIP(hipGetLastError());
}

void build_graph_fp32(cortex_net* n) {
    Tables t = upload_tables(n);
    // per-(source, tile) counts
    uint64_t cnt_len = 0;
    for (int b = 0; b < n->n_inst; ++b) cnt_len += (uint64_t)n->inst_N[b] * (n->inst_ntiles[b] + 1);
    uint32_t* cnt = dev_alloc_t<uint32_t>(n, cnt_len, true);
    dev_zero(n, cnt, cnt_len * sizeof(uint32_t));
    int32_t* dmm = dev_alloc_t<int32_t>(n, 2, true);
    const int32_t dinit[2] = {1 << 30, 0};
    CX_HIP(hipMemcpyAsync(dmm, dinit, sizeof dinit, hipMemcpyHostToDevice, n->stream));
    const bool need_canon = n->ckpt > 0;
    uint32_t* cnt_item = need_canon ? dev_alloc_t<uint32_t>(n, t.n_items, true) : nullptr;
    GenArgs a = base_args(n, t);
    a.cnt = cnt;
    a.dminmax = dmm;
    a.cnt_item = cnt_item;
    run_gen<kCountTiles>(n, a);
    int32_t dm[2];
    CX_HIP(hipMemcpyAsync(dm, dmm, sizeof dm, hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    // the plan fixed the delay range (ring slots) before generation
    require(dm[1] == 0 || (dm[0] >= n->dmin && dm[1] <= n->dmax), CORTEX_EDEVICE,
            "generated delays outside the planned range");
    // segment offsets and row starts
    n->d_off_rel = dev_alloc_t<uint32_t>(n, cnt_len);
    uint32_t* outdeg = dev_alloc_t<uint32_t>(n, n->N, true);
    n->d_row_start = dev_alloc_t<uint64_t>(n, n->N + 1);
    hipLaunchKernelGGL(row_scan_kernel, dim3(grid_for(n->N * 64, 256)), dim3(256), 0, n->stream,
                       cnt, n->d_off_rel, outdeg, n->d_inst_n0, n->d_inst_offbase,
                       n->d_inst_ntiles, n->n_inst, n->N);
    CX_HIP(hipGetLastError());
    hipLaunchKernelGGL(scan_u32_to_u64, dim3(1), dim3(1024), 0, n->stream, outdeg, n->d_row_start, n->N);
    CX_HIP(hipGetLastError());
    uint64_t E = 0;
    CX_HIP(hipMemcpyAsync(&E, n->d_row_start + n->N, sizeof E, hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    n->E = (int64_t)E;
    // one-load segment descriptors for the step kernels
    n->d_seg = dev_alloc_t<uint64_t>(n, cnt_len);
    n->n_seg = cnt_len;
    {
        int32_t* bad = dev_alloc_t<int32_t>(n, 1, true);
        dev_zero(n, bad, sizeof(int32_t));
        hipLaunchKernelGGL(seg_kernel, dim3(grid_for(n->N * 64, 256)), dim3(256), 0, n->stream, n->d_row_start,
                           n->d_off_rel, n->d_seg, n->d_inst_n0, n->d_inst_offbase, n->d_inst_ntiles, n->n_inst,
                           n->N, bad);
        CX_HIP(hipGetLastError());
        int32_t hb = 0;
        CX_HIP(hipMemcpyAsync(&hb, bad, sizeof hb, hipMemcpyDeviceToHost, n->stream));
        CX_HIP(hipStreamSynchronize(n->stream));
        require(hb == 0, CORTEX_EUNSUPPORTED, "a segment is too long (2^24 synapses) or lies past 2^40");
    }
    // record format
    // a record is (delay - dmin) T + target: every record is below R T
    const uint64_t rt = (uint64_t)n->R * (uint64_t)n->T;
    require(rt <= 0xFFFFFFFFull, CORTEX_EUNSUPPORTED, "tile size and delay range too large for 32-bit records");
    n->meta_bytes = (rt <= 65536) ? 2 : 4;
    n->w_bytes = (n->spec.weight_dtype == CORTEX_W_BF16) ? 2 : 4;
    if (n->w_bytes == 2) {
        // bf16 weights: one packed 32-bit word per synapse
        require(n->meta_bytes == 2, CORTEX_EUNSUPPORTED, "bf16 weights need 16-bit records (R x T <= 65536)");
        n->d_meta = dev_alloc(n, (size_t)n->E * 4 + 16);
        n->d_w = nullptr;
    } else {
        n->d_meta = dev_alloc(n, (size_t)n->E * n->meta_bytes + 16);
        n->d_w = dev_alloc(n, (size_t)n->E * n->w_bytes + 16);
    }
    uint32_t* item_rel = nullptr;
    uint64_t* cin = nullptr;
    if (need_canon) {
        require(n->E < (int64_t)0xFFFFFFFFll, CORTEX_EUNSUPPORTED, "adjoint needs fewer than 2^32 synapses");
        require(n->dmax <= 0xFFFF, CORTEX_EUNSUPPORTED, "adjoint needs delays below 65536 steps");
        item_rel = dev_alloc_t<uint32_t>(n, t.n_items, true);
        n->d_cin = dev_alloc_t<uint64_t>(n, n->N + 1);
        cin = n->d_cin;
        const int64_t Ec = canonical_offsets(n, t, cnt_item, item_rel, cin);
        require(Ec == n->E, CORTEX_EDEVICE, "canonical edge count mismatch");
        n->d_canon = dev_alloc_t<uint32_t>(n, n->E);
        n->d_csrc = dev_alloc_t<uint32_t>(n, n->E);
        n->d_cdel = dev_alloc_t<uint16_t>(n, n->E);
    }
    dev_zero(n, cnt, cnt_len * sizeof(uint32_t));
    a.row_start = n->d_row_start;
    a.off_rel = n->d_off_rel;
    a.meta = n->d_meta;
    a.w = n->d_w;
    a.T = n->T;
    a.dmin = n->dmin;
    a.meta16 = n->meta_bytes == 2;
    a.wbf16 = n->w_bytes == 2;
    a.cnt_item = nullptr;
    a.item_rel = item_rel;
    a.cin = cin;
    a.canon_out = n->d_canon;
    a.csrc_out = n->d_csrc;
    a.cdel_out = n->d_cdel;
    run_gen<kFillTiles>(n, a);
    CX_HIP(hipStreamSynchronize(n->stream));
}

void build_graph_fp64(cortex_net* n) {
    Tables t = upload_tables(n);
    int32_t* dmm = dev_alloc_t<int32_t>(n, 2, true);
    const int32_t dinit[2] = {1 << 30, 0};
    CX_HIP(hipMemcpyAsync(dmm, dinit, sizeof dinit, hipMemcpyHostToDevice, n->stream));
    uint32_t* cnt_item = dev_alloc_t<uint32_t>(n, t.n_items, true);
    GenArgs a = base_args(n, t);
    a.dminmax = dmm;
    a.cnt_item = cnt_item;
    run_gen<kCountItems>(n, a);
    uint32_t* item_rel = dev_alloc_t<uint32_t>(n, t.n_items, true);
    n->d_in_ptr = dev_alloc_t<uint64_t>(n, n->N + 1);
    n->E = canonical_offsets(n, t, cnt_item, item_rel, n->d_in_ptr);
    require(n->E < (int64_t)0xFFFFFFFFll, CORTEX_EUNSUPPORTED, "FP64 mode needs fewer than 2^32 synapses");
    int32_t dm[2];
    CX_HIP(hipMemcpyAsync(dm, dmm, sizeof dm, hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    n->dmin = (n->E == 0) ? 1 : dm[0];
    n->dmax = (n->E == 0) ? 1 : dm[1];
    n->R = n->dmax - n->dmin + 1;
    n->d_in_src = dev_alloc_t<uint32_t>(n, n->E);
    n->d_in_w = dev_alloc_t<double>(n, n->E);
    n->d_in_d = dev_alloc_t<uint16_t>(n, n->E);
    n->d_in_canon = dev_alloc_t<uint32_t>(n, n->E);
    require(n->dmax < 0xFFFF, CORTEX_EUNSUPPORTED, "delays must stay below 65535 steps");
    a.cnt_item = nullptr;
    a.item_rel = item_rel;
    a.cin = n->d_in_ptr;
    a.in_src = n->d_in_src;
    a.in_w = n->d_in_w;
    a.in_d = n->d_in_d;
    run_gen<kFillCanon>(n, a);
    // sort every target's in-edges into pull order (scratch freed with the net)
    if (n->E > 0) {
        uint64_t* ka = dev_alloc_t<uint64_t>(n, n->E, true);
        uint64_t* kb = dev_alloc_t<uint64_t>(n, n->E, true);
        uint32_t* ia = dev_alloc_t<uint32_t>(n, n->E, true);
        uint32_t* ib = dev_alloc_t<uint32_t>(n, n->E, true);
        uint32_t* st = dev_alloc_t<uint32_t>(n, n->E, true);
        double* wt = dev_alloc_t<double>(n, n->E, true);
        uint16_t* dtm = dev_alloc_t<uint16_t>(n, n->E, true);
        hipLaunchKernelGGL(sort_in_edges_kernel, dim3(grid_for(n->N, 64)), dim3(64), 0, n->stream,
                           n->d_in_ptr, n->d_in_src, n->d_in_w, n->d_in_d, n->d_in_canon, ka, kb,
                           ia, ib, st, wt, dtm, n->N);
        CX_HIP(hipGetLastError());
    }
    CX_HIP(hipStreamSynchronize(n->stream));
}

void init_state(cortex_net* n) {
    const bool fp64 = n->spec.precision == CORTEX_FP64_VERIFY;
    hipLaunchKernelGGL(init_state_kernel, dim3(grid_for(n->N, 256)), dim3(256), 0, n->stream,
                       n->d_inst_n0, n->n_inst, n->N, n->seed, n->spec.v0_lo, n->spec.v0_hi,
                       n->spec.E_L, fp64 ? nullptr : n->d_U, fp64 ? n->d_Ud : nullptr,
                       fp64 ? nullptr : n->d_U0, fp64 ? n->d_Ud0 : nullptr);
    CX_HIP(hipGetLastError());
}

}  // namespace cortex
