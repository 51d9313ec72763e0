// Tile-major staging of a window's synapse records, for the streamed plan
// when a source's segment into a tile holds only a few synapses (e.g. two
// million neurons in tiles of about a thousand: 5-6 synapses, 22 bytes).
//
// Delivered straight from the graph, every (spike, tile) pair costs the tile
// a cache line of records and a line of its segment descriptor, for some 30
// useful bytes; the segments of one spike into consecutive tiles are
// adjacent in memory (the graph is source-major, tiles in order), but the
// workgroups of those tiles run on different compute units at different
// times and rarely share the lines.  Here one launch per window first copies
// the window's records, spike by spike, from those contiguous source rows
// into a run per tile, so that every line is read once and the delivery
// launch then streams its tile's run.
//
// The sums do not depend on the order of the additions (the ring adds
// 32-bit fixed-point integers), so a tile's run holds its records in any
// order: each copy work item (64 spikes x a group of up to 16 tiles)
// reserves room in a tile's run with one atomic add on the tile's cursor,
// gathers its records into workgroup-local memory tile by tile, and writes
// each tile's share as one contiguous piece (whole cache lines but at the
// share's two ends).  A staged record carries its ring row relative to the
// window's first: meta + qi T, with qi the spike's delivered step in the
// window (below R T, as meta is).  The delivery kernel of the window reads
// the cursor of its tile and resets it; a cursor past the capacity `cap`
// means the run is incomplete, and that tile takes the whole window from
// the graph instead.  One instance only.
#include <algorithm>
#include <type_traits>

#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

constexpr int kGChunk = 64;     // spikes per work item
constexpr int kGTiles = 16;     // at most this many tiles per work item
constexpr int kGMaxQ = 8;       // delivered steps per window
constexpr int kGThreads = 512;  // threads per workgroup
constexpr int kGWaves = kGThreads / 64;
constexpr int kGPer = kGChunk / kGWaves;   // spikes of an item per wave
constexpr int kGU = 4;          // records in flight per lane
constexpr int kGXcd = 8;        // XCDs; workgroup b runs on XCD b mod 8
constexpr int kGatherGrid = 1024;          // four workgroups per compute unit, a multiple of kGXcd
constexpr int kGOutBytes = 29696;          // an item's records in workgroup-local memory

struct GatherArgs {
    const uint64_t* seg;        // (first synapse << 24) | length per (source, tile)
    const void* meta;           // records (packed 32-bit words with bf16 weights)
    const float* w;             // fp32 weights (separate array)
    const uint32_t* spk_cnt;    // [H] spikes per step
    const uint32_t* spk_ids;    // [H][N]
    const int64_t* clock;       // [2] window starts
    unsigned long long* cursor; // [ntb] records reserved in each tile's run
    void* stage;                // [ntb][cap] records: u32 (bf16 packed) or uint2 {meta, weight bits}
    uint64_t offb;              // the instance's first descriptor
    int64_t N;
    uint32_t cap, T;
    int parity, wn, H, dmin, ntb;
    int lg;                     // log2 of the tiles per work item
    KernelTime* ktime;          // launch timing (null: off)
};

struct CopyLds {
    uint32_t out[kGOutBytes / 4];         // the item's records, tile after tile
    uint32_t rel[kGChunk][kGTiles];       // low 32 bits of each segment's first record
    uint32_t dst[kGChunk][kGTiles];       // the segment's place in the item's share of its tile's run
    unsigned long long e0[kGChunk];       // the spike's first record in the tile group
    uint32_t end_lo[kGChunk];             // low 32 bits of the end of its records in the group
    uint32_t j[kGChunk];
    uint32_t qoff[kGChunk];               // ring row of its step, relative to the window's first: qi T
    uint32_t tot[kGTiles];                // the item's records per tile
    uint32_t obase[kGTiles + 1];          // their first place in `out`; obase[kGTiles]: the item's total
    unsigned long long base[kGTiles];     // their place in the tile's run
    uint32_t ok[kGTiles];
    uint32_t wpre[kGWaves][kGPer + 1];    // per wave: prefix of its spikes' record counts
};

// One work item per (64 consecutive spikes of the window, group of G = 2^lg
// tiles).  The item's descriptors go to workgroup-local memory; a
// workgroup-local atomic per segment gives its place in the item's share of
// the tile's run, and one global atomic per tile reserves that share (its
// result is needed only when the shares are written, so the atomics'
// latency overlaps the gathering).  Each wave then takes every kGWaves-th
// spike of the item and walks their records as one flat list (a spike's
// segments into the group are one contiguous range, in tile order), kGU
// records in flight per lane, into the item's buffer; the workgroup then
// writes the buffer out share by share.  An item whose records overflow the
// buffer writes them straight to the runs instead.
//
// The tile groups are split into kGXcd contiguous ranges, one per XCD, and
// an XCD's workgroups take its items spike chunk by spike chunk: the items
// of adjacent groups, which share the cache lines at the ends of each
// spike's row piece and of its descriptors, run at about the same time in
// the same L2, and so do the items that fill adjacent shares of one run.
template <bool WBF16, typename META>
__global__ void __launch_bounds__(kGThreads) __attribute__((amdgpu_waves_per_eu(8))) gather_copy_kernel(GatherArgs a) {
    using Rec = typename std::conditional<WBF16, uint32_t, uint2>::type;
    constexpr uint32_t kOutCap = kGOutBytes / sizeof(Rec);
    extern __shared__ __align__(16) unsigned char lds_raw[];
    if (a.ktime) ktime_mark(a.ktime, 0);
    CopyLds& s = *reinterpret_cast<CopyLds*>(lds_raw);
    Rec* out = reinterpret_cast<Rec*>(s.out);
    Rec* stage = static_cast<Rec*>(a.stage);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // the window's delivered steps and the prefix of their spike counts
    const int64_t t0 = a.clock[a.parity];
    const int64_t q_lo = max((int64_t)0, t0 - a.dmin);
    const int nq = (int)max((int64_t)0, t0 - a.dmin + a.wn - q_lo);
    uint32_t pc[kGMaxQ + 1];
    pc[0] = 0;
#pragma unroll
    for (int qi = 0; qi < kGMaxQ; ++qi)
        pc[qi + 1] = pc[qi] + (qi < nq ? a.spk_cnt[(size_t)((q_lo + qi) & (a.H - 1))] : 0u);
    const uint32_t S = pc[kGMaxQ];
    const uint32_t n_items_s = (S + kGChunk - 1) / kGChunk;
    const int G = 1 << a.lg;
    const uint32_t ngr = ((uint32_t)a.ntb + (uint32_t)G - 1) >> a.lg;
    const uint64_t rowlen = (uint64_t)a.ntb + 1;
    const uint32_t xcd = blockIdx.x % kGXcd, nl = gridDim.x / kGXcd;
    const uint32_t gx0 = ngr * xcd / kGXcd, ngx = ngr * (xcd + 1) / kGXcd - gx0;
    for (uint32_t i = blockIdx.x / kGXcd; i < n_items_s * ngx; i += nl) {
        const uint32_t c = i / ngx, g = gx0 + i % ngx;
        const uint32_t tb = g << a.lg;
        const int ntg = (int)min((uint32_t)G, (uint32_t)a.ntb - tb);
        const uint32_t kn = min((uint32_t)kGChunk, S - c * kGChunk);
        __syncthreads();   // the previous item's tables and buffer are read
        if (tid < (int)kn) {
            const uint32_t kf = c * kGChunk + (uint32_t)tid;
            int qi = 0;
#pragma unroll
            for (int q = 1; q < kGMaxQ; ++q)
                if (q < nq && pc[q] <= kf) qi = q;
            s.j[tid] = a.spk_ids[(size_t)((q_lo + qi) & (a.H - 1)) * a.N + (kf - pc[qi])];
            s.qoff[tid] = (uint32_t)qi * a.T;
        }
        if (tid < kGTiles) s.tot[tid] = 0;
        __syncthreads();
        // descriptors, all loads issued before their uses (an unused slot
        // reads spike 0's descriptor of the group's first tile)
        {
            constexpr int UD = kGChunk * kGTiles / kGThreads;
            uint64_t d[UD];
#pragma unroll
            for (int u = 0; u < UD; ++u) {
                const int p = tid + kGThreads * u, k = p >> a.lg, tt = p & (G - 1);
                const bool v = k < (int)kn && tt < ntg;
                d[u] = a.seg[a.offb + (uint64_t)s.j[v ? k : 0] * rowlen + tb + (v ? tt : 0)];
            }
#pragma unroll
            for (int u = 0; u < UD; ++u) {
                const int p = tid + kGThreads * u, k = p >> a.lg, tt = p & (G - 1);
                if (k < (int)kn && tt < ntg) {
                    const uint64_t first = d[u] >> 24;
                    const uint32_t len = (uint32_t)(d[u] & 0xFFFFFFu);
                    s.rel[k][tt] = (uint32_t)first;
                    s.dst[k][tt] = len ? atomicAdd(&s.tot[tt], len) : 0u;
                    if (tt == 0) s.e0[k] = first;
                    if (tt == ntg - 1) s.end_lo[k] = (uint32_t)(first + len);
                }
            }
        }
        __syncthreads();
        // wave 0: reserve each tile's share (result kept in a register until
        // the shares are written) and place the shares in the buffer
        const uint32_t my_n = (wave == 0 && lane < ntg) ? s.tot[lane] : 0u;
        unsigned long long my_b = 0;
        if (wave == 0) {
            if (my_n) my_b = atomicAdd(&a.cursor[tb + lane], (unsigned long long)my_n);
            const uint32_t incl = wave_incl_scan(my_n);
            if (lane < kGTiles) s.obase[lane] = incl - my_n;
            if (lane == kGTiles - 1) s.obase[kGTiles] = incl;
        }
        // this wave's spikes k = wave + kGWaves i: prefix of their record counts
        {
            const uint32_t k = (uint32_t)wave + (uint32_t)kGWaves * (uint32_t)lane;
            const uint32_t rl = (lane < kGPer && k < kn) ? s.end_lo[k] - (uint32_t)s.e0[k] : 0u;
            const uint32_t incl = wave_incl_scan(rl);
            if (lane < kGPer) s.wpre[wave][lane] = incl - rl;
            if (lane == kGPer - 1) s.wpre[wave][kGPer] = incl;
        }
        __syncthreads();
        const uint32_t total = s.obase[kGTiles];
        const bool fits = total <= kOutCap;   // the same for the whole workgroup
        if (!fits) {
            if (wave == 0 && lane < ntg) {
                s.base[lane] = my_b;
                s.ok[lane] = my_n > 0 && my_b + my_n <= a.cap;
            }
            __syncthreads();
        }
        const uint32_t* wp = s.wpre[wave];
        const uint32_t wtotal = wp[kGPer];
        constexpr int U = kGU;
        for (uint32_t f0 = (uint32_t)lane; f0 < wtotal; f0 += 64u * U) {
            uint64_t e[U];
            uint32_t qo[U], tls[U], sh[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // past the end: the last record (a valid address, stored
                // again to its own place)
                const uint32_t f = min(f0 + 64u * (uint32_t)u, wtotal - 1);
                // fixed-step searches (no data-dependent branches, so that the
                // records' lookups overlap): the spike, last i with
                // wp[i] <= f ...
                int lo = 0;
#pragma unroll
                for (int step = kGPer / 2; step > 0; step >>= 1)
                    lo += wp[lo + step] <= f ? step : 0;
                const uint32_t k = (uint32_t)wave + (uint32_t)kGWaves * (uint32_t)lo;
                const uint32_t off = f - wp[lo];
                const uint32_t r0 = (uint32_t)s.e0[k];
                // ... and the tile, the last segment starting at or before off
                int tl = 0;
#pragma unroll
                for (int step = kGTiles / 2; step > 0; step >>= 1) {
                    const int cand = tl + step;
                    const uint32_t rv = s.rel[k][cand];   // cand <= kGTiles - 1: read either way, no branch
                    tl = ((cand < ntg) & (rv - r0 <= off)) ? cand : tl;
                }
                ok[u] = f0 + 64u * (uint32_t)u < wtotal;
                e[u] = s.e0[k] + off;
                qo[u] = s.qoff[k];
                tls[u] = (uint32_t)tl;
                sh[u] = s.dst[k][tl] + (off - (s.rel[k][tl] - r0));   // place in the item's share
            }
            Rec r[U];
            if constexpr (WBF16) {
#pragma unroll
                for (int u = 0; u < U; ++u)   // meta + qi T stays below 2^16: no carry into the weight
                    r[u] = static_cast<const uint32_t*>(a.meta)[e[u]] + qo[u];
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    r[u] = make_uint2((uint32_t) static_cast<const META*>(a.meta)[e[u]] + qo[u],
                                      __float_as_uint(a.w[e[u]]));
            }
            if (fits) {
#pragma unroll
                for (int u = 0; u < U; ++u) out[s.obase[tls[u]] + sh[u]] = r[u];
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (ok[u] && s.ok[tls[u]])
                        stage[(size_t)(tb + tls[u]) * a.cap + s.base[tls[u]] + sh[u]] = r[u];
            }
        }
        if (fits) {
            if (wave == 0 && lane < ntg) {
                s.base[lane] = my_b;
                s.ok[lane] = my_n > 0 && my_b + my_n <= a.cap;
            }
            __syncthreads();
            // the shares, each as one contiguous piece of its tile's run
            // written by one wave
            for (int t = wave; t < ntg; t += kGWaves) {
                if (!s.ok[t]) continue;
                const uint32_t n = s.tot[t];
                Rec* to = stage + (size_t)(tb + t) * a.cap + s.base[t];
                const Rec* from = out + s.obase[t];
                for (uint32_t f = (uint32_t)lane; f < n; f += 64u) to[f] = from[f];
            }
        }
    }
}

void (*copy_kernel(const cortex_net* n))(GatherArgs) {
    if (n->w_bytes == 2) return gather_copy_kernel<true, uint16_t>;
    return n->meta_bytes == 2 ? gather_copy_kernel<false, uint16_t> : gather_copy_kernel<false, uint32_t>;
}

}  // namespace

int gather_out_records(int rec_bytes) { return kGOutBytes / rec_bytes; }

// Once per network, before any launch is captured.
void gather_prepare(cortex_net* n) {
    CX_HIP(hipFuncSetAttribute((const void*)copy_kernel(n), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)sizeof(CopyLds)));
}

void launch_gather(cortex_net* n, int parity, int wn, hipStream_t stream) {
    GatherArgs a{};
    a.seg = n->d_seg;
    a.meta = n->d_meta;
    a.w = static_cast<const float*>(n->d_w);
    a.spk_cnt = n->d_spk_cnt;
    a.spk_ids = n->d_spk_ids;
    a.clock = n->d_clock;
    a.cursor = n->d_cursor;
    a.stage = n->d_stage;
    a.offb = n->inst_offbase[0];
    a.N = n->N;
    a.cap = n->stage_cap;
    a.T = (uint32_t)n->T;
    a.parity = parity;
    a.wn = wn;
    a.H = n->H;
    a.dmin = n->dmin;
    a.ntb = n->n_tiles;
    a.lg = __builtin_ctz((unsigned)n->stage_group);
    a.ktime = n->ktiming ? n->d_ktime : nullptr;
    hipLaunchKernelGGL(copy_kernel(n), dim3(kGatherGrid), dim3(kGThreads), sizeof(CopyLds), stream, a);
    CX_HIP(hipGetLastError());
}

}  // namespace cortex
