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
    uint32_t j[kGChunk];
    uint32_t qoff[kGChunk];               // ring row of its step, relative to the window's first: qi T
    uint32_t tot[kGTiles];                // the item's records per tile
    uint32_t obase[kGTiles + 1];          // their first place in `out`; obase[kGTiles]: the item's total
    unsigned long long base[kGTiles];     // their place in the tile's run
    uint32_t ok[kGTiles];
};

// One work item per (64 consecutive spikes of the window, group of G = 2^lg
// tiles).  Each thread takes the item's segments (spike, tile) at tid and
// tid + kGThreads and keeps their descriptors in registers; a
// workgroup-local atomic per segment gives its place in the item's share of
// the tile's run, and one global atomic per tile reserves that share (its
// result is needed only when the shares are written, so the atomics'
// latency overlaps the gathering).  The thread then copies its segments'
// records, a few 16-byte loads per segment, into the item's buffer (no
// per-record search: a record's place is its segment's place plus its
// index); the workgroup then writes the buffer out share by share.  An item
// whose records overflow the buffer writes them straight to the runs
// instead.
//
// The tile groups are split into kGXcd contiguous ranges, one per XCD, and
// an XCD's workgroups take its items spike chunk by spike chunk: the items
// of adjacent groups, which share the cache lines at the ends of each
// spike's row piece and of its descriptors, run at about the same time in
// the same L2, and so do the items that fill adjacent shares of one run.
template <bool WBF16, typename META>
__global__ void __launch_bounds__(kGThreads) __attribute__((amdgpu_waves_per_eu(8))) gather_copy_kernel(GatherArgs a) {
    using Rec = typename std::conditional<WBF16, uint32_t, uint2>::type;
    // a lane loads PR consecutive records of a segment at once: 16 bytes of
    // packed records, or one record and its separate weight
    using Piece = typename std::conditional<WBF16, uint4, uint2>::type;
    constexpr uint32_t PR = WBF16 ? 4u : 1u;
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
            // (the step and its first spike selected in the unrolled loop:
            // no runtime index into pc, which would put it in scratch)
            int qi = 0;
            uint32_t k0 = 0;
#pragma unroll
            for (int q = 1; q < kGMaxQ; ++q)
                if (q < nq && pc[q] <= kf) {
                    qi = q;
                    k0 = pc[q];
                }
            s.j[tid] = a.spk_ids[(size_t)((q_lo + qi) & (a.H - 1)) * a.N + (kf - k0)];
            s.qoff[tid] = (uint32_t)qi * a.T;
        }
        if (tid < kGTiles) s.tot[tid] = 0;
        __syncthreads();
        // descriptors: thread tid takes the segments (spike k, tile tt) of
        // p = tid + kGThreads h, h < UD, and keeps each segment's first
        // record, length, ring-row offset and place in the item's share of
        // its tile (a workgroup-local atomic) in registers; the loads are all
        // issued before their uses (an unused slot reads spike 0's
        // descriptor of the group's first tile and has length 0)
        constexpr int UD = kGChunk * kGTiles / kGThreads;
        uint64_t sf[UD];
        uint32_t sl[UD], sd[UD], sq[UD];
        int st[UD];
        {
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
                const bool v = k < (int)kn && tt < ntg;
                sf[u] = d[u] >> 24;
                sl[u] = v ? (uint32_t)(d[u] & 0xFFFFFFu) : 0u;
                st[u] = v ? tt : 0;
                sq[u] = v ? s.qoff[k] : 0u;
                sd[u] = sl[u] ? atomicAdd(&s.tot[tt], sl[u]) : 0u;
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
        // every thread copies its segments, PR x UR records of each at a
        // time: a lane's loads read its segments' own records (a segment of
        // a few records is one or two 16-byte loads); a load at or past a
        // segment's end is clamped to its last records (at most PR - 1
        // records past the segment, inside the record array and its 16 bytes
        // of slack), and only the segment's records are stored
        uint32_t dst0[UD];
        bool wr[UD];
        uint32_t mx = 0;
#pragma unroll
        for (int u = 0; u < UD; ++u) {
            mx = max(mx, sl[u]);
            dst0[u] = fits ? s.obase[st[u]] + sd[u] : s.base[st[u]] + sd[u];
            wr[u] = fits || s.ok[st[u]];
        }
        constexpr int UR = WBF16 ? 2 : 4;
        for (uint32_t i0 = 0; i0 < mx; i0 += PR * UR) {
            Piece v[UD][UR];
#pragma unroll
            for (int u = 0; u < UD; ++u)
#pragma unroll
                for (int r = 0; r < UR; ++r) {
                    const uint64_t e = sf[u] + min(i0 + (uint32_t)r * PR, max(sl[u], 1u) - 1u);
                    if constexpr (WBF16) {
                        __builtin_memcpy(&v[u][r], static_cast<const uint32_t*>(a.meta) + e, sizeof(Piece));
                    } else {
                        v[u][r] = make_uint2((uint32_t) static_cast<const META*>(a.meta)[e], __float_as_uint(a.w[e]));
                    }
                }
#pragma unroll
            for (int u = 0; u < UD; ++u)
#pragma unroll
                for (int r = 0; r < UR; ++r)
#pragma unroll
                    for (int c = 0; c < (int)PR; ++c) {
                        const uint32_t i = i0 + (uint32_t)r * PR + (uint32_t)c;
                        if (!wr[u] || i >= sl[u]) continue;
                        Rec rec;
                        if constexpr (WBF16) {
                            // meta + qi T stays below 2^16: no carry into the weight
                            const uint32_t w4 = c == 0 ? v[u][r].x : c == 1 ? v[u][r].y : c == 2 ? v[u][r].z : v[u][r].w;
                            rec = w4 + sq[u];
                        } else {
                            rec = make_uint2(v[u][r].x + sq[u], v[u][r].y);
                        }
                        if (fits) out[dst0[u] + i] = rec;
                        else stage[(size_t)(tb + st[u]) * a.cap + dst0[u] + i] = rec;
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
