// Device helpers: counter-based random numbers and workgroup scans.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cortex {

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Every random quantity
// of a network is a pure function of (counter, key): key = (seed, instance),
// counter = (c0, c1, c2, stream tag).  Ten rounds; each multiplies words 0
// and 2 by the two Philox constants, mixes the high halves with words 1 and
// 3 and the round key, and advances the key by the Weyl constants.
struct Philox4 {
    uint64_t v[4];
};

__device__ __forceinline__ Philox4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                          uint64_t k0, uint64_t k1) {
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a_hi = __umul64hi(kMulA, c0), a_lo = kMulA * c0;
        const uint64_t b_hi = __umul64hi(kMulB, c2), b_lo = kMulB * c2;
        c0 = b_hi ^ c1 ^ k0;
        c1 = b_lo;
        c2 = a_hi ^ c3 ^ k1;
        c3 = a_lo;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    Philox4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Word i (0..3) of a Philox block, chosen by selects: an array indexed by a
// run-time value would be kept in scratch memory.
__device__ __forceinline__ uint64_t philox_word(const Philox4& p, uint32_t i) {
    const uint64_t lo = (i & 1u) ? p.v[1] : p.v[0];
    const uint64_t hi = (i & 1u) ? p.v[3] : p.v[2];
    return (i & 2u) ? hi : lo;
}

// Stream tags of the counter's last word.
enum : uint64_t { kTagEdge = 1, kTagPoisson = 2, kTagV0 = 3, kTagPair = 5 };

// Integer uniform on [0, n): high word of u * n.
__device__ __forceinline__ uint64_t uniform_below(uint64_t u, uint64_t n) { return __umul64hi(u, n); }
// Double in [0, 1) from the top 53 bits; (0, 1] variant for logarithms.
__device__ __forceinline__ double unit_closed0(uint64_t u) { return (double)(u >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double unit_open0(uint64_t u) { return (double)((u >> 11) + 1) * 0x1.0p-53; }

// Wave (64 lanes) inclusive scan of 32-bit values with DPP lane moves:
// shifts by 1, 2, 4, 8 inside each row of 16 lanes (lanes shifted in from
// outside the row read 0), then the last lane of row 0 is added to row 1 and
// that of row 2 to row 3 (row_bcast:15), then the last lane of row 1 to rows
// 2 and 3 (row_bcast:31).  Lanes a row mask leaves out keep `old` = 0.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Exclusive scan of data[0..n) in LDS, in place, by the whole workgroup.
// `wsum` is LDS scratch of at least (blockDim.x / 64 + 1) words.  Returns
// the total.  Must be called by every thread of the workgroup.
__device__ inline uint32_t block_excl_scan(uint32_t* data, int n, uint32_t* wsum) {
    const int tid = threadIdx.x, bs = blockDim.x;
    const int per = (n + bs - 1) / bs;
    const int beg = min(n, tid * per), end = min(n, beg + per);
    uint32_t local = 0;
    for (int i = beg; i < end; ++i) local += data[i];
    const uint32_t inc = wave_incl_scan(local);
    const int wave = tid >> 6, lane = tid & 63;
    const int nw = (bs + 63) >> 6;
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        // exclusive offsets of the waves (nw <= 16), and the total
        const uint32_t v = lane < nw ? wsum[lane] : 0u;
        const uint32_t vi = wave_incl_scan(v);
        if (lane < nw) wsum[lane] = vi - v;
        if (lane == nw - 1) wsum[nw] = vi;
    }
    __syncthreads();
    uint32_t run = wsum[wave] + inc - local;
    for (int i = beg; i < end; ++i) { uint32_t t = data[i]; data[i] = run; run += t; }
    const uint32_t total = wsum[nw];
    __syncthreads();
    return total;
}

// Index of the last entry of the ascending prefix array pfx[0..n) that is
// <= x (pfx[0] == 0 <= x).
__device__ __forceinline__ int seg_of(const uint32_t* pfx, int n, uint32_t x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pfx[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

}  // namespace cortex
