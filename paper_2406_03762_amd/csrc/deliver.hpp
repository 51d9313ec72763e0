// Delivery of one chunk of spike segments into a workgroup-local input ring.
//
// A chunk is a list of segments in LDS: s_sg[k] = (length, step offset y of
// the spike inside the delivered steps, first synapse as 64 bits) and the
// exclusive prefix s_len[k] of their lengths (s_len[cn] = EL, the chunk's
// synapse count).  Every synapse record r = (delay - d_min) T + target lands
// in ring cell (r + (base_slot + y) T) mod R T, one LDS integer atomic per
// synapse (the ring belongs to this workgroup alone, so no global atomic is
// needed: the tile owns the indegree sub-graph of its targets, Eq. 5, and
// only its spiking part, Eq. 11, is read).
//
// Two mappings of lanes to synapses:
//  - long segments (>= 32 synapses on average): every wave takes a run of
//    whole segments [kw0, kw1) holding about EL / n_waves synapses and reads
//    8 descriptors at once; a descriptor is wave-uniform (scalar registers)
//    and lane l handles synapses l, l + 64, ... of a segment, so its loads
//    are contiguous;
//  - short segments: lanes take consecutive synapses of the flattened chunk;
//    s_blk[b] names the segment holding synapse 64 b of a piece of kBlk
//    blocks, from which a lane walks forward.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace cortex {

constexpr int kDeliverBlk = 512;   // 64-synapse blocks per piece of the short-segment mapping

// Ring cells: 64-bit (long long) or 32-bit (int) signed sums; or, for the
// conductance model (unsigned long long), two 32-bit channels in one cell:
// excitatory weights (>= 0) in the low half, inhibitory ones (< 0, as |w|)
// in the high half.  Each half stays below 2^31 (the fixed-point scale is
// set from the largest sum of |w| a target can receive), so no carry ever
// crosses from one channel into the other.
template <typename RING>
__device__ __forceinline__ void ring_add(RING* ring, uint32_t x, int32_t iw) {
    if (std::is_same<RING, unsigned long long>::value) {
        const unsigned long long v = iw >= 0 ? (unsigned long long)(uint32_t)iw
                                             : (unsigned long long)(uint32_t)(-iw) << 32;
        atomicAdd(reinterpret_cast<unsigned long long*>(&ring[x]), v);
    } else if (sizeof(RING) == 8) {
        atomicAdd(reinterpret_cast<unsigned long long*>(&ring[x]), (unsigned long long)(long long)iw);
    } else {
        atomicAdd(reinterpret_cast<unsigned int*>(&ring[x]), (unsigned int)iw);
    }
}

// Record e: meta (delay - d_min) T + target and the weight.  Two layouts:
// META (16 or 32 bits) and an fp32 weight in separate arrays, or, for bf16
// weights, one packed 32-bit word (weight in the high half, 16-bit record
// below; a bf16 value is the high half of its fp32 value) in `meta`.
template <typename META, bool WBF16>
__device__ __forceinline__ void load_rec(const void* meta, const void* w, uint64_t e, uint32_t& m, float& wv) {
    if (WBF16) {
        const uint32_t r = static_cast<const uint32_t*>(meta)[e];
        m = r & 0xFFFFu;
        wv = __uint_as_float(r & 0xFFFF0000u);
    } else {
        m = static_cast<const META*>(meta)[e];
        wv = static_cast<const float*>(w)[e];
    }
}

// Long segments: wave-owned runs of whole segments [kw0, kw1).
template <typename META, bool WBF16, typename RING>
__device__ __forceinline__ void deliver_long(const uint4* s_sg, RING* ring, int kw0, int kw1, int lane,
                                             const void* meta, const void* w, int base_slot, uint32_t T,
                                             uint32_t RT, float fxw_scale) {
    const int kb = __builtin_amdgcn_readfirstlane(kw0);
    const int ke = __builtin_amdgcn_readfirstlane(kw1);
    for (int k0 = kb; k0 < ke; k0 += 8) {
        constexpr int U8 = 8;
        const unsigned char* mp[U8];
        const unsigned char* wp[U8];
        uint32_t len[U8], roff[U8];
        uint32_t len_max = 0;
        // all eight descriptors are read before any is used (past the run's
        // end the last one is re-read and given length 0)
        uint4 gd[U8];
#pragma unroll
        for (int u = 0; u < U8; ++u) gd[u] = s_sg[min(k0 + u, ke - 1)];
#pragma unroll
        for (int u = 0; u < U8; ++u) {
            const uint4 g = gd[u];
            // readfirstlane yields a signed int: every word goes through
            // uint32_t, or a first synapse at or past 2^31 would be
            // sign-extended into the high half of the 64-bit index
            len[u] = k0 + u < ke ? (uint32_t)__builtin_amdgcn_readfirstlane((int)g.x) : 0u;
            const uint32_t y = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.y);
            const uint32_t e_lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.z);
            const uint32_t e_hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)g.w);
            const uint64_t e0 = ((uint64_t)e_hi << 32) | (uint64_t)e_lo;
            mp[u] = static_cast<const unsigned char*>(meta) + e0 * (WBF16 ? 4 : sizeof(META));
            wp[u] = WBF16 ? nullptr : static_cast<const unsigned char*>(w) + e0 * 4;
            roff[u] = (uint32_t)(base_slot + (int)y) * T;
            len_max = max(len_max, len[u]);
        }
        for (uint32_t o0 = 0; o0 < len_max; o0 += 64u) {
            const uint32_t o = o0 + (uint32_t)lane;
            uint32_t m[U8];
            float wv[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                // m[u] and wv[u] are read below under the same condition
                if (o < len[u]) {
                    if (WBF16) {
                        const uint32_t r = *reinterpret_cast<const uint32_t*>(mp[u] + o * 4u);
                        m[u] = r & 0xFFFFu;
                        wv[u] = __uint_as_float(r & 0xFFFF0000u);
                    } else {
                        m[u] = *reinterpret_cast<const META*>(mp[u] + o * (uint32_t)sizeof(META));
                        wv[u] = *reinterpret_cast<const float*>(wp[u] + o * 4u);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                if (o < len[u]) {
                    uint32_t x = m[u] + roff[u];
                    x = min(x, x - RT);
                    ring_add(ring, x, __float2int_rn(wv[u] * fxw_scale));
                }
            }
        }
    }
}

// Short segments: lanes over the flattened synapses [0, EL) of the chunk.
// Contains workgroup barriers: every thread of the workgroup must call it.
template <typename META, bool WBF16, typename RING>
__device__ __forceinline__ void deliver_short(const uint4* s_sg, const uint32_t* s_len, uint32_t* s_blk,
                                              RING* ring, int cn, uint32_t EL, int tid, int bs, int lane,
                                              int wave, int n_waves, const void* meta, const void* w,
                                              int base_slot, uint32_t T, uint32_t RT, float fxw_scale) {
    for (uint32_t pc0 = 0; pc0 < EL; pc0 += 64u * kDeliverBlk) {
        const uint32_t pc1 = min(EL, pc0 + 64u * kDeliverBlk);
        for (int k = tid; k < cn; k += bs) {
            const uint32_t lo = max(s_len[k], pc0), hi = min(s_len[k + 1], pc1);
            for (uint32_t bb = (lo + 63u) >> 6; (bb << 6) < hi; ++bb) s_blk[bb - (pc0 >> 6)] = (uint32_t)k;
        }
        __syncthreads();
        const uint32_t per = ((pc1 - pc0 + n_waves - 1) / n_waves + 63) & ~63u;
        const uint32_t f_beg = pc0 + min(pc1 - pc0, (uint32_t)wave * per);
        const uint32_t f_end = min(pc1, f_beg + per);
        for (uint32_t f = f_beg + lane; f < f_end; f += 64u * 8u) {
            constexpr int U8 = 8;
            uint32_t m[U8], q[U8];
            float wv[U8];
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                const uint32_t fu = f + 64u * u;
                m[u] = 0;
                wv[u] = 0.f;
                q[u] = 0;
                if (fu < f_end) {
                    int seg = (int)s_blk[((fu - (uint32_t)lane) - pc0) >> 6];
                    while (s_len[seg + 1] <= fu) ++seg;
                    const uint4 g = s_sg[seg];
                    const uint64_t e = (((uint64_t)g.w << 32) | g.z) + (fu - s_len[seg]);
                    q[u] = g.y | 8u;
                    load_rec<META, WBF16>(meta, w, e, m[u], wv[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < U8; ++u) {
                if (q[u] & 8u) {
                    uint32_t x = m[u] + (uint32_t)(base_slot + (int)(q[u] & 7u)) * T;
                    x = min(x, x - RT);
                    ring_add(ring, x, __float2int_rn(wv[u] * fxw_scale));
                }
            }
        }
        __syncthreads();   // s_blk is refilled for the next piece
    }
}

// s_kw[w] = first segment k with s_len[k] >= min(EL, w * share) for the
// waves w = 0..n_waves: segment k owns the share boundaries in
// (s_len[k - 1], s_len[k]].  Also sets s_len[cn] = EL.  Every thread calls
// it; a barrier must follow before s_kw is read.
__device__ __forceinline__ void wave_runs(uint32_t* s_len, int* s_kw, int cn, uint32_t EL, int n_waves, int tid,
                                          int bs) {
    const uint32_t share = (EL + n_waves - 1) / n_waves;
    for (int k = tid; k <= cn; k += bs) {
        const int64_t lo = k == 0 ? -1 : (int64_t)s_len[k - 1];
        const uint32_t hi = k < cn ? s_len[k] : EL;
        for (int w = 0; w <= n_waves; ++w) {
            const uint32_t tw = min(EL, (uint32_t)w * share);
            if ((int64_t)tw > lo && tw <= hi) s_kw[w] = k;
        }
    }
    if (tid == 0) s_len[cn] = EL;
}

}  // namespace cortex
