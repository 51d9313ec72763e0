// Spike-timing dependent plasticity of the E->E synapses (the plastic
// synapses of the paper's verification network, Sec. IV-A), for the
// streamed plan: one launch per window, right before the window's delivery
// launch.  The rule (power-law potentiation, multiplicative depression,
// all-to-all pairing, every delay dendritic) is stated with the spec fields
// in cortex.h.
//
// One workgroup per tile, as in delivery: the tile owns its targets'
// in-synapses (Eq. 5), so every weight it rewrites has this workgroup as its
// only writer, and the same holds for the per-(source, tile) presynaptic
// trace and the tile's targets' spike histories -- no atomics, no locks
// (the race-freedom the paper checks on this network).  A launch
//  1. appends the spikes its targets emitted since the previous launch
//     (read from the per-step spike lists the delivery launches publish) to
//     their histories: step and postsynaptic trace just after the spike;
//  2. for every spike the coming delivery launch delivers (steps
//     [t0 - d_min, t0 - d_min + wn), at most one per source since the
//     window is at most n_ref + 1 steps), one wave walks the source's
//     segment into the tile and updates each plastic synapse from the
//     segment's presynaptic trace and the target's history, then records
//     the new presynaptic trace.
// Every spike a synapse needs is in the past at this point: a spike at q is
// delivered no earlier than t0 - d_min, and the update reads postsynaptic
// spikes up to step q - d <= t0 - 1.
#include <cmath>

#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

struct StdpArgs {
    const int32_t* tile_inst;
    const int32_t* tile_size;
    const int32_t* inst_tile0;
    const int32_t* inst_ntiles;
    const int32_t* inst_T;
    const int64_t* inst_n0;
    const uint64_t* inst_offbase;
    const uint64_t* seg;           // (first synapse << 24) | length per (source, tile)
    const void* meta;              // (delay - d_min) T + target
    int meta16;
    float* w;                      // fp32 weights, rewritten in place
    const uint32_t* spk_cnt;       // [H][n_inst]
    const uint32_t* spk_ids;       // [H][N]
    const int64_t* clock;          // [2] window starts
    uint64_t* seg_state;           // per (source, tile): x bits | (q + 1) << 32
    int32_t* hist_step;            // [N][kHistLen]
    float* hist_y;                 // [N][kHistLen]
    uint32_t* hist_cnt;            // [N]
    int64_t* hist_upto;            // [n_tiles]
    int32_t* err;                  // [4]; err[1] set when a needed spike left a history
    int64_t N, plo, phi;           // plastic population [plo, phi), global ids
    int parity, wn, H, n_inst, T, dmin;
    float c_pot, lam_alpha, mu, dt_tp, dt_tm, wmax;   // lambda w0^(1-mu), lambda alpha, mu, dt/tau+, dt/tau-
};

__global__ void __launch_bounds__(512) stdp_kernel(StdpArgs a) {
    const int tile = blockIdx.x;
    const int b = a.tile_inst[tile];
    const int tl = tile - a.inst_tile0[b];
    const int ntb = a.inst_ntiles[b];
    const int tsz = a.tile_size[tile];
    const int64_t n0b = a.inst_n0[b];
    const int64_t g0 = n0b + (int64_t)tl * a.inst_T[b];
    const uint64_t offb = a.inst_offbase[b];
    const int tid = threadIdx.x, bs = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, n_waves = bs >> 6;
    const int64_t t0 = a.clock[a.parity];
    const int H = a.H;
    // 1. the tile's plastic targets that spiked in [hist_upto, t0)
    const int64_t lo_t = max(g0, a.plo), hi_t = min(g0 + tsz, a.phi);
    for (int64_t s = a.hist_upto[tile]; s < t0; ++s) {
        const size_t slot = (size_t)(s & (H - 1));
        const uint32_t cnt = a.spk_cnt[slot * a.n_inst + b];
        const uint32_t* ids = a.spk_ids + slot * a.N + n0b;
        for (uint32_t k = tid; k < cnt; k += bs) {
            const int64_t i = ids[k];
            if (i < lo_t || i >= hi_t) continue;
            // a neuron spikes at most once per step: one thread per neuron here
            const uint32_t c = a.hist_cnt[i];
            float y = 1.f;
            if (c > 0) {
                const uint32_t k0 = (c - 1) % kHistLen;
                y += a.hist_y[i * kHistLen + k0] * expf(-(float)(s - a.hist_step[i * kHistLen + k0]) * a.dt_tm);
            }
            a.hist_step[i * kHistLen + c % kHistLen] = (int32_t)s;
            a.hist_y[i * kHistLen + c % kHistLen] = y;
            a.hist_cnt[i] = c + 1;
        }
        __syncthreads();   // the next step's appends read what this step wrote
    }
    __syncthreads();
    if (tid == 0) a.hist_upto[tile] = t0;
    // 2. the plastic synapses of the spikes delivered next, one wave per spike
    const uint32_t T = (uint32_t)a.T;
    const int64_t q_lo = max((int64_t)0, t0 - a.dmin), q_hi = t0 - a.dmin + a.wn;
    for (int64_t q = q_lo; q < q_hi; ++q) {
        const size_t slot = (size_t)(q & (H - 1));
        const uint32_t cnt = a.spk_cnt[slot * a.n_inst + b];
        const uint32_t* ids = a.spk_ids + slot * a.N + n0b;
        for (uint32_t k = wave; k < cnt; k += n_waves) {
            const int64_t j = ids[k];
            if (j < a.plo || j >= a.phi) continue;   // a static source (wave-uniform)
            const uint64_t si = offb + (uint64_t)(j - n0b) * (uint64_t)(ntb + 1) + (uint64_t)tl;
            const uint64_t d = a.seg[si];
            const uint64_t e0 = d >> 24, e1 = e0 + (d & 0xFFFFFFu);
            if (e1 == e0) continue;
            const uint64_t st = a.seg_state[si];
            const float x_last = __uint_as_float((uint32_t)st);
            const int64_t q_last = (int64_t)(st >> 32) - 1;   // -1: no earlier spike
            for (uint64_t e = e0 + lane; e < e1; e += 64) {
                const uint32_t m = a.meta16 ? static_cast<const uint16_t*>(a.meta)[e]
                                            : static_cast<const uint32_t*>(a.meta)[e];
                const int64_t i = g0 + (int64_t)(m % T);
                if (i < a.plo || i >= a.phi) continue;   // a static synapse
                const int64_t dd = a.dmin + (int64_t)(m / T);
                const uint32_t c = a.hist_cnt[i];
                const uint32_t kept = min(c, (uint32_t)kHistLen);
                const int32_t* hs = a.hist_step + i * kHistLen;
                const float* hy = a.hist_y + i * kHistLen;
                float w = a.w[e];
                // potentiation: spikes p of i with q_last < p + d <= q, oldest first
                if (q_last >= 0 && kept > 0) {
                    uint32_t first = kept;   // index (0 = oldest kept) of the first such spike
                    for (uint32_t r = 0; r < kept; ++r) {
                        const uint32_t kk = (c - kept + r) % kHistLen;
                        if ((int64_t)hs[kk] + dd > q_last) { first = r; break; }
                    }
                    // a spike older than the kept ones may be missing
                    if (c > (uint32_t)kHistLen && first == 0) atomicOr(&a.err[1], 1);
                    for (uint32_t r = first; r < kept; ++r) {
                        const uint32_t kk = (c - kept + r) % kHistLen;
                        const int64_t arr = (int64_t)hs[kk] + dd;
                        if (arr > q) break;
                        const float x = x_last * expf(-(float)(arr - q_last) * a.dt_tp);
                        w = fminf(a.wmax, w + a.c_pot * powf(w, a.mu) * x);
                    }
                }
                // depression: y_i at q - d from the latest spike before it
                float y = 0.f;
                bool found = false;
                for (uint32_t r = kept; r-- > 0;) {
                    const uint32_t kk = (c - kept + r) % kHistLen;
                    if ((int64_t)hs[kk] < q - dd) {
                        y = hy[kk] * expf(-(float)(q - dd - hs[kk]) * a.dt_tm);
                        found = true;
                        break;
                    }
                }
                if (!found && c > (uint32_t)kHistLen) atomicOr(&a.err[1], 1);
                w = fmaxf(0.f, w - a.lam_alpha * w * y);
                a.w[e] = w;
            }
            if (lane == 0) {
                const float x = 1.f + (q_last >= 0 ? x_last * expf(-(float)(q - q_last) * a.dt_tp) : 0.f);
                a.seg_state[si] = (uint64_t)__float_as_uint(x) | ((uint64_t)(q + 1) << 32);
            }
        }
    }
}

}  // namespace

void launch_stdp(cortex_net* n, int parity, int wn, hipStream_t stream) {
    StdpArgs a{};
    a.tile_inst = n->d_tile_inst;
    a.tile_size = n->d_tile_size;
    a.inst_tile0 = n->d_inst_tile0;
    a.inst_ntiles = n->d_inst_ntiles;
    a.inst_T = n->d_inst_T;
    a.inst_n0 = n->d_inst_n0;
    a.inst_offbase = n->d_inst_offbase;
    a.seg = n->d_seg;
    a.meta = n->d_meta;
    a.meta16 = n->meta_bytes == 2;
    a.w = static_cast<float*>(n->d_w);
    a.spk_cnt = n->d_spk_cnt;
    a.spk_ids = n->d_spk_ids;
    a.clock = n->d_clock;
    a.seg_state = n->d_seg_state;
    a.hist_step = n->d_hist_step;
    a.hist_y = n->d_hist_y;
    a.hist_cnt = n->d_hist_cnt;
    a.hist_upto = n->d_hist_upto;
    a.err = n->d_err;
    a.N = n->N;
    a.plo = n->stdp_lo;
    a.phi = n->stdp_hi;
    a.parity = parity;
    a.wn = wn;
    a.H = n->H;
    a.n_inst = n->n_inst;
    a.T = n->T;
    a.dmin = n->dmin;
    a.c_pot = (float)n->stdp_c;
    a.lam_alpha = (float)n->stdp_lam_alpha;
    a.mu = (float)n->stdp_mu;
    a.dt_tp = (float)(n->spec.dt / n->stdp_tp);
    a.dt_tm = (float)(n->spec.dt / n->stdp_tm);
    a.wmax = (float)n->stdp_wmax;
    hipLaunchKernelGGL(stdp_kernel, dim3(n->n_tiles), dim3(512), 0, stream, a);
    CX_HIP(hipGetLastError());
}

}  // namespace cortex
