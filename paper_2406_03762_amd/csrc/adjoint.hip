// Adjoint of the membrane-voltage loss with respect to every synaptic weight,
// spikes frozen to the forward raster.
//
// With the raster fixed, each neuron's state is an affine function of the
// inputs it consumed, and the input consumed by target i at step n is
// x_i(n) = sum_e w_e s_src(e)(n - d_e) (the delivery of Sec. II-B), so the
// loss L = sum_b 1/(N_b T) sum_{i,n} (V_i(n) - V*_i(n))^2 is quadratic in the
// weights and dL/dw_e = sum_{m : src(e) spiked at m} g_tgt(e)(m + d_e), with
// g_i(n) = dL/dx_i(n) from a backward recursion through the exact
// propagators.  The forward stores the raster and, every C steps, the neuron
// state and the input rings.  The backward
//  1. puts the raster on the device once, indexed per (step, tile) for the
//     replays and regrouped by source (each source's spike steps, ascending)
//     for the gradient;
//  2. walks the segments last to first: restores the segment's checkpoint
//     and re-runs it on the frozen raster with the step kernel (integer input
//     sums make this a bit-exact replay), which yields V(n) and the mask
//     m(n) = "integrated and did not spike"; then one thread per neuron runs
//     the reverse recursion and writes g for the segment's steps into the
//     neuron's row of g over the whole window;
//  3. computes every weight's gradient in canonical order (the in-synapses
//     of each target, Eq. 5's indegree sub-graph read target by target): one
//     wave per target, a lane per synapse sums g of the target at the
//     arrivals of its source's spikes; each gradient is written once, in
//     order, with no atomics.
#include <algorithm>
#include <cstring>
#include <vector>

#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

// Write step records and spike ids of steps [q0, q1) (from the raster) into
// the publication buffer, as the forward kernel had published them.
__global__ void republish_kernel(uint64_t* pub, int H, int n_tiles, int T, int64_t q0, int nq,
                                 const uint32_t* ids, const uint64_t* ptr, uint64_t n_ids) {
    const int64_t pairs = (int64_t)nq * n_tiles;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pairs;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t qi = p / n_tiles;
        const int tile = (int)(p - qi * n_tiles);
        const int64_t q = q0 + qi;
        const uint64_t tag = (uint64_t)(uint32_t)(q + 1) << 32;
        uint64_t* base = pub + (size_t)(q & (H - 1)) * n_tiles * (T + 1) + (size_t)tile * (T + 1);
        const uint64_t b1 = min(ptr[p + 1], n_ids), b0 = min(ptr[p], b1);
        if (b1 - b0 > (uint64_t)T) continue;   // a tile publishes at most T ids
        for (uint64_t k = b0; k < b1; ++k)
            __hip_atomic_store(base + 1 + (k - b0), tag | ids[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(base, tag | (uint32_t)(b1 - b0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

struct ReverseArgs {
    const float* vtr;      // [len][N] V after each step of the segment
    const uint8_t* mtr;    // [len][N]
    const float* vstar;    // [T][N]
    float* gT;             // [N][T] dL/dx, one row per neuron over the whole window
    double* aU;            // carried adjoint state at step s1
    double* a1;
    double* a2;
    uint8_t* m_next;
    double* loss_part;     // [gridDim.x] per-block partial sums of the loss
    const int64_t* inst_n0;
    const int64_t* inst_N;
    int n_inst;
    int64_t N, s0, len, T;
    int model;
    double P22, P11, P21, P31, P32, P21s, P22s, jump;
};

// Per neuron, with m_n = 1 iff step n integrated and did not spike and
// l_n = dL/dV_n:  aU_n = l_n + m_{n+1} P22 aU_{n+1};
// exp:   aI_n = m_{n+1} P21 aU_{n+1} + P11 aI_{n+1},             g_n = aI_n;
// alpha: a2_n = m_{n+1} P32 aU_{n+1} + P22s a2_{n+1},
//        a1_n = m_{n+1} P31 aU_{n+1} + P21s a2_{n+1} + P11 a1_{n+1}, g_n = jump a1_n;
// delta: g_n = m_n aU_n.
// A workgroup takes 256 consecutive neurons; the steps are walked backwards
// in chunks of up to 16 (aligned to multiples of 16), whose g values go
// through LDS so that each neuron's row of g is written as whole lines.
constexpr int kRevChunk = 16;

__global__ void __launch_bounds__(256) reverse_kernel(ReverseArgs a) {
    __shared__ float s_g[kRevChunk][257];
    double lsum = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < a.N; base += (int64_t)gridDim.x * 256) {
        const int64_t i = base + threadIdx.x;
        const bool ok = i < a.N;
        double scale = 0.0, aU = 0.0, a1 = 0.0, a2 = 0.0;
        int mn = 0;
        if (ok) {
            int lo = 0, hi = a.n_inst;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.inst_n0[mid] <= i) lo = mid; else hi = mid;
            }
            scale = 1.0 / ((double)a.inst_N[lo] * (double)a.T);
            aU = a.aU[i];
            a1 = a.a1[i];
            a2 = a.a2[i];
            mn = a.m_next[i];
        }
        for (int64_t n_hi = a.s0 + a.len; n_hi > a.s0;) {
            const int64_t n_lo = max(a.s0, ((n_hi - 1) / kRevChunk) * kRevChunk);
            for (int64_t n = n_hi - 1; n >= n_lo; --n) {
                float gv = 0.f;
                if (ok) {
                    const int64_t k = n - a.s0;
                    const double diff = (double)a.vtr[k * a.N + i] - (double)a.vstar[n * a.N + i];
                    lsum += scale * diff * diff;
                    const double l = 2.0 * scale * diff;
                    const double naU = l + (mn ? a.P22 * aU : 0.0);
                    double na1 = 0.0, na2 = 0.0;
                    if (a.model == CORTEX_MODEL_EXP) {
                        na1 = (mn ? a.P21 * aU : 0.0) + a.P11 * a1;
                    } else if (a.model == CORTEX_MODEL_ALPHA) {
                        na2 = (mn ? a.P32 * aU : 0.0) + a.P22s * a2;
                        na1 = (mn ? a.P31 * aU : 0.0) + a.P21s * a2 + a.P11 * a1;
                    }
                    aU = naU;
                    a1 = na1;
                    a2 = na2;
                    mn = a.mtr[k * a.N + i];
                    double g;
                    if (a.model == CORTEX_MODEL_DELTA) g = mn ? aU : 0.0;
                    else if (a.model == CORTEX_MODEL_EXP) g = a1;
                    else g = a.jump * a1;
                    gv = (float)g;
                }
                s_g[n - n_lo][threadIdx.x] = gv;
            }
            __syncthreads();
            const int w = (int)(n_hi - n_lo);
            for (int idx = threadIdx.x; idx < 256 * kRevChunk; idx += 256) {
                const int r = idx / kRevChunk, c = idx % kRevChunk;
                if (c < w && base + r < a.N) a.gT[(base + r) * a.T + n_lo + c] = s_g[c][r];
            }
            __syncthreads();
            n_hi = n_lo;
        }
        if (ok) {
            a.aU[i] = aU;
            a.a1[i] = a1;
            a.a2[i] = a2;
            a.m_next[i] = (uint8_t)mn;
        }
    }
    // block reduction of the loss into this block's slot; the slots are
    // summed in a fixed order afterwards, so the loss is reproducible
    __shared__ double red[256];
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.loss_part[blockIdx.x] = red[0];
}

// loss += sum of the per-block partials, in block order (one workgroup).
__global__ void __launch_bounds__(256) loss_sum_kernel(const double* part, int n_part, double* loss) {
    __shared__ double red[256];
    double s = 0.0;
    const int per = (n_part + 255) / 256;
    const int b0 = min(n_part, (int)threadIdx.x * per), b1 = min(n_part, b0 + per);
    for (int b = b0; b < b1; ++b) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss += red[0];
}

// Spikes of the raster regrouped by source: cnt[j] = spikes of j; after a
// scan into sptr, steps of j's spikes in sstep[sptr[j] .. sptr[j + 1]),
// ascending.
__global__ void src_count_kernel(const uint32_t* r_ids, int64_t n_spk, uint32_t* cnt) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_spk; q += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[r_ids[q]], 1u);
}

__global__ void src_fill_kernel(const uint32_t* r_steps, const uint32_t* r_ids, int64_t n_spk, const uint64_t* sptr,
                                uint32_t* cur, int32_t* sstep) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n_spk; q += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t j = r_ids[q];
        sstep[sptr[j] + atomicAdd(&cur[j], 1u)] = (int32_t)r_steps[q];
    }
}

// The fill's order is that of its atomics: sort each source's few steps.
__global__ void src_sort_kernel(const uint64_t* sptr, int32_t* sstep, int64_t N) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t b = sptr[j], e = sptr[j + 1];
        for (uint64_t k = b + 1; k < e; ++k) {
            const int32_t v = sstep[k];
            uint64_t m = k;
            while (m > b && sstep[m - 1] > v) {
                sstep[m] = sstep[m - 1];
                --m;
            }
            sstep[m] = v;
        }
    }
}

// Each source's spikes in one 16-byte word when the window is shorter than
// 65536 steps: eight 16-bit fields, the spike count (saturated) and its
// first seven steps; further spikes stay in the sorted list.
__global__ void src_pack_kernel(const uint64_t* sptr, const int32_t* sstep, int64_t N, uint4* s8) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t b = sptr[j], n = sptr[j + 1] - b;
        uint32_t f[8] = {(uint32_t)min<uint64_t>(n, 0xFFFF), 0, 0, 0, 0, 0, 0, 0};
        for (uint64_t k = 0; k < min<uint64_t>(n, 7); ++k) f[1 + k] = (uint32_t)sstep[b + k];
        s8[j] = make_uint4(f[0] | (f[1] << 16), f[2] | (f[3] << 16), f[4] | (f[5] << 16), f[6] | (f[7] << 16));
    }
}

// dL/dw_c = sum over the spikes q of src_c with q + d_c < T of
// g_tgt(q + d_c), for every synapse c in canonical order (target, then
// projection and slot): one wave per target, a lane per synapse, four
// synapses per lane at a time (independent loads in flight).  The target's
// row of g (T values) is read from cache by every lane; each gradient is
// written once, in order, straight into the caller's buffer.
__global__ void __launch_bounds__(256) pull_grad_kernel(const uint64_t* cin, const uint32_t* csrc,
                                                        const uint16_t* cdel, const uint4* s8,
                                                        const uint64_t* sptr, const int32_t* sstep,
                                                        const float* gT, int64_t N, int64_t T, float* grad) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    constexpr int U = 8;   // synapses per lane in flight (4: backward 4 % slower on the 64-instance batch)
    for (int64_t i = wave; i < N; i += n_waves) {
        const float* g = gT + i * T;
        const uint64_t c1 = cin[i + 1];
        for (uint64_t cb = cin[i] + lane; cb < c1; cb += 64 * U) {
            uint32_t j[U];
            int64_t d[U];
            uint4 sp[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t c = cb + 64u * u;
                j[u] = c < c1 ? csrc[c] : 0u;
                d[u] = c < c1 ? (int64_t)cdel[c] : T;   // past the window: contributes nothing
            }
#pragma unroll
            for (int u = 0; u < U; ++u) sp[u] = s8[j[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t c = cb + 64u * u;
                if (c >= c1) continue;
                const uint32_t f[8] = {sp[u].x & 0xFFFFu, sp[u].x >> 16, sp[u].y & 0xFFFFu, sp[u].y >> 16,
                                       sp[u].z & 0xFFFFu, sp[u].z >> 16, sp[u].w & 0xFFFFu, sp[u].w >> 16};
                const uint32_t cnt = f[0];
                float acc = 0.f;
                bool more = true;
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    if ((uint32_t)k < cnt && more) {
                        const int64_t arr = (int64_t)f[1 + k] + d[u];
                        if (arr < T) acc += g[arr];
                        else more = false;   // ascending steps
                    }
                }
                if (cnt > 7 && more) {   // spikes past the seventh (or a saturated count)
                    const uint64_t p1 = sptr[j[u] + 1];
                    for (uint64_t p = sptr[j[u]] + 7; p < p1; ++p) {
                        const int64_t arr = (int64_t)sstep[p] + d[u];
                        if (arr >= T) break;
                        acc += g[arr];
                    }
                }
                grad[c] = acc;
            }
        }
    }
}

// The raster of steps [0, T) from the spike log, sorted by (step, id), on
// the device.  The log holds, per tile, its spikes step after step, and
// cnt[s][t] per (step, tile) (0xFFFFFFFF: the tile's log overflowed).
// 1. per tile, the offset of each step's spikes inside its log (a scan
//    along the steps, one wave per tile); flag overflow marks;
__global__ void log_offsets_kernel(const uint32_t* cnt, int64_t T, int n_tiles, uint64_t* tile_off, int32_t* bad) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= n_tiles) return;
    const int t = (int)wave;
    uint64_t carry = 0;
    for (int64_t s0 = 0; s0 < T; s0 += 64) {
        const int64_t s = s0 + lane;
        uint32_t c = s < T ? cnt[s * n_tiles + t] : 0u;
        if (c == 0xFFFFFFFFu) {
            atomicOr(bad, 1);
            c = 0;
        }
        const uint32_t inc = wave_incl_scan(c);
        if (s < T) tile_off[s * n_tiles + t] = carry + inc - c;
        carry += (uint32_t)__shfl((int)inc, 63, 64);
    }
}

// 2. (after a scan of cnt in step-major order into gpos) one thread per
//    (step, tile) copies its spikes to their place and sorts them by id;
//    flag ids out of range.
__global__ void log_copy_kernel(const uint32_t* cnt, const uint64_t* tile_off, const uint64_t* gpos,
                                const uint64_t* log_base, const uint32_t* log_ids, int64_t T, int n_tiles,
                                int64_t N, uint32_t* r_steps, uint32_t* r_ids, int32_t* bad) {
    const int64_t pairs = T * n_tiles;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pairs; p += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = cnt[p];
        if (c == 0xFFFFFFFFu || c == 0) continue;
        const int t = (int)(p % n_tiles);
        const uint32_t s = (uint32_t)(p / n_tiles);
        const uint32_t* src = log_ids + log_base[t] + tile_off[p];
        const uint64_t o = gpos[p];
        for (uint32_t k = 0; k < c; ++k) {
            uint32_t v = src[k];
            if (v >= (uint64_t)N) {
                atomicOr(bad, 2);
                v = 0;
            }
            uint32_t m = k;   // insertion into the sorted prefix
            while (m > 0 && r_ids[o + m - 1] > v) {
                r_ids[o + m] = r_ids[o + m - 1];
                --m;
            }
            r_ids[o + m] = v;
            r_steps[o + k] = s;
        }
    }
}

// The counts of overflowed pairs enter the step-major scan as 0.
__global__ void log_clean_counts_kernel(const uint32_t* cnt, int64_t pairs, uint32_t* clean) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < pairs; p += (int64_t)gridDim.x * blockDim.x)
        clean[p] = cnt[p] == 0xFFFFFFFFu ? 0u : cnt[p];
}

int grid_of(int64_t work, int bs) {
    int64_t g = (work + bs - 1) / bs;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

}  // namespace

void republish(cortex_net* n, int64_t q0, int64_t q1, const uint32_t* ids, const uint64_t* ptr,
               uint64_t n_ids) {
    if (q1 <= q0) return;
    const int64_t pairs = (q1 - q0) * n->n_tiles;
    hipLaunchKernelGGL(republish_kernel, dim3(grid_of(pairs, 256)), dim3(256), 0, n->stream, n->d_pub, n->H,
                       n->n_tiles, n->T, q0, (int)(q1 - q0), ids, ptr, n_ids);
    CX_HIP(hipGetLastError());
}

// Host side of the backward pass (see the file comment).
void adjoint_backward(cortex_net* n, const float* vstar, float* grad_w, double* loss_out);

}  // namespace cortex

namespace cortex {

// Helper defined in api.hip.
void restore_checkpoint(cortex_net* n, int k);

void adjoint_backward(cortex_net* n, const float* vstar, float* grad_w, double* loss_out) {
    const int64_t T = n->step;
    const int C = n->ckpt;
    require(C > 0, CORTEX_ESTATE, "adjoint needs ckpt_every > 0 at build");
    require(T >= 1 && T <= n->adj_steps, CORTEX_ESTATE, "forward window empty or longer than adjoint_steps");
    require(n->log_step0 == 0, CORTEX_ESTATE, "spike log was cleared since the build; the raster is incomplete");
    require(vstar != nullptr && grad_w != nullptr && loss_out != nullptr, CORTEX_EINVAL, "NULL argument");
    require(n->log_steps >= T, CORTEX_ESTATE, "the spike log does not cover the forward window");
    require(T <= 0xFFFF, CORTEX_EUNSUPPORTED, "the adjoint covers at most 65535 steps");
    const int64_t N = n->N;
    const size_t ring_n = (size_t)n->n_tiles * n->R * n->T;
    const size_t pub_n = (size_t)n->H * n->n_tiles * (n->T + 1) + 8;
    // keep the forward's end state to restore afterwards
    float* sv_U = dev_alloc_t<float>(n, N, true);
    float* sv_y1 = dev_alloc_t<float>(n, N, true);
    float* sv_y2 = dev_alloc_t<float>(n, N, true);
    int32_t* sv_r = dev_alloc_t<int32_t>(n, N, true);
    unsigned char* sv_ring = dev_alloc_t<unsigned char>(n, ring_n * n->ring_bytes, true);
    uint64_t* sv_pub = dev_alloc_t<uint64_t>(n, pub_n, true);
    uint64_t* sv_ev = dev_alloc_t<uint64_t>(n, 2 * (size_t)n->n_tiles, true);
    auto d2d = [&](void* dst, const void* src, size_t bytes) {
        CX_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, n->stream));
    };
    d2d(sv_U, n->d_U, N * 4);
    d2d(sv_y1, n->d_y1, N * 4);
    d2d(sv_y2, n->d_y2, N * 4);
    d2d(sv_r, n->d_r, N * 4);
    d2d(sv_ring, n->d_ring, ring_n * n->ring_bytes);
    d2d(sv_pub, n->d_pub, pub_n * 8);
    d2d(sv_ev, n->d_events, n->n_tiles * 8);
    d2d(sv_ev + n->n_tiles, n->d_spikes, n->n_tiles * 8);
    // segment buffers
    float* vtr = dev_alloc_t<float>(n, (size_t)C * N, true);
    uint8_t* mtr = dev_alloc_t<uint8_t>(n, (size_t)C * N, true);
    float* gT = dev_alloc_t<float>(n, (size_t)N * T, true);   // dL/dx over the whole window, per neuron
    double* aU = dev_alloc_t<double>(n, N, true);
    double* a1 = dev_alloc_t<double>(n, N, true);
    double* a2 = dev_alloc_t<double>(n, N, true);
    uint8_t* mnext = dev_alloc_t<uint8_t>(n, N, true);
    double* dloss = dev_alloc_t<double>(n, 1, true);
    const int rev_grid = grid_of(N, 256);
    double* dloss_part = dev_alloc_t<double>(n, rev_grid, true);
    int64_t* inst_N = dev_alloc_t<int64_t>(n, n->n_inst, true);
    CX_HIP(hipMemcpyAsync(inst_N, n->inst_N.data(), n->n_inst * 8, hipMemcpyHostToDevice, n->stream));
    dev_zero(n, aU, N * 8);
    dev_zero(n, a1, N * 8);
    dev_zero(n, a2, N * 8);
    dev_zero(n, mnext, N);
    dev_zero(n, dloss, 8);
    const int64_t saved_log_steps = n->log_steps;
    n->log_steps = 0;   // the replays must not append to the spike log
    // The raster on the device, from the spike log, with its offsets per
    // (step, tile) (the replays' frozen lists and the republished steps) and
    // regrouped by source (the weight gradient), built once for all
    // segments.
    const int64_t pairs = T * n->n_tiles;
    uint64_t* tile_off = dev_alloc_t<uint64_t>(n, (size_t)pairs, true);
    uint32_t* clean = dev_alloc_t<uint32_t>(n, (size_t)pairs, true);
    uint64_t* gpos = dev_alloc_t<uint64_t>(n, (size_t)pairs + 1, true);
    int32_t* bad = dev_alloc_t<int32_t>(n, 1, true);
    dev_zero(n, bad, sizeof(int32_t));
    hipLaunchKernelGGL(log_offsets_kernel, dim3(grid_of((int64_t)n->n_tiles * 64, 256)), dim3(256), 0, n->stream,
                       n->d_log_cnt, T, n->n_tiles, tile_off, bad);
    CX_HIP(hipGetLastError());
    hipLaunchKernelGGL(log_clean_counts_kernel, dim3(grid_of(pairs, 256)), dim3(256), 0, n->stream, n->d_log_cnt,
                       pairs, clean);
    CX_HIP(hipGetLastError());
    scan_counts(n, clean, gpos, pairs);
    int64_t n_spk = 0;
    {
        uint64_t tot = 0;
        int32_t hb = 0;
        CX_HIP(hipMemcpyAsync(&tot, gpos + pairs, sizeof tot, hipMemcpyDeviceToHost, n->stream));
        CX_HIP(hipMemcpyAsync(&hb, bad, sizeof hb, hipMemcpyDeviceToHost, n->stream));
        CX_HIP(hipStreamSynchronize(n->stream));
        require(hb == 0, CORTEX_ESTATE, "spike log overflowed; the raster is incomplete");
        n_spk = (int64_t)tot;
    }
    uint32_t* r_steps = dev_alloc_t<uint32_t>(n, std::max<int64_t>(1, n_spk), true);
    uint32_t* r_ids = dev_alloc_t<uint32_t>(n, std::max<int64_t>(1, n_spk), true);
    uint64_t* r_tile_ptr = dev_alloc_t<uint64_t>(n, (size_t)T * n->n_tiles + 1, true);
    uint32_t* s_cnt = dev_alloc_t<uint32_t>(n, N, true);
    uint32_t* s_cur = dev_alloc_t<uint32_t>(n, N, true);
    uint64_t* sptr = dev_alloc_t<uint64_t>(n, N + 1, true);
    int32_t* sstep = dev_alloc_t<int32_t>(n, std::max<int64_t>(1, n_spk), true);
    uint4* s8 = dev_alloc_t<uint4>(n, N, true);
    {
        hipLaunchKernelGGL(log_copy_kernel, dim3(grid_of(pairs, 256)), dim3(256), 0, n->stream, n->d_log_cnt, tile_off,
                           gpos, n->d_log_base, n->d_log_ids, T, n->n_tiles, N, r_steps, r_ids, bad);
        CX_HIP(hipGetLastError());
        raster_index(n, r_steps, r_ids, n_spk, 0, T, n->d_tile_start, n->n_tiles, r_tile_ptr);
        dev_zero(n, s_cnt, N * 4);
        dev_zero(n, s_cur, N * 4);
        hipLaunchKernelGGL(src_count_kernel, dim3(grid_of(n_spk, 256)), dim3(256), 0, n->stream, r_ids, n_spk, s_cnt);
        CX_HIP(hipGetLastError());
        scan_counts(n, s_cnt, sptr, N);
        hipLaunchKernelGGL(src_fill_kernel, dim3(grid_of(n_spk, 256)), dim3(256), 0, n->stream, r_steps, r_ids, n_spk,
                           sptr, s_cur, sstep);
        CX_HIP(hipGetLastError());
        hipLaunchKernelGGL(src_sort_kernel, dim3(grid_of(N, 256)), dim3(256), 0, n->stream, sptr, sstep, N);
        CX_HIP(hipGetLastError());
        hipLaunchKernelGGL(src_pack_kernel, dim3(grid_of(N, 256)), dim3(256), 0, n->stream, sptr, sstep, N, s8);
        CX_HIP(hipGetLastError());
        int32_t hb = 0;
        CX_HIP(hipMemcpyAsync(&hb, bad, sizeof hb, hipMemcpyDeviceToHost, n->stream));
        CX_HIP(hipStreamSynchronize(n->stream));
        require(hb == 0, CORTEX_EDEVICE, "spike log holds an invalid entry");
    }
    const int K = (int)((T + C - 1) / C);
    try {
        for (int k = K - 1; k >= 0; --k) {
            const int64_t s0 = (int64_t)k * C, s1 = std::min<int64_t>(T, s0 + C), len = s1 - s0;
            restore_checkpoint(n, k);
            n->step = s0;
            // Records left in the publication buffer by the forward run or a
            // later segment carry the same step tags as this replay's and
            // may list the same spikes in another order; a reader mixing two
            // of them would deliver a spike twice and drop another.  Clear
            // the buffer (tag 0 matches no step) before republishing.
            dev_zero(n, n->d_pub, pub_n * 8);
            // spikes of [s0 - d_min, s0) are published but not yet delivered at s0
            const int64_t r0 = std::max<int64_t>(0, s0 - n->dmin);
            if (s0 > r0) republish(n, r0, s0, r_ids, r_tile_ptr + (size_t)r0 * n->n_tiles, (uint64_t)n_spk);
            // bit-exact replay of the segment on the frozen raster; the error
            // flag is read after the last segment (the kernels in between
            // index only by the raster and the records, so a failed replay
            // leaves them in bounds)
            launch_step_fp32(n, len, r_ids, r_tile_ptr + (size_t)s0 * n->n_tiles, (uint64_t)n_spk, nullptr, vtr,
                             mtr);
            // reverse recursion over the segment
            ReverseArgs ra{};
            ra.vtr = vtr; ra.mtr = mtr; ra.vstar = vstar; ra.gT = gT;
            ra.aU = aU; ra.a1 = a1; ra.a2 = a2; ra.m_next = mnext; ra.loss_part = dloss_part;
            ra.inst_n0 = n->d_inst_n0; ra.inst_N = inst_N; ra.n_inst = n->n_inst;
            ra.N = N; ra.s0 = s0; ra.len = len; ra.T = T; ra.model = n->spec.model;
            ra.P22 = n->k.P22; ra.P11 = n->k.P11; ra.P21 = n->k.P21; ra.P31 = n->k.P31;
            ra.P32 = n->k.P32; ra.P21s = n->k.P21s; ra.P22s = n->k.P22s; ra.jump = n->k.jump;
            hipLaunchKernelGGL(reverse_kernel, dim3(rev_grid), dim3(256), 0, n->stream, ra);
            CX_HIP(hipGetLastError());
            hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, n->stream, dloss_part, rev_grid, dloss);
            CX_HIP(hipGetLastError());
        }
        CX_HIP(hipStreamSynchronize(n->stream));
        {
            int32_t e = 0;
            CX_HIP(hipMemcpy(&e, n->d_err, sizeof e, hipMemcpyDeviceToHost));
            if (e != 0) {
                n->failed = true;
                throw Error{CORTEX_ETIMEOUT, "a device-side wait in the adjoint replay exceeded its spin limit"};
            }
        }
        // the weight gradient, in canonical order, into the caller's buffer
        hipLaunchKernelGGL(pull_grad_kernel, dim3(grid_of(N * 64, 256)), dim3(256), 0, n->stream, n->d_cin,
                           n->d_csrc, n->d_cdel, s8, sptr, sstep, gT, N, T, grad_w);
        CX_HIP(hipGetLastError());
        CX_HIP(hipMemcpyAsync(loss_out, dloss, 8, hipMemcpyDeviceToHost, n->stream));
    } catch (...) {
        // drain queued uploads before the staging vectors go away
        (void)hipStreamSynchronize(n->stream);
        n->log_steps = saved_log_steps;
        throw;
    }
    n->log_steps = saved_log_steps;
    d2d(n->d_U, sv_U, N * 4);
    d2d(n->d_y1, sv_y1, N * 4);
    d2d(n->d_y2, sv_y2, N * 4);
    d2d(n->d_r, sv_r, N * 4);
    d2d(n->d_ring, sv_ring, ring_n * n->ring_bytes);
    d2d(n->d_pub, sv_pub, pub_n * 8);
    d2d(n->d_events, sv_ev, n->n_tiles * 8);
    d2d(n->d_spikes, sv_ev + n->n_tiles, n->n_tiles * 8);
    n->step = T;
    CX_HIP(hipStreamSynchronize(n->stream));
}

}  // namespace cortex
