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
// state and the input rings.  The backward walks the segments last to first:
//  1. restore the segment's checkpoint and re-run it on the frozen raster with
//     the step kernel (integer input sums make this a bit-exact replay), which
//     yields V(n) and the mask m(n) = "integrated and did not spike";
//  2. one thread per neuron runs the reverse recursion and writes g(n);
//  3. one workgroup per tile walks, for every source that spiked in the
//     window, the segment of its synapses into the tile -- the same spiking
//     sub-graph (Eq. 11) that delivery reads -- and adds the g values at the
//     arrival steps; each synapse has a single writer (the tile's workgroup,
//     one wave per source), so no atomics are needed.
// A final scatter writes the gradient in canonical synapse order.
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
    float* gtr;            // [len][N] dL/dx
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
__global__ void __launch_bounds__(256) reverse_kernel(ReverseArgs a) {
    double lsum = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.N;
         i += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = a.n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.inst_n0[mid] <= i) lo = mid; else hi = mid;
        }
        const double scale = 1.0 / ((double)a.inst_N[lo] * (double)a.T);
        double aU = a.aU[i], a1 = a.a1[i], a2 = a.a2[i];
        int mn = a.m_next[i];
        for (int64_t k = a.len - 1; k >= 0; --k) {
            const double diff = (double)a.vtr[k * a.N + i] - (double)a.vstar[(a.s0 + k) * a.N + i];
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
            a.gtr[k * a.N + i] = (float)g;
        }
        a.aU[i] = aU;
        a.a1[i] = a1;
        a.a2[i] = a2;
        a.m_next[i] = (uint8_t)mn;
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

struct WgradArgs {
    const int32_t* tile_inst;
    const int32_t* tile_size;
    const int32_t* inst_tile0;
    const int32_t* inst_ntiles;
    const int32_t* inst_T;
    const int64_t* inst_n0;
    const uint64_t* inst_offbase;
    const uint64_t* row_start;
    const uint32_t* off_rel;
    const void* meta;
    int meta16;                 // 16-bit records (alone, or under a bf16 weight when packed)
    int packed;
    int T, dmin, dmax;          // record = (delay - dmin) T + target in tile
    int sw, n_sub;              // steps per sub-window, sub-windows of the segment
    int n_inst;
    const uint32_t* r_ids;      // the raster's ids, sorted by (step, id)
    const uint64_t* r_ptr;      // [step * (n_inst + 1) + b]: instance b's spikes of a step
    int64_t r_steps;            // steps of the raster
    const float* gtr;           // [len][N]
    float* grad;                // [E] storage order
    int64_t N, s0, s1;
};

// Lane i's value of v, for a wave-uniform i.
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int i) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), i);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, i);
    return ((uint64_t)hi << 32) | lo;
}

// One workgroup (16 waves) per tile.  The segment's steps are taken in
// sub-windows of sw steps; for each, the tile's dL/dx values of those steps
// are staged in LDS ([sw][tile size]), then the spikes of the tile's
// instance that can arrive in the sub-window (steps q with [q + d_min,
// q + d_max] meeting it) are read from the raster, 64 at a time per wave.
// Source j belongs to wave j mod 16: that wave walks j's segment into the
// tile (lanes over its synapses) for each of j's spikes in turn and adds,
// per synapse whose arrival q + d falls in the sub-window, the staged value
// there.  A synapse's gradient therefore has one writer, with no atomics.
__global__ void __launch_bounds__(1024) wgrad_kernel(WgradArgs a) {
    extern __shared__ float s_g[];
    const int tile = blockIdx.x;
    const int b = a.tile_inst[tile];
    const int tl = tile - a.inst_tile0[b];
    const int ntb = a.inst_ntiles[b];
    const int tsz = a.tile_size[tile];
    const int64_t n0b = a.inst_n0[b];
    const int64_t g0 = n0b + (int64_t)tl * a.inst_T[b];
    const uint64_t offb = a.inst_offbase[b];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, n_waves = blockDim.x >> 6;
    const uint32_t T = (uint32_t)a.T;
    for (int w = 0; w < a.n_sub; ++w) {
        const int64_t t = a.s0 + (int64_t)w * a.sw;
        const int nw = (int)min((int64_t)a.sw, a.s1 - t);
        __syncthreads();   // the previous sub-window's readers are done
        for (int i = threadIdx.x; i < nw * tsz; i += blockDim.x) {
            const int k = i / tsz, li = i - k * tsz;
            s_g[i] = a.gtr[(t - a.s0 + k) * a.N + g0 + li];
        }
        __syncthreads();
        const int64_t q_lo = max((int64_t)0, t - a.dmax);
        const int64_t q_hi = min(a.r_steps, t + nw - a.dmin);
        for (int64_t q = q_lo; q < q_hi; ++q) {
            const uint64_t p0 = a.r_ptr[q * (a.n_inst + 1) + b], p1 = a.r_ptr[q * (a.n_inst + 1) + b + 1];
            for (uint64_t pc = p0; pc < p1; pc += 64) {
                // this wave's spikes among the next 64: their segment bounds
                // are loaded by their own lanes, together
                const uint64_t p = pc + (uint64_t)lane;
                uint32_t j = 0;
                bool own = false;
                uint64_t e0l = 0, e1l = 0;
                if (p < p1) {
                    j = a.r_ids[p];
                    own = (int)(j % (uint32_t)n_waves) == wave;
                    if (own) {
                        const uint64_t ob = offb + (uint64_t)(j - n0b) * (uint64_t)(ntb + 1) + (uint64_t)tl;
                        const uint64_t rs = a.row_start[j];
                        e0l = rs + a.off_rel[ob];
                        e1l = rs + a.off_rel[ob + 1];
                    }
                }
                uint64_t mask = __ballot(own);
                while (mask) {
                    const int i = __ffsll((unsigned long long)mask) - 1;
                    mask &= mask - 1;
                    const uint64_t e0 = lane_u64(e0l, i), e1 = lane_u64(e1l, i);
                    // four synapses per lane at a time: records first, then
                    // the gradients of those arriving in the sub-window
                    for (uint64_t eb = e0 + lane; eb < e1; eb += 256) {
                        int32_t at[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const uint64_t e = eb + 64u * u;
                            at[u] = -1;
                            if (e < e1) {
                                const uint32_t m = a.packed ? (static_cast<const uint32_t*>(a.meta)[e] & 0xFFFFu)
                                                   : a.meta16 ? static_cast<const uint16_t*>(a.meta)[e]
                                                              : static_cast<const uint32_t*>(a.meta)[e];
                                const int64_t tau = q + a.dmin + (int64_t)(m / T);
                                if (tau >= t && tau < t + nw) at[u] = (int32_t)((tau - t) * tsz + (int64_t)(m % T));
                            }
                        }
                        float g[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) g[u] = at[u] >= 0 ? a.grad[eb + 64u * u] : 0.f;
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            if (at[u] >= 0) a.grad[eb + 64u * u] = g[u] + s_g[at[u]];
                    }
                }
            }
        }
    }
}

// dst in canonical order from src in storage order: dst[c] = src[inv[c]].
__global__ void gather_kernel(const float* src, const uint32_t* inv, float* dst, int64_t E) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < E;
         c += (int64_t)gridDim.x * blockDim.x)
        dst[c] = src[inv[c]];
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

// Helpers defined in api.hip.
std::vector<std::pair<uint32_t, uint32_t>> collect_spikes(cortex_net* n, int64_t s0, int64_t s1, bool* trunc);
void restore_checkpoint(cortex_net* n, int k);

void adjoint_backward(cortex_net* n, const float* vstar, float* grad_w, double* loss_out) {
    const int64_t T = n->step;
    const int C = n->ckpt;
    require(C > 0, CORTEX_ESTATE, "adjoint needs ckpt_every > 0 at build");
    require(T >= 1 && T <= n->adj_steps, CORTEX_ESTATE, "forward window empty or longer than adjoint_steps");
    require(n->log_step0 == 0, CORTEX_ESTATE, "spike log was cleared since the build; the raster is incomplete");
    require(vstar != nullptr && grad_w != nullptr && loss_out != nullptr, CORTEX_EINVAL, "NULL argument");
    bool trunc = false;
    const auto raster = collect_spikes(n, 0, T, &trunc);
    require(!trunc, CORTEX_ESTATE, "spike log overflowed; the raster is incomplete");
    for (const auto& sp : raster)
        require((int64_t)sp.first < T && (int64_t)sp.second < n->N, CORTEX_EDEVICE, "spike log holds an invalid entry");
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
    float* gtr = dev_alloc_t<float>(n, (size_t)C * N, true);
    double* aU = dev_alloc_t<double>(n, N, true);
    double* a1 = dev_alloc_t<double>(n, N, true);
    double* a2 = dev_alloc_t<double>(n, N, true);
    uint8_t* mnext = dev_alloc_t<uint8_t>(n, N, true);
    double* dloss = dev_alloc_t<double>(n, 1, true);
    const int rev_grid = grid_of(N, 256);
    double* dloss_part = dev_alloc_t<double>(n, rev_grid, true);
    float* grad = dev_alloc_t<float>(n, n->E, true);
    int64_t* inst_N = dev_alloc_t<int64_t>(n, n->n_inst, true);
    // weight-gradient sub-windows: sw steps of a tile's dL/dx in at most
    // 160 KB of LDS
    const int sw = (int)std::max<int64_t>(1, std::min<int64_t>(C, 40960 / std::max(1, n->T)));
    const size_t wgrad_lds = (size_t)sw * n->T * sizeof(float);
    CX_HIP(hipFuncSetAttribute((const void*)wgrad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)wgrad_lds));
    CX_HIP(hipMemcpyAsync(inst_N, n->inst_N.data(), n->n_inst * 8, hipMemcpyHostToDevice, n->stream));
    dev_zero(n, aU, N * 8);
    dev_zero(n, a1, N * 8);
    dev_zero(n, a2, N * 8);
    dev_zero(n, mnext, N);
    dev_zero(n, dloss, 8);
    dev_zero(n, grad, (size_t)n->E * 4);
    const int64_t saved_log_steps = n->log_steps;
    n->log_steps = 0;   // the replays must not append to the spike log
    // The raster on the device, with its offsets per (step, tile) (the
    // replays' frozen lists and the republished steps) and per (step,
    // instance) (the weight gradient's spikes), built once for all segments.
    const int64_t n_spk = (int64_t)raster.size();
    uint32_t* r_steps = dev_alloc_t<uint32_t>(n, std::max<int64_t>(1, n_spk), true);
    uint32_t* r_ids = dev_alloc_t<uint32_t>(n, std::max<int64_t>(1, n_spk), true);
    uint64_t* r_tile_ptr = dev_alloc_t<uint64_t>(n, (size_t)T * n->n_tiles + 1, true);
    uint64_t* r_inst_ptr = dev_alloc_t<uint64_t>(n, (size_t)T * (n->n_inst + 1) + 1, true);
    int64_t* inst_keys = dev_alloc_t<int64_t>(n, n->n_inst + 1, true);
    {
        std::vector<uint32_t> hs((size_t)n_spk), hi((size_t)n_spk);
        for (int64_t q = 0; q < n_spk; ++q) {
            hs[q] = raster[q].first;
            hi[q] = raster[q].second;
        }
        std::vector<int64_t> keys(n->inst_n0.begin(), n->inst_n0.end());
        keys.push_back(N);
        if (n_spk > 0) {
            CX_HIP(hipMemcpyAsync(r_steps, hs.data(), n_spk * 4, hipMemcpyHostToDevice, n->stream));
            CX_HIP(hipMemcpyAsync(r_ids, hi.data(), n_spk * 4, hipMemcpyHostToDevice, n->stream));
        }
        CX_HIP(hipMemcpyAsync(inst_keys, keys.data(), keys.size() * 8, hipMemcpyHostToDevice, n->stream));
        raster_index(n, r_steps, r_ids, n_spk, 0, T, n->d_tile_start, n->n_tiles, r_tile_ptr);
        raster_index(n, r_steps, r_ids, n_spk, 0, T, inst_keys, n->n_inst + 1, r_inst_ptr);
        CX_HIP(hipStreamSynchronize(n->stream));   // before the staging vectors go away
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
            ra.vtr = vtr; ra.mtr = mtr; ra.vstar = vstar; ra.gtr = gtr;
            ra.aU = aU; ra.a1 = a1; ra.a2 = a2; ra.m_next = mnext; ra.loss_part = dloss_part;
            ra.inst_n0 = n->d_inst_n0; ra.inst_N = inst_N; ra.n_inst = n->n_inst;
            ra.N = N; ra.s0 = s0; ra.len = len; ra.T = T; ra.model = n->spec.model;
            ra.P22 = n->k.P22; ra.P11 = n->k.P11; ra.P21 = n->k.P21; ra.P31 = n->k.P31;
            ra.P32 = n->k.P32; ra.P21s = n->k.P21s; ra.P22s = n->k.P22s; ra.jump = n->k.jump;
            hipLaunchKernelGGL(reverse_kernel, dim3(rev_grid), dim3(256), 0, n->stream, ra);
            CX_HIP(hipGetLastError());
            hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, n->stream, dloss_part, rev_grid, dloss);
            CX_HIP(hipGetLastError());
            // weight gradient of the synapses whose arrivals land in the segment
            if (n_spk > 0) {
                WgradArgs wa{};
                wa.tile_inst = n->d_tile_inst; wa.tile_size = n->d_tile_size; wa.inst_tile0 = n->d_inst_tile0;
                wa.inst_ntiles = n->d_inst_ntiles; wa.inst_T = n->d_inst_T; wa.inst_n0 = n->d_inst_n0;
                wa.inst_offbase = n->d_inst_offbase;
                wa.row_start = n->d_row_start; wa.off_rel = n->d_off_rel; wa.meta = n->d_meta;
                wa.meta16 = n->meta_bytes == 2; wa.packed = n->w_bytes == 2; wa.T = n->T;
                wa.dmin = n->dmin; wa.dmax = n->dmax;
                wa.sw = sw; wa.n_sub = (int)((len + sw - 1) / sw); wa.n_inst = n->n_inst;
                wa.r_ids = r_ids; wa.r_ptr = r_inst_ptr; wa.r_steps = T;
                wa.gtr = gtr; wa.grad = grad; wa.N = N; wa.s0 = s0; wa.s1 = s1;
                hipLaunchKernelGGL(wgrad_kernel, dim3(n->n_tiles), dim3(1024), wgrad_lds, n->stream, wa);
                CX_HIP(hipGetLastError());
            }
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
        hipLaunchKernelGGL(gather_kernel, dim3(grid_of(n->E, 256)), dim3(256), 0, n->stream, grad,
                           n->d_canon_inv, grad_w, n->E);
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
