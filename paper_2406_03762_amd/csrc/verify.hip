// FP64 verification step: bit-reproducible pull formulation of one step.
//
// Each target sums, over its in-synapses in the order (delay descending,
// source ascending, canonical index ascending), the weights whose source
// spiked `delay` steps ago; this is exactly the order in which an
// event-driven push fills the target's input buffer (older spikes first,
// then ascending source id), so the FP64 sum is bit-identical to it.  The
// neuron update then applies the same unfused FP64 operations, in the same
// order, as the CPU reference recipe.  Spikes of the recent steps are kept
// as a bitmask ring (one bit per neuron and step, one 64-bit word per
// wavefront written by one lane), the delay history of Sec. III-C.
//
// This file is compiled with -ffp-contract=off.
#include <algorithm>

#include "device_common.hpp"
#include "internal.hpp"

namespace cortex {
namespace {

struct VerifyArgs {
    const uint64_t* in_ptr;
    const uint32_t* in_src;
    const double* in_w;
    const uint16_t* in_d;
    const int64_t* inst_n0;
    int n_inst;
    double* U;
    double* y1;
    double* y2;
    int32_t* r;
    uint64_t* hist;        // [Hr][W] spike bits of recent steps
    uint64_t* log_bits;    // [log_steps][W] or null
    const uint64_t* frz;   // [n_steps][W] frozen spikes or null
    double* x_trace;
    double* v_trace;
    unsigned long long* events;
    int64_t N, W, n0, log_step0, log_steps;
    int Hr, model, n_ref, n_thr;
    double P22, P20Ie, P11, P21, P31, P32, P21s, P22s, jump, theta, Ur, w_ext, E_L;
    double gL, Eex, Ein, Ie, dt_C;   // conductance model (reversal potentials relative to E_L)
    uint64_t seed;
    uint32_t thr[64];
};

template <int MODEL>
__global__ void __launch_bounds__(256) verify_step_kernel(VerifyArgs a, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    bool spk = false;
    unsigned long long ev = 0;
    if (i < a.N) {
        // conductances: excitatory (w >= 0) and inhibitory (|w|) arrivals in
        // two sums, each in the canonical order
        double x = 0.0, xin = 0.0;
        for (uint64_t e = a.in_ptr[i]; e < a.in_ptr[i + 1]; ++e) {
            const int64_t m = n - (int64_t)a.in_d[e];
            if (m < 0) continue;
            const uint32_t j = a.in_src[e];
            const uint64_t word = a.hist[(m & (a.Hr - 1)) * a.W + (j >> 6)];
            if ((word >> (j & 63)) & 1ull) {
                if (MODEL == CORTEX_MODEL_COND && a.in_w[e] < 0.0) xin = xin + (-a.in_w[e]);
                else x = x + a.in_w[e];
                ++ev;
            }
        }
        int lo = 0, hi = a.n_inst;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (a.inst_n0[mid] <= i) lo = mid; else hi = mid;
        }
        int kc = 0;
        if (a.n_thr > 0) {
            const Philox4 p = philox((uint64_t)(i - a.inst_n0[lo]), (uint64_t)(n >> 3), 0, kTagPoisson,
                                     a.seed, (uint64_t)lo);
            const uint64_t word = philox_word(p, (uint32_t)(n & 7) >> 1);
            const uint32_t u = (n & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
            for (int m = 0; m < a.n_thr; ++m) kc += (u >= a.thr[m]) ? 1 : 0;
        }
        const double ext = a.w_ext * (double)kc;
        double U = a.U[i];
        int rr = a.r[i];
        bool integ = false;
        if (MODEL == CORTEX_MODEL_COND) {
            if (rr > 0) {
                rr -= 1;
                U = a.Ur;
            } else {
                integ = true;
                double G = a.gL + a.y1[i];
                G = G + a.y2[i];
                double num = a.y1[i] * a.Eex;
                num = num + a.y2[i] * a.Ein;
                num = num + a.Ie;
                const double u_inf = num / G;
                const double e = exp(-a.dt_C * G);
                U = u_inf + (U - u_inf) * e;
            }
            double gex = a.P11 * a.y1[i];
            double gin = a.P11 * a.y2[i];
            if (ext >= 0.0) gex = gex + ext; else gin = gin - ext;
            a.y1[i] = gex + x;
            a.y2[i] = gin + xin;
            x = x - xin;   // the trace records the signed sum of the arrivals
        } else if (rr > 0) {
            rr -= 1;
            U = a.Ur;
        } else {
            integ = true;
            U = a.P22 * U;
            if (MODEL == CORTEX_MODEL_EXP) {
                U = U + a.P21 * a.y1[i];
            } else if (MODEL == CORTEX_MODEL_ALPHA) {
                U = U + a.P31 * a.y1[i];
                U = U + a.P32 * a.y2[i];
            }
            U = U + a.P20Ie;
            if (MODEL == CORTEX_MODEL_DELTA) U = U + (x + ext);
        }
        if (MODEL == CORTEX_MODEL_EXP) {
            const double c = a.P11 * a.y1[i];
            a.y1[i] = c + (x + ext);
        } else if (MODEL == CORTEX_MODEL_ALPHA) {
            const double y1o = a.y1[i];
            const double t1 = a.P21s * y1o;
            const double t2 = a.P22s * a.y2[i];
            a.y2[i] = t1 + t2;
            const double c = a.P11 * y1o;
            const double jj = a.jump * (x + ext);
            a.y1[i] = c + jj;
        }
        if (a.frz) {
            spk = (a.frz[(n - a.n0) * a.W + (i >> 6)] >> (i & 63)) & 1ull;
        } else {
            spk = integ && U >= a.theta;
        }
        if (spk) {
            U = a.Ur;
            rr = a.n_ref;
        }
        a.U[i] = U;
        a.r[i] = rr;
        if (a.x_trace) {
            a.x_trace[(n - a.n0) * a.N + i] = x;
            a.v_trace[(n - a.n0) * a.N + i] = U + a.E_L;
        }
    }
    // one 64-bit word per wavefront, written by its first lane
    const uint64_t bits = __ballot(spk);
    const int64_t i0 = i - lane;
    if (lane == 0 && i0 < a.N) {
        a.hist[(n & (a.Hr - 1)) * a.W + (i0 >> 6)] = bits;
        if (a.log_bits && n >= a.log_step0 && n < a.log_step0 + a.log_steps)
            a.log_bits[(n - a.log_step0) * a.W + (i0 >> 6)] = bits;
    }
    // events: wave reduction, one counter update per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) ev += __shfl_xor(ev, o, 64);
    if (lane == 0 && ev) atomicAdd(a.events, ev);
    if (lane == 0 && bits) atomicAdd(a.events + 1, (unsigned long long)__popcll(bits));
}

}  // namespace

void launch_step_fp64(cortex_net* n, int64_t n_steps, const uint64_t* frz_bits, double* x_trace,
                      double* v_trace) {
    if (n_steps <= 0) return;
    VerifyArgs a{};
    a.in_ptr = n->d_in_ptr;
    a.in_src = n->d_in_src;
    a.in_w = n->d_in_w;
    a.in_d = n->d_in_d;
    a.inst_n0 = n->d_inst_n0;
    a.n_inst = n->n_inst;
    a.U = n->d_Ud;
    a.y1 = n->d_y1d;
    a.y2 = n->d_y2d;
    a.r = n->d_r;
    a.hist = n->d_hist;
    a.log_bits = n->d_raster;
    a.frz = frz_bits;
    a.x_trace = x_trace;
    a.v_trace = v_trace;
    a.events = reinterpret_cast<unsigned long long*>(n->d_events);
    a.N = n->N;
    a.W = n->W64;
    a.n0 = n->step;
    a.log_step0 = n->log_step0;
    a.log_steps = n->log_steps;
    a.Hr = n->H;
    a.model = n->spec.model;
    a.n_ref = n->k.n_ref;
    a.n_thr = n->n_thr;
    a.P22 = n->k.P22;
    a.P20Ie = n->k.P20 * n->spec.I_e;
    a.P11 = n->k.P11;
    a.P21 = n->k.P21;
    a.P31 = n->k.P31;
    a.P32 = n->k.P32;
    a.P21s = n->k.P21s;
    a.P22s = n->k.P22s;
    a.jump = n->k.jump;
    a.theta = n->spec.V_th - n->spec.E_L;
    a.Ur = n->spec.V_reset - n->spec.E_L;
    a.w_ext = n->w_ext_native;
    a.E_L = n->spec.E_L;
    a.gL = n->spec.C_m / n->spec.tau_m;
    a.Eex = n->spec.E_ex - n->spec.E_L;
    a.Ein = n->spec.E_in - n->spec.E_L;
    a.Ie = n->spec.I_e;
    a.dt_C = n->spec.dt / n->spec.C_m;
    a.seed = n->seed;
    for (int m = 0; m < n->n_thr; ++m) a.thr[m] = n->thr[m];
    const int grid = (int)((n->N + 255) / 256);
    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t step = n->step + s;
        switch (n->spec.model) {
            case CORTEX_MODEL_DELTA:
                hipLaunchKernelGGL(verify_step_kernel<CORTEX_MODEL_DELTA>, dim3(grid), dim3(256), 0,
                                   n->stream, a, step);
                break;
            case CORTEX_MODEL_EXP:
                hipLaunchKernelGGL(verify_step_kernel<CORTEX_MODEL_EXP>, dim3(grid), dim3(256), 0,
                                   n->stream, a, step);
                break;
            case CORTEX_MODEL_COND:
                hipLaunchKernelGGL(verify_step_kernel<CORTEX_MODEL_COND>, dim3(grid), dim3(256), 0,
                                   n->stream, a, step);
                break;
            default:
                hipLaunchKernelGGL(verify_step_kernel<CORTEX_MODEL_ALPHA>, dim3(grid), dim3(256), 0,
                                   n->stream, a, step);
                break;
        }
        CX_HIP(hipGetLastError());
    }
    n->step += n_steps;
}

}  // namespace cortex
