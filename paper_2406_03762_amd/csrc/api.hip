// Host side of libcortex: specification checks, model constants, planning of
// the indegree tiles, device memory, and the extern "C" entry points.
//
// This file is compiled with -ffp-contract=off: the FP64 model constants
// follow the documented recipe operation by operation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace cortex {

namespace {
thread_local std::string g_error = "";
}

void set_error(const std::string& msg) { g_error = msg; }

static void save_checkpoint(cortex_net* n, int k);

// ----------------------------------------------------------------------------
// Model constants.  The membrane equation tau dU/dt = -U + R I (Eq. 1, with
// U = u - u_rest and R = tau/C) is linear between spikes, so one step of
// length dt is the exact linear map exp(A dt) of the (U, synaptic state)
// system:
//   P22 = e^{-dt/tm}                        U <- P22 U
//   P20 = (tm/C)(1 - e^{-dt/tm})            constant current I_e
//   exp kernel, a = 1/ts - 1/tm:
//   P11 = e^{-dt/ts}                        I <- P11 I
//   P21 = P22 (1 - e^{-a dt}) / (C a)       U gains P21 I
//   alpha kernel (y1 auxiliary, y2 current):
//   P21s = dt P11, P22s = P11               y2 <- P21s y1 + P22s y2
//   P31 = P22 (1 - e^{-a dt}(1 + a dt)) / (C a^2)   U gains P31 y1 + P32 y2
//   P32 = P21;  an input w adds (e/ts) w to y1 (current peaks at w).
// The expressions below are the shared recipe (same operations as the CPU
// reference), so FP64 networks reproduce its rounding exactly.
Consts model_constants(const cortex_spec& s) {
    Consts k{};
    const double dt = s.dt, tm = s.tau_m, ts = s.tau_syn, C = s.C_m;
    k.P22 = std::exp(-dt / tm);
    k.P20 = -(tm / C) * std::expm1(-dt / tm);
    k.jump = 1.0;
    k.conv = 1.0;
    if (s.model == CORTEX_MODEL_COND) {
        k.P11 = std::exp(-dt / ts);   // conductance decay per step
    } else if (s.model != CORTEX_MODEL_DELTA) {
        const double a = 1.0 / ts - 1.0 / tm;
        k.P11 = std::exp(-dt / ts);
        k.P21 = (a == 0.0) ? k.P22 * dt / C : k.P22 * (-std::expm1(-a * dt)) / (C * a);
        if (s.model == CORTEX_MODEL_ALPHA) {
            k.P21s = dt * k.P11;
            k.P22s = k.P11;
            k.P32 = k.P21;
            k.P31 = (a == 0.0) ? k.P22 * dt * dt / (2.0 * C)
                               : k.P22 * (1.0 - std::exp(-a * dt) * (1.0 + a * dt)) / (C * a * a);
            k.jump = 2.71828182845904523536 / ts;
        }
        if (s.weight_unit == CORTEX_UNIT_PSP_MV) {
            // PSP of a unit input: v(t) = (1/C) int_0^t e^{-(t-s)/tm} I(s) ds with
            // I(s) = e^{-s/ts} (exp) or (s/ts) e^{1-s/ts} (alpha); its maximum is
            // where v'(t) = I(t)/C - v(t)/tm = 0.  Newton on v' from a bracket.
            auto v = [&](double t) {
                if (s.model == CORTEX_MODEL_EXP)
                    return (a == 0.0) ? std::exp(-t / tm) * t / C
                                      : std::exp(-t / tm) * (-std::expm1(-a * t)) / (C * a);
                const double g = (a == 0.0) ? t * t / 2.0
                                            : (1.0 - std::exp(-a * t) * (1.0 + a * t)) / (a * a);
                return (2.71828182845904523536 / (C * ts)) * std::exp(-t / tm) * g;
            };
            auto cur = [&](double t) {
                return s.model == CORTEX_MODEL_EXP ? std::exp(-t / ts)
                                                   : (t / ts) * std::exp(1.0 - t / ts);
            };
            auto dv = [&](double t) { return cur(t) / C - v(t) / tm; };
            double lo = 1e-9 * std::min(ts, tm), hi = 50.0 * std::max(ts, tm);
            for (int it = 0; it < 200 && hi - lo > 1e-15 * hi; ++it) {
                const double mid = 0.5 * (lo + hi);
                (dv(mid) > 0.0 ? lo : hi) = mid;
            }
            double t = 0.5 * (lo + hi);
            for (int it = 0; it < 5; ++it) {   // polish with secant steps on v'
                const double h = 1e-7 * t;
                const double d1 = dv(t), d2 = (dv(t + h) - dv(t - h)) / (2.0 * h);
                if (d2 == 0.0) break;
                const double tn = t - d1 / d2;
                if (!(tn > 0.0)) break;
                t = tn;
            }
            k.conv = 1.0 / v(t);
        }
    }
    k.n_ref = (int)std::floor(s.t_ref / dt + 0.5);
    if (k.n_ref < 0) k.n_ref = 0;
    return k;
}

// Poisson counts by inversion: count = #{m : u >= thr[m]} for a uniform
// 32-bit u, with thr[m] = floor(F(m) 2^32) while that is below 2^32 - 1
// (the omitted tail is below 2^-32); F accumulated as p_m = p_{m-1} l / m.
int poisson_thresholds(double lambda, uint32_t* thr, int cap) {
    if (lambda == 0.0) return 0;
    double p = std::exp(-lambda);
    double F = p;
    int m = 0;
    for (; m < cap; ) {
        const double t = F * 4294967296.0;
        if (t >= 4294967295.0) break;
        thr[m] = (uint32_t)t;
        ++m;
        p = p * lambda / (double)m;
        F = F + p;
    }
    return m < cap ? m : -1;
}

// ----------------------------------------------------------------------------
// Device memory through the caller's allocator.
void* dev_alloc(cortex_net* n, size_t bytes, bool scratch) {
    bytes = (bytes + 255) & ~(size_t)255;
    void* p = nullptr;
    if (n->dev.alloc) {
        p = n->dev.alloc(bytes, n->dev.user);
        require(p != nullptr, CORTEX_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    } else {
        const hipError_t e = hipMalloc(&p, bytes);
        require(e == hipSuccess && p, CORTEX_ENOMEM,
                "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    (scratch ? n->scratch : n->bufs).push_back(DevBuf{p, bytes});
    n->dev_bytes += scratch ? 0 : bytes;
    return p;
}

static void release(cortex_net* n, std::vector<DevBuf>& v) {
    for (auto& b : v) {
        if (!b.p) continue;
        if (n->dev.alloc) {
            if (n->dev.free) n->dev.free(b.p, n->dev.user);
        } else {
            (void)hipFree(b.p);
        }
    }
    v.clear();
}

void free_scratch(cortex_net* n) {
    (void)hipStreamSynchronize(n->stream);
    release(n, n->scratch);
}

void free_scratch_from(cortex_net* n, size_t mark) {
    if (mark >= n->scratch.size()) return;
    (void)hipStreamSynchronize(n->stream);
    std::vector<DevBuf> tail(n->scratch.begin() + (std::ptrdiff_t)mark, n->scratch.end());
    n->scratch.resize(mark);
    release(n, tail);
}

void dev_zero(cortex_net* n, void* p, size_t bytes) {
    if (bytes) CX_HIP(hipMemsetAsync(p, 0, bytes, n->stream));
}

// Host-to-device copy that has completed on return, so `src` may be freed.
template <class T>
static void upload(cortex_net* n, T* dst, const std::vector<T>& src) {
    if (src.empty()) return;
    CX_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
}

template <class T>
static std::vector<T> download(cortex_net* n, const T* src, size_t count) {
    std::vector<T> v(count);
    if (count) CX_HIP(hipMemcpyAsync(v.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, n->stream));
    CX_HIP(hipStreamSynchronize(n->stream));
    return v;
}

// ----------------------------------------------------------------------------
static int32_t steps_of_ms(double ms, double dt) {
    const double x = ms / dt + 0.5;
    const double f = std::floor(x);
    if (f < 1.0) return 1;
    if (f > 1e9) return 1000000000;
    return (int32_t)f;
}

static void validate(const cortex_spec* s) {
    require(s != nullptr, CORTEX_EINVAL, "spec is NULL");
    require(s->abi_version == CORTEX_ABI_VERSION, CORTEX_EINVAL, "spec ABI version mismatch");
    require(s->struct_size == sizeof(cortex_spec), CORTEX_EINVAL, "spec struct size mismatch");
    require(s->model >= 0 && s->model <= 3, CORTEX_EINVAL, "unknown neuron model");
    if (s->model == CORTEX_MODEL_COND) {
        require(s->weight_unit == CORTEX_UNIT_NATIVE, CORTEX_EINVAL, "conductance synapses take native weights (nS)");
        require(s->weight_dtype == CORTEX_W_FP32 && !s->stdp_enable && s->ckpt_every == 0 &&
                    s->plan_kind != CORTEX_PLAN_STREAMED,
                CORTEX_EUNSUPPORTED,
                "conductance synapses run on the resident plan with FP32 weights, without plasticity or adjoint");
    }
    require(s->precision == CORTEX_FP32 || s->precision == CORTEX_FP64_VERIFY, CORTEX_EINVAL, "unknown precision");
    require(s->weight_dtype == CORTEX_W_FP32 || s->weight_dtype == CORTEX_W_BF16, CORTEX_EINVAL, "unknown weight dtype");
    require(s->weight_unit == CORTEX_UNIT_NATIVE || s->weight_unit == CORTEX_UNIT_PSP_MV, CORTEX_EINVAL, "unknown weight unit");
    require(s->dt > 0 && s->tau_m > 0 && s->C_m > 0, CORTEX_EINVAL, "dt, tau_m and C_m must be positive");
    require(s->model == CORTEX_MODEL_DELTA || s->tau_syn > 0, CORTEX_EINVAL, "tau_syn must be positive");
    require(s->V_reset < s->V_th, CORTEX_EINVAL, "V_reset must lie below V_th");
    require(s->t_ref >= 0, CORTEX_EINVAL, "t_ref must be >= 0");
    require(s->poisson_lambda >= 0 && s->poisson_lambda <= 50, CORTEX_EINVAL, "poisson_lambda must be in [0, 50]");
    require(s->n_instances >= 1 && s->n_pops >= 1 && s->pops, CORTEX_EINVAL, "need instances and populations");
    require(s->block_size == 0 || s->block_size == 256 || s->block_size == 512 || s->block_size == 1024,
            CORTEX_EINVAL, "block_size must be 0, 256, 512 or 1024");
    require(s->tile_size >= 0 && s->record_steps >= 0 && s->ckpt_every >= 0 && s->adjoint_steps >= 0 &&
                s->spin_limit_log2 >= 0 && s->spin_limit_log2 <= 40 && s->steps_per_sync >= 0,
            CORTEX_EINVAL, "negative planning field");
    require(s->plan_kind >= CORTEX_PLAN_AUTO && s->plan_kind <= CORTEX_PLAN_STREAMED, CORTEX_EINVAL,
            "unknown plan kind");
    require(s->wg_per_cu == 0 || s->wg_per_cu == 1 || s->wg_per_cu == 2 || s->wg_per_cu == 4 || s->wg_per_cu == 8,
            CORTEX_EINVAL, "wg_per_cu must be 0, 1, 2, 4 or 8");
    require(s->n_projs >= 0 && (s->n_projs == 0 || s->projs), CORTEX_EINVAL, "projection list is NULL");
    require(s->ckpt_every == 0 || s->adjoint_steps <= 0xFFFF, CORTEX_EUNSUPPORTED,
            "the adjoint covers at most 65535 steps");
    if (s->stdp_enable) {
        require(s->stdp_pop >= 0 && s->stdp_pop < s->n_pops, CORTEX_EINVAL, "stdp_pop out of range");
        require(s->stdp_lambda >= 0 && s->stdp_alpha >= 0 && s->stdp_tau_plus > 0 && s->stdp_tau_minus > 0 &&
                    s->stdp_w0 > 0 && s->stdp_wmax > 0,
                CORTEX_EINVAL, "bad plasticity parameters");
        require(s->precision == CORTEX_FP32 && s->weight_dtype == CORTEX_W_FP32, CORTEX_EUNSUPPORTED,
                "plasticity needs FP32 precision and FP32 weights");
        require(s->ckpt_every == 0, CORTEX_EUNSUPPORTED, "the adjoint of a plastic network is not supported");
        require(s->plan_kind != CORTEX_PLAN_RESIDENT, CORTEX_EUNSUPPORTED,
                "plasticity runs on the streamed plan only");
    }
    int prev = 0;
    std::vector<int> seen(s->n_instances, 0);
    int64_t N = 0;
    for (int p = 0; p < s->n_pops; ++p) {
        const cortex_pop& P = s->pops[p];
        require(P.instance >= 0 && P.instance < s->n_instances && P.instance >= prev, CORTEX_EINVAL,
                "populations must be grouped by instance in ascending order");
        require(P.size >= 1, CORTEX_EINVAL, "population size must be >= 1");
        prev = P.instance;
        seen[P.instance] = 1;
        N += P.size;
    }
    for (int b = 0; b < s->n_instances; ++b) require(seen[b], CORTEX_EINVAL, "instance without population");
    require(N < ((int64_t)1 << 31), CORTEX_EUNSUPPORTED, "at most 2^31 - 1 neurons");
    for (int q = 0; q < s->n_projs; ++q) {
        const cortex_proj& R = s->projs[q];
        require(R.src_pop >= 0 && R.src_pop < s->n_pops && R.tgt_pop >= 0 && R.tgt_pop < s->n_pops,
                CORTEX_EINVAL, "projection population index out of range");
        require(s->pops[R.src_pop].instance == s->pops[R.tgt_pop].instance, CORTEX_EINVAL,
                "projection crosses instances");
        require(R.rule == CORTEX_RULE_FIXED_INDEGREE || R.rule == CORTEX_RULE_PAIRWISE, CORTEX_EINVAL, "unknown rule");
        require(R.rule != CORTEX_RULE_FIXED_INDEGREE || (R.k >= 0 && R.k < (1 << 30)), CORTEX_EINVAL, "bad in-degree");
        require(R.rule != CORTEX_RULE_PAIRWISE || (R.p >= 0 && R.p <= 1), CORTEX_EINVAL, "p outside [0, 1]");
        require(R.delay_kind >= 0 && R.delay_kind <= 2, CORTEX_EINVAL, "unknown delay kind");
        require(R.delay_kind != CORTEX_DELAY_UNIFORM_INT || (R.d0 >= 1 && R.d1 >= R.d0 && R.d1 < 65535),
                CORTEX_EINVAL, "uniform delay needs 1 <= lo <= hi steps");
        require(R.w_sd >= 0 && std::isfinite(R.w_mean), CORTEX_EINVAL, "bad weight distribution");
        const bool same = R.src_pop == R.tgt_pop && !R.autapses;
        require(!(same && R.rule == CORTEX_RULE_FIXED_INDEGREE && R.k > 0 && s->pops[R.src_pop].size < 2),
                CORTEX_EINVAL, "no source left without autapses");
    }
}

// Generation blocks in canonical order and instance tables.
static void make_blocks(cortex_net* n) {
    const cortex_spec& s = n->spec;
    std::vector<int64_t> pop_g0(n->pops.size() + 1, 0);
    for (size_t p = 0; p < n->pops.size(); ++p) pop_g0[p + 1] = pop_g0[p] + n->pops[p].size;
    n->N = pop_g0.back();
    n->n_inst = s.n_instances;
    n->inst_n0.assign(n->n_inst, 0);
    n->inst_N.assign(n->n_inst, 0);
    for (int b = n->n_inst - 1, p = (int)n->pops.size() - 1; b >= 0; --b) {
        while (p >= 0 && n->pops[p].instance == b) {
            n->inst_n0[b] = pop_g0[p];
            n->inst_N[b] += n->pops[p].size;
            --p;
        }
    }
    std::vector<int32_t> proj_local(n->projs.size(), 0);
    std::vector<int> count(n->n_inst, 0);
    for (size_t q = 0; q < n->projs.size(); ++q) {
        const int b = n->pops[n->projs[q].tgt_pop].instance;
        proj_local[q] = count[b]++;
    }
    n->blocks.clear();
    for (size_t p = 0; p < n->pops.size(); ++p) {
        const int b = n->pops[p].instance;
        for (size_t q = 0; q < n->projs.size(); ++q) {
            const cortex_proj& R = n->projs[q];
            if (R.tgt_pop != (int32_t)p) continue;
            GenBlock B{};
            B.tgt0 = pop_g0[p];
            B.n_tgt = n->pops[p].size;
            B.inst_n0 = n->inst_n0[b];
            B.src0_local = pop_g0[R.src_pop] - n->inst_n0[b];
            B.n_src = n->pops[R.src_pop].size;
            B.k = R.rule == CORTEX_RULE_FIXED_INDEGREE ? R.k : 0;
            B.all_pairs = R.rule == CORTEX_RULE_PAIRWISE && R.p >= 1.0;
            B.thr_p = (R.rule == CORTEX_RULE_PAIRWISE && R.p < 1.0) ? (uint64_t)std::ldexp(R.p, 64) : ~0ull;
            B.w_mean = R.w_mean;
            B.w_sd = R.w_sd;
            B.d0 = R.d0;
            B.d1 = R.d1;
            B.rule = R.rule;
            B.delay_kind = R.delay_kind;
            B.same_pop_no_autapse = (R.src_pop == R.tgt_pop && !R.autapses) ? 1 : 0;
            B.proj_local = proj_local[q];
            B.instance = b;
            const bool empty = (R.rule == CORTEX_RULE_FIXED_INDEGREE && R.k == 0) ||
                               (R.rule == CORTEX_RULE_PAIRWISE && R.p <= 0.0);
            if (!empty) n->blocks.push_back(B);
        }
    }
}

// Delay range known from the specification.  Normal delays need a device
// pass over the drawn values, unless `bound` asks for the widest range any
// draw can give (a Box-Muller normal stays within 8.6 standard deviations).
static bool host_delay_range(const cortex_net* n, int* dmin, int* dmax, bool bound = false) {
    int lo = 1 << 30, hi = 0;
    for (const auto& B : n->blocks) {
        if (B.delay_kind == CORTEX_DELAY_NORMAL && !bound) return false;
        int a, b;
        if (B.delay_kind == CORTEX_DELAY_NORMAL) {
            a = steps_of_ms(B.d0 - 8.6 * B.d1, n->spec.dt);
            b = steps_of_ms(B.d0 + 8.6 * B.d1, n->spec.dt);
        } else if (B.delay_kind == CORTEX_DELAY_CONST) {
            a = b = steps_of_ms(B.d0, n->spec.dt);
        } else {
            a = (int)B.d0;
            b = (int)B.d1;
        }
        lo = std::min(lo, a);
        hi = std::max(hi, b);
    }
    if (hi == 0) lo = hi = 1;
    *dmin = lo;
    *dmax = hi;
    return true;
}

// Fraction bits of the 64-bit fixed-point input rings: the largest scale at
// which every target's total absolute in-weight still fits in 62 bits.  A
// Box-Muller normal never exceeds sqrt(-2 ln 2^-53) < 8.6, which bounds every
// drawn weight; pairwise projections count every source as connected.
static int fixed_point_bits(const cortex_net* n) {
    const double conv = (n->spec.weight_unit == CORTEX_UNIT_PSP_MV) ? n->k.conv : 1.0;
    std::vector<double> per_pop(n->pops.size(), 0.0);
    for (const auto& B : n->blocks) {
        const double wmax = (std::fabs(B.w_mean) + 8.6 * B.w_sd) * std::fabs(conv) * (1.0 + 1e-6);
        const double cnt = (B.rule == CORTEX_RULE_FIXED_INDEGREE) ? (double)B.k : (double)B.n_src;
        for (size_t p = 0; p < n->pops.size(); ++p) {
            int64_t g0 = 0;
            for (size_t q = 0; q < p; ++q) g0 += n->pops[q].size;
            if (g0 == B.tgt0) per_pop[p] += cnt * wmax;
        }
    }
    double bound = 1e-30;
    for (double v : per_pop) bound = std::max(bound, v);
    int fx = 61 - (int)std::ceil(std::log2(bound + 1.0));
    return std::max(0, std::min(fx, 52));
}

// Shift that keeps every single weight below 2^31 at scale 2^(fx - shift),
// so the kernel converts a weight with one 32-bit rounding and widens it to
// the ring's 64-bit scale 2^fx with an exact shift.
static int fixed_point_shift(const cortex_net* n, int fx) {
    const double conv = (n->spec.weight_unit == CORTEX_UNIT_PSP_MV) ? n->k.conv : 1.0;
    double wmax = 1e-30;
    for (const auto& B : n->blocks)
        wmax = std::max(wmax, (std::fabs(B.w_mean) + 8.6 * B.w_sd) * std::fabs(conv) * (1.0 + 1e-6));
    const int fxw = 30 - (int)std::ceil(std::log2(wmax));
    return std::max(0, fx - std::max(0, fxw));
}

static int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Tiles of T_b consecutive targets per instance b (the last one shorter):
// the partition of Eq. 9-10, one indegree sub-graph per tile.
static void make_tiles(cortex_net* n, const std::vector<int32_t>& Tb) {
    n->inst_T = Tb;
    n->n_tiles = 0;
    n->inst_tile0.assign(n->n_inst, 0);
    n->inst_ntiles.assign(n->n_inst, 0);
    n->inst_offbase.assign(n->n_inst, 0);
    n->tile_start.clear();
    n->tile_size.clear();
    n->tile_inst.clear();
    uint64_t off = 0;
    n->ntb_max = 1;
    for (int b = 0; b < n->n_inst; ++b) {
        const int Tb_ = Tb[b];
        const int nt = (int)((n->inst_N[b] + Tb_ - 1) / Tb_);
        n->inst_tile0[b] = n->n_tiles;
        n->inst_ntiles[b] = nt;
        n->inst_offbase[b] = off;
        off += (uint64_t)n->inst_N[b] * (nt + 1);
        for (int t = 0; t < nt; ++t) {
            n->tile_start.push_back(n->inst_n0[b] + (int64_t)t * Tb_);
            n->tile_size.push_back((int32_t)std::min<int64_t>(Tb_, n->inst_N[b] - (int64_t)t * Tb_));
            n->tile_inst.push_back(b);
        }
        n->n_tiles += nt;
        n->ntb_max = std::max(n->ntb_max, nt);
    }
}

// Mean in-degree of every instance (expected synapses per target).
static std::vector<double> mean_indegree(const cortex_net* n) {
    std::vector<double> K(n->n_inst, 0.0);
    for (const auto& B : n->blocks) {
        const double per_tgt = B.rule == CORTEX_RULE_FIXED_INDEGREE
                                   ? (double)B.k
                                   : (B.all_pairs ? 1.0 : std::ldexp((double)B.thr_p, -64)) * (double)B.n_src;
        K[B.instance] += per_tgt * (double)B.n_tgt;
    }
    for (int b = 0; b < n->n_inst; ++b) K[b] = std::max(1.0, K[b] / (double)n->inst_N[b]);
    return K;
}

// Tile sizes.  Every tile's workgroup must be resident at once and its input
// ring must fit the workgroup-local memory.  Instances of different sizes get
// different tile sizes so that every tile holds about the same number of
// synapses (the memory/edge-count balance of Sec. III-A): T_b ~ C / K_b for
// mean in-degree K_b, with C the smallest load that fits the device.
// Resident workgroups of a kernel variant per compute unit: asked of the
// runtime on a live device, else bounded by LDS and threads alone.
static int occupancy(const cortex_net* n, bool streamed, int meta, int w_bytes, int npt, int bs, size_t lds) {
    if (n->dd.live)
        return streamed ? stream_occupancy(n->spec.model, meta, w_bytes, npt, bs, lds)
                        : step_occupancy(n->spec.model, meta, w_bytes, npt, bs, lds, n->ring_bytes);
    if (w_bytes == 2 && meta != 2) return 0;   // no kernel for bf16 with 32-bit records
    if (!streamed && npt == 4 && bs != 512) return 0;   // launch bound of the four-neuron variant
    return (int)std::min<size_t>((size_t)(n->dd.thr_cu / bs), lds ? n->dd.lds_cu / lds : 64);
}

static void plan_tiles(cortex_net* n) {
    const int n_cu = n->dd.n_cu;
    const size_t lds_cu = n->dd.lds_cu;
    const int thr_cu = n->dd.thr_cu;
    std::vector<double> K(n->n_inst, 0.0);
    for (const auto& B : n->blocks) {
        const double per_tgt = B.rule == CORTEX_RULE_FIXED_INDEGREE
                                   ? (double)B.k
                                   : (B.all_pairs ? 1.0 : std::ldexp((double)B.thr_p, -64)) * (double)B.n_src;
        K[B.instance] += per_tgt * (double)B.n_tgt;
    }
    for (int b = 0; b < n->n_inst; ++b) K[b] = std::max(1.0, K[b] / (double)n->inst_N[b]);
    auto sizes_for = [&](double C, int Tcap) {
        std::vector<int32_t> Tb(n->n_inst);
        for (int b = 0; b < n->n_inst; ++b) {
            const double t = std::floor(C / K[b]);
            Tb[b] = (int32_t)std::max<double>(1.0, std::min<double>({t, (double)n->inst_N[b], (double)Tcap}));
        }
        return Tb;
    };
    auto tiles_of = [&](const std::vector<int32_t>& Tb) {
        int64_t t = 0;
        for (int b = 0; b < n->n_inst; ++b) t += (n->inst_N[b] + Tb[b] - 1) / Tb[b];
        return t;
    };
    auto ntb_max_of = [&](const std::vector<int32_t>& Tb) {
        int m = 1;
        for (int b = 0; b < n->n_inst; ++b) m = std::max<int>(m, (int)((n->inst_N[b] + Tb[b] - 1) / Tb[b]));
        return m;
    };
    auto lds_for = [&](int T, int ntbm, int per_cu, int* chunk) {
        for (int c = 1024; c >= 128; c /= 2) {
            const size_t l = step_lds_bytes(n->R, T, n->W, ntbm, c, n->ring_bytes);
            if (l * per_cu <= lds_cu) { *chunk = c; return l; }
        }
        *chunk = 128;
        return step_lds_bytes(n->R, T, n->W, ntbm, 128, n->ring_bytes);
    };
    std::vector<int32_t> Tb;
    int BS = n->spec.block_size;
    int chunk = 1024;
    if (n->spec.tile_size > 0) {
        Tb.assign(n->n_inst, n->spec.tile_size);
        const int T = n->spec.tile_size;
        if (BS == 0) BS = T > 2048 ? 512 : 1024;
        lds_for(T, ntb_max_of(Tb), 1, &chunk);
    } else {
        bool found = false;
        const int w_bytes = (n->spec.weight_dtype == CORTEX_W_BF16) ? 2 : 4;
        const int pc_lo = n->spec.wg_per_cu > 0 ? n->spec.wg_per_cu : 1;
        const int pc_hi = n->spec.wg_per_cu > 0 ? n->spec.wg_per_cu : 8;
        for (int per_cu = pc_lo; per_cu <= pc_hi && !found; per_cu *= 2) {
            const int64_t cap = (int64_t)n_cu * per_cu;
            const int bs_top = BS ? BS : std::min(1024, std::max(256, thr_cu / per_cu));
            for (int bs = bs_top; bs >= (BS ? BS : 256) && !found; bs /= 2) {
                int Tcap = bs <= 512 ? 4 * bs : 2 * bs;
                double hi0 = 1.0;
                for (int b = 0; b < n->n_inst; ++b) hi0 = std::max(hi0, K[b] * (double)n->inst_N[b]);
                // Balance synapses per tile (bisection on the per-tile synapse
                // budget), then cap tiles whose input rings would overflow the
                // workgroup's share of LDS and balance again.
                for (int pass = 0; pass < 4 && !found; ++pass) {
                    if (tiles_of(sizes_for(hi0, Tcap)) > cap) break;
                    double lo = 1.0, hi = hi0;
                    for (int it = 0; it < 100 && hi - lo > 0.5; ++it) {
                        const double mid = 0.5 * (lo + hi);
                        if (tiles_of(sizes_for(mid, Tcap)) <= cap) hi = mid; else lo = mid;
                    }
                    auto cand = sizes_for(hi, Tcap);
                    const int Tm = *std::max_element(cand.begin(), cand.end());
                    const int ntbm = ntb_max_of(cand);
                    int c = 1024;
                    const size_t lds = lds_for(Tm, ntbm, per_cu, &c);
                    if (lds * per_cu <= lds_cu && bs * per_cu <= thr_cu) {
                        // the variant's registers must allow per_cu resident
                        // workgroups of bs threads
                        int npt = (Tm + bs - 1) / bs;
                        if (npt == 3) npt = 4;
                        // the record width the graph build will choose
                        const int meta = (uint64_t)Tm * (uint64_t)n->R <= 65536 ? 2 : 4;
                        // four neurons per thread only in 512-thread workgroups
                        if ((npt <= 2 || (npt == 4 && bs == 512)) &&
                            occupancy(n, false, meta, w_bytes, npt, bs, lds) >= per_cu) {
                            Tb = cand;
                            BS = bs;
                            chunk = c;
                            found = true;
                        }
                        break;
                    }
                    // largest tile whose LDS fits at this occupancy
                    int tl = 1, th = Tm;
                    while (th - tl > 1) {
                        const int mid = (tl + th) / 2;
                        int cc = 128;
                        if (lds_for(mid, ntbm, per_cu, &cc) * per_cu <= lds_cu) tl = mid; else th = mid;
                    }
                    if (tl >= Tcap) break;
                    Tcap = tl;
                }
                if (BS) break;
            }
        }
        require(found, CORTEX_EUNSUPPORTED,
                "network too large for workgroup-local input rings on this device");
    }
    const int T = *std::max_element(Tb.begin(), Tb.end());
    n->NPT = (T + BS - 1) / BS;
    if (n->NPT == 3) n->NPT = 4;
    require(n->NPT <= 2 || (n->NPT == 4 && BS == 512), CORTEX_EINVAL,
            "tile_size must be at most 2 x block_size (4 x for block_size 512)");
    n->T = T;
    n->BS = BS;
    n->chunk = chunk;
    make_tiles(n, Tb);
    n->lds_bytes = step_lds_bytes(n->R, T, n->W, n->ntb_max, chunk, n->ring_bytes);
    require(n->lds_bytes <= lds_cu, CORTEX_EUNSUPPORTED, "input ring does not fit workgroup-local memory");
    // every tile's workgroup must be resident at once
    {
        const int meta = (uint64_t)T * (uint64_t)n->R <= 65536 ? 2 : 4;
        const int w_bytes = (n->spec.weight_dtype == CORTEX_W_BF16) ? 2 : 4;
        const int per_cu = occupancy(n, false, meta, w_bytes, n->NPT, BS, n->lds_bytes);
        require((int64_t)per_cu * n_cu >= n->n_tiles, CORTEX_EUNSUPPORTED,
                "not every tile's workgroup can be resident at once (" + std::to_string(n->n_tiles) +
                    " tiles, " + std::to_string(per_cu) + " per CU)");
    }
    n->xcd_map = (n->n_tiles % 8 == 0) ? 1 : 0;
}

// Streamed plan: no co-residency, so tiles are as large as one tile's ring
// and work arrays allow in the workgroup-local memory share of `wg_per_cu`
// workgroups (T a multiple of 4, so that rings move as 16-byte words).  The
// launch order of the tiles: with tiles of one size, XCD-aware (the
// workgroups the hardware places on one XCD take a contiguous run of tiles,
// whose segments of a source are adjacent in memory and share its L2);
// otherwise the largest expected synapse count first (longest-processing-
// time order for the load balance of Sec. III-A).
static void plan_stream(cortex_net* n) {
    const cortex_spec& s = n->spec;
    const size_t lds_cu = n->dd.lds_cu;
    const int per_cu = s.wg_per_cu > 0 ? s.wg_per_cu : 1;
    n->W = s.steps_per_sync > 0 ? s.steps_per_sync : std::min(n->dmin, 8);
    if (s.stdp_enable) {
        // a source spikes at most once per window, so that the plasticity
        // pass updates each synapse at most once per launch
        require(s.steps_per_sync == 0 || s.steps_per_sync <= n->k.n_ref + 1, CORTEX_EINVAL,
                "with plasticity steps_per_sync must be at most n_ref + 1");
        n->W = std::min(n->W, n->k.n_ref + 1);
    }
    n->R = n->dmax - n->dmin + n->W;
    n->H = pow2_at_least(n->dmin + 2 * n->W);
    n->ring_bytes = 4;
    // one workgroup of 1024 threads per compute unit, or several of 512
    const int BS = s.block_size ? s.block_size : (per_cu >= 2 ? 512 : 1024);
    // descriptor slots: a chunk, or 64 per wave of the wave-flattened mapping
    n->chunk = std::max(512, BS);
    int Tmax = 0;
    for (int t = 4; t <= 4096; t += 4)
        if (stream_lds_bytes(n->R, t, n->W, n->chunk) * per_cu <= lds_cu) Tmax = t;
    require(Tmax >= 4, CORTEX_EUNSUPPORTED, "delay range too long for a streamed tile's input ring");
    if (s.tile_size > 0) {
        require(((s.tile_size + 3) & ~3) <= Tmax, CORTEX_EUNSUPPORTED,
                "tile_size too large for the streamed plan's workgroup-local memory");
        Tmax = s.tile_size;
    }
    // one neuron per thread when the ring allows only a few more: a thread
    // with two neurons doubles the update's critical path
    if (s.tile_size == 0 && Tmax > BS && Tmax < 2 * BS) Tmax = BS;
    std::vector<int32_t> Tb(n->n_inst);
    for (int b = 0; b < n->n_inst; ++b) Tb[b] = (int32_t)std::min<int64_t>(Tmax, n->inst_N[b]);
    const int Tm = *std::max_element(Tb.begin(), Tb.end());
    n->T = (Tm + 3) & ~3;
    int npt = (n->T + BS - 1) / BS;
    if (npt == 3) npt = 4;
    require(npt <= 4, CORTEX_EINVAL, "tile_size must be at most 4 x block_size");
    n->BS = BS;
    n->NPT = npt;
    make_tiles(n, Tb);
    n->lds_bytes = stream_lds_bytes(n->R, n->T, n->W, n->chunk);
    require(n->lds_bytes <= lds_cu, CORTEX_EUNSUPPORTED, "streamed tile does not fit workgroup-local memory");
    const int meta = (uint64_t)n->T * (uint64_t)n->R <= 65536 ? 2 : 4;
    const int w_bytes = (s.weight_dtype == CORTEX_W_BF16) ? 2 : 4;
    require(occupancy(n, true, meta, w_bytes, n->NPT, n->BS, n->lds_bytes) >= 1, CORTEX_EUNSUPPORTED,
            "streamed kernel does not fit a compute unit with this plan");
    // launch order
    const auto K = mean_indegree(n);
    // mean segment length (synapses of one source into one tile): a few
    // synapses make one thread per segment the better mapping
    double seg = 0.0;
    for (int b = 0; b < n->n_inst; ++b) seg = std::max(seg, K[b] * (double)Tb[b] / (double)n->inst_N[b]);
    n->thread_segments = seg < 16.0 ? 1 : 0;
    // tile-major staging of each window's records (one instance, short
    // segments): capacity per tile for a window at 50 Hz by default, the
    // whole buffer within 4 GiB; a denser window delivers its excess from
    // the graph
    n->stage_cap = 0;
    if (n->thread_segments && n->n_inst == 1 && s.stage_records >= 0) {
        const uint64_t rec = (s.weight_dtype == CORTEX_W_BF16) ? 4 : 8;
        // (a multiple of 4 records, so that every tile's run starts
        // 16-byte aligned for the delivery launch's 16-byte loads)
        const uint64_t lim =
            std::min<uint64_t>((4ull << 30) / ((uint64_t)n->n_tiles * rec), 0x7FFFFFFFull) & ~3ull;
        uint64_t cap = ((uint64_t)s.stage_records + 3) & ~3ull;
        if (cap == 0) {
            const double per = K[0] * (double)Tb[0] * (double)n->W * s.dt * 1e-3 * 50.0;
            cap = std::max<uint64_t>(4096, ((uint64_t)std::ceil(per) + 63) & ~63ull);
        }
        n->stage_cap = (uint32_t)std::min(cap, lim);
        // tiles per copy work item: the records of 64 spikes into the
        // group fit the copy's workgroup-local buffer with room to spare
        n->stage_group = 16;
        while (n->stage_group > 1 &&
               64.0 * n->stage_group * seg * 1.15 > (double)gather_out_records((int)rec))
            n->stage_group /= 2;
    }
    std::vector<double> load(n->n_tiles);
    for (int t = 0; t < n->n_tiles; ++t) load[t] = K[n->tile_inst[t]] * n->tile_size[t];
    const bool uniform = *std::max_element(load.begin(), load.end()) <= 1.05 * *std::min_element(load.begin(), load.end());
    std::vector<int32_t>& order = n->order;
    order.assign(n->n_tiles, 0);
    if (uniform) {
        const int n8 = n->n_tiles / 8, rem = n->n_tiles % 8;
        for (int bid = 0; bid < n->n_tiles; ++bid) {
            const int x = bid % 8, r = bid / 8;
            order[bid] = x * n8 + std::min(x, rem) + r;
        }
    } else {
        for (int t = 0; t < n->n_tiles; ++t) order[t] = t;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load[a] > load[b]; });
    }
    n->xcd_map = 0;
}

static bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

// Every index the step kernels derive from a plan stays inside the array it
// addresses: the LDS carve-up (step_lds_bytes / stream_lds_bytes, in the
// kernels' order) fits the device, neurons fit the threads, record fields
// fit their width, the spike windows fit the per-step arrays and the
// publication / spike-list slots outlive every reader.  Returns what is
// violated ("" if nothing).
static std::string plan_violation(const cortex_net* n) {
    std::string v;
    auto need = [&](bool ok, const char* what) {
        if (!ok) v += std::string(v.empty() ? "" : "; ") + what;
    };
    const bool streamed = n->plan_kind == CORTEX_PLAN_STREAMED;
    need(n->BS == 256 || n->BS == 512 || n->BS == 1024, "block size");
    need(n->NPT == 1 || n->NPT == 2 || n->NPT == 4, "neurons per thread");
    need((int64_t)n->NPT * n->BS >= n->T, "tile larger than its threads' neurons");
    need(streamed || n->NPT != 4 || n->BS == 512, "four neurons per thread outside 512-thread workgroups");
    need(n->W >= 1 && n->W <= 8 && n->W <= n->dmin, "steps per exchange");
    need(n->R == n->dmax - n->dmin + n->W, "ring slots");
    need((uint64_t)n->R * (uint64_t)n->T <= 0xFFFFFFFFull, "record width");
    need(n->spec.weight_dtype != CORTEX_W_BF16 || (uint64_t)n->R * n->T <= 65536, "packed bf16 records");
    need(is_pow2(n->H) && n->H >= (streamed ? n->dmin + 2 * n->W : 2 * n->dmin + 2 * n->W + 2), "history slots");
    need(n->BS / 64 + 1 <= 20, "per-wave arrays");
    need(n->chunk >= 128, "chunk");
    need(n->lds_bytes <= n->dd.lds_cu, "LDS per workgroup");
    int64_t covered = 0;
    int tiles = 0;
    for (int b = 0; b < n->n_inst; ++b) {
        need(n->inst_T[b] <= n->T && n->inst_ntiles[b] <= n->ntb_max, "instance tiles");
        tiles += n->inst_ntiles[b];
    }
    need(tiles == n->n_tiles && (int)n->tile_size.size() == n->n_tiles, "tile table");
    for (int t = 0; t < n->n_tiles; ++t) {
        need(n->tile_size[t] >= 1 && n->tile_size[t] <= n->inst_T[n->tile_inst[t]], "tile size");
        need(n->tile_start[t] == covered, "tiles do not partition the neurons");
        covered += n->tile_size[t];
    }
    need(covered == n->N, "tiles do not cover the neurons");
    if (streamed) {
        need(n->T % 4 == 0 && n->T <= 65535, "streamed tile stride");
        need(n->ring_bytes == 4, "streamed ring width");
        need(n->chunk >= n->BS, "streamed descriptor slots (64 per wave)");
        need(n->lds_bytes == stream_lds_bytes(n->R, n->T, n->W, n->chunk), "streamed LDS carve-up");
        std::vector<char> seen(n->n_tiles, 0);
        bool perm = (int)n->order.size() == n->n_tiles;
        for (size_t i = 0; perm && i < n->order.size(); ++i) {
            const int t = n->order[i];
            perm = t >= 0 && t < n->n_tiles && !seen[t];
            if (perm) seen[t] = 1;
        }
        need(perm, "workgroup order is not a permutation of the tiles");
        if (n->stage_cap) {
            need(n->thread_segments && n->n_inst == 1, "staging needs one instance with short segments");
            need(n->W <= 8, "staging window");
            // a staged record's ring row relative to the window, meta + qi T,
            // stays below R T (and 2^16 with 16-bit records)
            need(n->stage_cap >= 4 && n->stage_cap < 0x80000000u && n->stage_cap % 4 == 0, "staging capacity");
            need(n->stage_group >= 1 && n->stage_group <= 16 && (n->stage_group & (n->stage_group - 1)) == 0,
                 "tiles per copy work item");
        }
    } else {
        need(n->lds_bytes == step_lds_bytes(n->R, n->T, n->W, n->ntb_max, n->chunk, n->ring_bytes),
             "resident LDS carve-up");
        need(n->ring_bytes == 8 || n->ring_bytes == 4, "ring width");
        need(!n->xcd_map || n->n_tiles % 8 == 0, "XCD map");
    }
    return v;
}

// FP32 plan: the resident persistent plan when every tile's ring fits the
// workgroup-local memory (64-bit sums first, then 32-bit, then shorter
// exchange windows), else (or when asked) the streamed plan.  Host-side
// only (no device memory); the plan is checked before it is used.
static void plan_fp32(cortex_net* n) {
    const cortex_spec& s = n->spec;
    const int dmin = n->dmin, dmax = n->dmax;
    // spikes are exchanged every W steps (W <= d_min keeps every input on
    // time); pending arrivals then span d_max - d_min + W steps
    const int W0 = s.steps_per_sync > 0 ? s.steps_per_sync : std::min(dmin, 8);
    require(W0 >= 1 && W0 <= dmin && W0 <= 8, CORTEX_EINVAL, "steps_per_sync must lie in [1, min(d_min, 8)]");
    bool planned = false;
    if (s.plan_kind != CORTEX_PLAN_STREAMED && !s.stdp_enable) {
        n->plan_kind = CORTEX_PLAN_RESIDENT;
        const int rb_min = s.model == CORTEX_MODEL_COND ? 8 : 4;   // two 32-bit channels per cell
        for (int rb = 8; rb >= rb_min && !planned; rb -= 4) {
            n->ring_bytes = rb;
            for (int W = W0;; W = std::max(1, W / 2)) {
                n->W = W;
                n->R = dmax - dmin + n->W;
                n->H = pow2_at_least(2 * dmin + 2 * n->W + 2);
                try {
                    plan_tiles(n);
                    planned = true;
                    break;
                } catch (const Error& e) {
                    const bool last = rb == rb_min && (W == 1 || s.steps_per_sync > 0);
                    if (e.status != CORTEX_EUNSUPPORTED || (last && s.plan_kind == CORTEX_PLAN_RESIDENT)) throw;
                    if (W == 1 || s.steps_per_sync > 0) break;
                }
            }
        }
    }
    if (!planned) {
        require(s.model != CORTEX_MODEL_COND, CORTEX_EUNSUPPORTED,
                "conductance synapses need the resident plan, and this network does not fit it");
        n->plan_kind = CORTEX_PLAN_STREAMED;
        require(n->ckpt == 0, CORTEX_EUNSUPPORTED, "the adjoint needs the resident plan (the network is too "
                                                     "large for workgroup-local input rings)");
        plan_stream(n);
    }
    const std::string bad = plan_violation(n);
    require(bad.empty(), CORTEX_EUNSUPPORTED, "plan check failed: " + bad);
}

static void upload_tables_fp32(cortex_net* n) {
    n->d_tile_start = dev_alloc_t<int64_t>(n, n->n_tiles);
    n->d_tile_size = dev_alloc_t<int32_t>(n, n->n_tiles);
    n->d_tile_inst = dev_alloc_t<int32_t>(n, n->n_tiles);
    n->d_inst_tile0 = dev_alloc_t<int32_t>(n, n->n_inst);
    n->d_inst_ntiles = dev_alloc_t<int32_t>(n, n->n_inst);
    n->d_inst_T = dev_alloc_t<int32_t>(n, n->n_inst);
    n->d_inst_offbase = dev_alloc_t<uint64_t>(n, n->n_inst);
    upload(n, n->d_tile_start, n->tile_start);
    upload(n, n->d_tile_size, n->tile_size);
    upload(n, n->d_tile_inst, n->tile_inst);
    upload(n, n->d_inst_tile0, n->inst_tile0);
    upload(n, n->d_inst_ntiles, n->inst_ntiles);
    upload(n, n->d_inst_T, n->inst_T);
    upload(n, n->d_inst_offbase, n->inst_offbase);
}

static void alloc_checkpoints(cortex_net* n) {
    if (n->ckpt <= 0) return;
    n->n_ckpt = (int)((n->adj_steps + n->ckpt - 1) / n->ckpt);
    const int64_t N = n->N;
    const size_t ring_n = (size_t)n->n_tiles * n->R * n->T;
    n->d_ck_U = dev_alloc_t<float>(n, (size_t)n->n_ckpt * N);
    n->d_ck_y1 = dev_alloc_t<float>(n, (size_t)n->n_ckpt * N);
    n->d_ck_y2 = dev_alloc_t<float>(n, (size_t)n->n_ckpt * N);
    n->d_ck_r = dev_alloc_t<int32_t>(n, (size_t)n->n_ckpt * N);
    n->d_ck_ring = dev_alloc_t<unsigned char>(n, (size_t)n->n_ckpt * ring_n * n->ring_bytes);
}

static void alloc_state_fp32(cortex_net* n) {
    const int64_t N = n->N;
    n->d_U = dev_alloc_t<float>(n, N);
    n->d_U0 = dev_alloc_t<float>(n, N);
    n->d_y1 = dev_alloc_t<float>(n, N);
    n->d_y2 = dev_alloc_t<float>(n, N);
    n->d_r = dev_alloc_t<int32_t>(n, N);
    n->d_ring = dev_alloc(n, (size_t)n->n_tiles * n->R * n->T * n->ring_bytes);
    if (n->plan_kind == CORTEX_PLAN_STREAMED) {
        n->d_spk_cnt = dev_alloc_t<uint32_t>(n, (size_t)n->H * n->n_inst);
        n->d_spk_ids = dev_alloc_t<uint32_t>(n, (size_t)n->H * n->N);
        n->d_clock = dev_alloc_t<int64_t>(n, 2);
        n->use_graph = true;
        n->d_kcache = dev_alloc_t<unsigned long long>(n, n->N);
        if (n->stage_cap) {
            const size_t rec = n->w_bytes == 2 ? 4 : 8;
            n->d_stage = dev_alloc(n, (size_t)n->n_tiles * n->stage_cap * rec);
            n->d_cursor = dev_alloc_t<unsigned long long>(n, n->n_tiles);
        }
        if (n->stdp) {
            n->d_seg_state = dev_alloc_t<uint64_t>(n, std::max<uint64_t>(1, n->n_seg));
            n->d_hist_step = dev_alloc_t<int32_t>(n, (size_t)n->N * kHistLen);
            n->d_hist_y = dev_alloc_t<float>(n, (size_t)n->N * kHistLen);
            n->d_hist_cnt = dev_alloc_t<uint32_t>(n, n->N);
            n->d_hist_upto = dev_alloc_t<int64_t>(n, n->n_tiles);
        }
    } else {
        // (+8 words: a reader fetches a few id words past a record without bounds checks)
        n->d_pub = dev_alloc_t<uint64_t>(n, (size_t)n->H * n->n_tiles * (n->T + 1) + 8);
    }
    n->log_steps = std::max<int64_t>(0, n->spec.record_steps);
    if (n->ckpt > 0) n->log_steps = std::max(n->log_steps, n->adj_steps);   // the adjoint replays the raster
    n->d_log_cnt = dev_alloc_t<uint32_t>(n, (size_t)std::max<int64_t>(1, n->log_steps) * n->n_tiles);
    std::vector<uint64_t> base(n->n_tiles + 1, 0);
    const int64_t per = (n->log_steps + n->k.n_ref) / (n->k.n_ref + 1);
    for (int t = 0; t < n->n_tiles; ++t) base[t + 1] = base[t] + (uint64_t)n->tile_size[t] * per;
    n->d_log_base = dev_alloc_t<uint64_t>(n, n->n_tiles + 1);
    upload(n, n->d_log_base, base);
    n->d_log_ids = dev_alloc_t<uint32_t>(n, std::max<uint64_t>(1, base.back()));
    n->d_log_pos = dev_alloc_t<uint64_t>(n, n->n_tiles);
    n->d_events = dev_alloc_t<uint64_t>(n, n->n_tiles);
    n->d_spikes = dev_alloc_t<uint64_t>(n, n->n_tiles);
    n->d_err = dev_alloc_t<int32_t>(n, 4);
}

// Forget the captured window graph (its arguments hold the log window and
// the fixed-point scale).
static void drop_graph(cortex_net* n) {
    if (n->graph_exec) {
        (void)hipStreamSynchronize(n->graph_stream);
        (void)hipGraphExecDestroy(n->graph_exec);
        n->graph_exec = nullptr;
    }
}

static void zero_dynamic_fp32(cortex_net* n) {
    const int64_t N = n->N;
    CX_HIP(hipMemcpyAsync(n->d_U, n->d_U0, N * sizeof(float), hipMemcpyDeviceToDevice, n->stream));
    dev_zero(n, n->d_y1, N * sizeof(float));
    dev_zero(n, n->d_y2, N * sizeof(float));
    dev_zero(n, n->d_r, N * sizeof(int32_t));
    dev_zero(n, n->d_ring, (size_t)n->n_tiles * n->R * n->T * n->ring_bytes);
    if (n->plan_kind == CORTEX_PLAN_STREAMED) {
        dev_zero(n, n->d_spk_cnt, (size_t)n->H * n->n_inst * sizeof(uint32_t));
        dev_zero(n, n->d_clock, 2 * sizeof(int64_t));
        if (n->stage_cap) dev_zero(n, n->d_cursor, (size_t)n->n_tiles * sizeof(unsigned long long));
        dev_zero(n, n->d_kcache, (size_t)n->N * sizeof(unsigned long long));
        n->clock_parity = 0;
        drop_graph(n);
        if (n->stdp) {   // traces and histories restart; the weights stay
            dev_zero(n, n->d_seg_state, std::max<uint64_t>(1, n->n_seg) * sizeof(uint64_t));
            dev_zero(n, n->d_hist_cnt, (size_t)n->N * sizeof(uint32_t));
            dev_zero(n, n->d_hist_upto, (size_t)n->n_tiles * sizeof(int64_t));
        }
    } else {
        dev_zero(n, n->d_pub, (size_t)n->H * n->n_tiles * (n->T + 1) * sizeof(uint64_t));
    }
    dev_zero(n, n->d_log_pos, n->n_tiles * sizeof(uint64_t));
    dev_zero(n, n->d_log_cnt, (size_t)std::max<int64_t>(1, n->log_steps) * n->n_tiles * sizeof(uint32_t));
    dev_zero(n, n->d_events, n->n_tiles * sizeof(uint64_t));
    dev_zero(n, n->d_spikes, n->n_tiles * sizeof(uint64_t));
    dev_zero(n, n->d_err, 4 * sizeof(int32_t));
}

static void alloc_state_fp64(cortex_net* n) {
    const int64_t N = n->N;
    n->W64 = (N + 63) / 64;
    n->H = pow2_at_least(n->dmax + 1);
    n->d_Ud = dev_alloc_t<double>(n, N);
    n->d_Ud0 = dev_alloc_t<double>(n, N);
    n->d_y1d = dev_alloc_t<double>(n, N);
    n->d_y2d = dev_alloc_t<double>(n, N);
    n->d_r = dev_alloc_t<int32_t>(n, N);
    n->d_hist = dev_alloc_t<uint64_t>(n, (size_t)n->H * n->W64);
    n->log_steps = std::max<int64_t>(0, n->spec.record_steps);
    n->d_raster = dev_alloc_t<uint64_t>(n, (size_t)std::max<int64_t>(1, n->log_steps) * n->W64);
    n->d_events = dev_alloc_t<uint64_t>(n, 2);   // synaptic events, spikes
    n->d_err = dev_alloc_t<int32_t>(n, 4);
}

static void zero_dynamic_fp64(cortex_net* n) {
    const int64_t N = n->N;
    CX_HIP(hipMemcpyAsync(n->d_Ud, n->d_Ud0, N * sizeof(double), hipMemcpyDeviceToDevice, n->stream));
    dev_zero(n, n->d_y1d, N * sizeof(double));
    dev_zero(n, n->d_y2d, N * sizeof(double));
    dev_zero(n, n->d_r, N * sizeof(int32_t));
    dev_zero(n, n->d_hist, (size_t)n->H * n->W64 * sizeof(uint64_t));
    dev_zero(n, n->d_raster, (size_t)std::max<int64_t>(1, n->log_steps) * n->W64 * sizeof(uint64_t));
    dev_zero(n, n->d_events, 2 * sizeof(uint64_t));
    dev_zero(n, n->d_err, 4 * sizeof(int32_t));
}

// Device error flag raised by a kernel (a wait that exceeded its limit).
void check_device_flag(cortex_net* n) {
    CX_HIP(hipStreamSynchronize(n->stream));
    int32_t e[2] = {0, 0};
    CX_HIP(hipMemcpy(e, n->d_err, sizeof e, hipMemcpyDeviceToHost));
    if (e[0] != 0) {
        n->failed = true;
        throw Error{CORTEX_ETIMEOUT, "a device-side wait exceeded its spin limit; network state is invalid"};
    }
    if (e[1] != 0) {
        n->failed = true;
        throw Error{CORTEX_ETRUNC, "a plastic synapse needed a postsynaptic spike older than the 32 a neuron "
                                   "keeps; weights are invalid"};
    }
}

static void build(cortex_net* n) {
    const cortex_spec& s = n->spec;
    n->k = model_constants(s);
    n->n_thr = poisson_thresholds(s.poisson_lambda, n->thr, 64);
    require(n->n_thr >= 0, CORTEX_EINVAL, "Poisson table too long");
    n->w_ext_native = (s.weight_unit == CORTEX_UNIT_PSP_MV && n->k.conv != 1.0) ? s.w_ext * n->k.conv : s.w_ext;
    if (s.stdp_enable && s.precision == CORTEX_FP32) {
        const double cw = (s.weight_unit == CORTEX_UNIT_PSP_MV && n->k.conv != 1.0) ? n->k.conv : 1.0;
        int64_t off = 0;
        for (int p = 0; p < s.stdp_pop; ++p) off += n->pops[p].size;
        n->stdp = true;
        n->stdp_lo = off;
        n->stdp_hi = off + n->pops[s.stdp_pop].size;
        n->stdp_c = s.stdp_lambda * std::pow(s.stdp_w0 * cw, 1.0 - s.stdp_mu);
        n->stdp_lam_alpha = s.stdp_lambda * s.stdp_alpha;
        n->stdp_mu = s.stdp_mu;
        n->stdp_tp = s.stdp_tau_plus;
        n->stdp_tm = s.stdp_tau_minus;
        n->stdp_wmax = s.stdp_wmax * cw;
    }
    make_blocks(n);
    n->d_inst_n0 = dev_alloc_t<int64_t>(n, n->n_inst);
    upload(n, n->d_inst_n0, n->inst_n0);
    n->ckpt = s.precision == CORTEX_FP64_VERIFY ? 0 : s.ckpt_every;
    n->adj_steps = s.adjoint_steps;
    require(n->ckpt == 0 || n->adj_steps >= 1, CORTEX_EINVAL, "adjoint_steps must be >= 1 with ckpt_every > 0");
    if (s.precision == CORTEX_FP64_VERIFY) {
        build_graph_fp64(n);
        alloc_state_fp64(n);
        zero_dynamic_fp64(n);
        init_state(n);
        zero_dynamic_fp64(n);   // copies U0 into U after init
    } else {
        int dmin = 1, dmax = 1;
        if (!host_delay_range(n, &dmin, &dmax)) delay_range(n, &dmin, &dmax);
        n->dmin = dmin;
        n->dmax = dmax;
        plan_fp32(n);
        if (n->plan_kind == CORTEX_PLAN_STREAMED) {
            n->d_order = dev_alloc_t<int32_t>(n, n->n_tiles);
            upload(n, n->d_order, n->order);
        }
        n->fx = fixed_point_bits(n);
        n->fx_shift = fixed_point_shift(n, n->fx);
        upload_tables_fp32(n);
        build_graph_fp32(n);
        if (n->ring_bytes == 4 || s.model == CORTEX_MODEL_COND) {
            // (conductances: each 32-bit half of a cell holds one channel's sum)
            const double bound = max_abs_input(n) * (1.0 + 1e-4) + 1e-30;
            n->fx = std::max(0, std::min(52, 30 - (int)std::ceil(std::log2(bound))));
            n->fx_shift = 0;
        }
        alloc_state_fp32(n);
        alloc_checkpoints(n);
        init_state(n);
        zero_dynamic_fp32(n);
        save_checkpoint(n, 0);
        if (n->plan_kind == CORTEX_PLAN_RESIDENT) {
            const int per_cu = step_max_blocks_per_cu(n);
            require((int64_t)per_cu * n->dd.n_cu >= n->n_tiles, CORTEX_EUNSUPPORTED,
                    "not every tile's workgroup can be resident at once (" + std::to_string(n->n_tiles) +
                        " tiles, " + std::to_string(per_cu) + " per CU)");
        }
    }
    n->step = 0;
    n->log_step0 = 0;
    free_scratch(n);
    CX_HIP(hipStreamSynchronize(n->stream));
}

// Per-(step, tile) lists of a frozen raster for the FP32 kernel: spikes with
// step in [step0, step0 + n_steps), sorted by (step, id).
void frozen_lists_at(cortex_net* n, int64_t step0, const std::vector<std::pair<uint32_t, uint32_t>>& spikes,
                     int64_t n_steps, std::vector<uint32_t>& ids, std::vector<uint64_t>& ptr) {
    ptr.assign((size_t)n_steps * n->n_tiles + 1, 0);
    ids.clear();
    size_t q = 0;
    const size_t ns = spikes.size();
    for (int64_t s = 0; s < n_steps; ++s) {
        const int64_t step = step0 + s;
        while (q < ns && (int64_t)spikes[q].first < step) ++q;
        for (int t = 0; t < n->n_tiles; ++t) {
            ptr[(size_t)s * n->n_tiles + t] = ids.size();
            const int64_t t0 = n->tile_start[t], t1 = t0 + n->tile_size[t];
            while (q < ns && (int64_t)spikes[q].first == step && (int64_t)spikes[q].second < t1) {
                require((int64_t)spikes[q].second >= t0, CORTEX_EINVAL, "raster not sorted by (step, id)");
                ids.push_back(spikes[q].second);
                ++q;
            }
        }
    }
    ptr[(size_t)n_steps * n->n_tiles] = ids.size();
}

// Spikes with step in [s0, s1) from the log, sorted by (step, id).
std::vector<std::pair<uint32_t, uint32_t>> collect_spikes(cortex_net* n, int64_t step0, int64_t step1,
                                                          bool* trunc) {
    const int64_t w0 = n->log_step0, w1 = std::min(n->log_step0 + n->log_steps, n->step);
    *trunc = step0 < w0 || step1 > w1;
    const int64_t s0 = std::max(step0, w0), s1 = std::min(step1, w1);
    std::vector<std::pair<uint32_t, uint32_t>> out;
    if (s1 <= s0) return out;
    if (n->spec.precision == CORTEX_FP64_VERIFY) {
        auto bits = download(n, n->d_raster + (size_t)(s0 - w0) * n->W64, (size_t)(s1 - s0) * n->W64);
        for (int64_t s = s0; s < s1; ++s)
            for (int64_t w = 0; w < n->W64; ++w) {
                uint64_t x = bits[(size_t)(s - s0) * n->W64 + w];
                while (x) {
                    const int b = __builtin_ctzll(x);
                    out.emplace_back((uint32_t)s, (uint32_t)(w * 64 + b));
                    x &= x - 1;
                }
            }
        return out;
    }
    auto cnt = download(n, n->d_log_cnt, (size_t)(s1 - w0) * n->n_tiles);
    auto pos = download(n, n->d_log_pos, n->n_tiles);
    auto base = download(n, n->d_log_base, n->n_tiles + 1);
    std::vector<std::vector<uint32_t>> tid(n->n_tiles);
    for (int t = 0; t < n->n_tiles; ++t) tid[t] = download(n, n->d_log_ids + base[t], (size_t)pos[t]);
    // Each tile's log lists its spikes step by step; tiles hold increasing
    // id ranges, so walking the steps and, within a step, the tiles in
    // order, with each (step, tile) group sorted, yields (step, id) order.
    // A tile's log ends at its first overflow mark.
    std::vector<uint64_t> p(n->n_tiles, 0);
    std::vector<char> ended(n->n_tiles, 0);
    for (int64_t s = w0; s < s1; ++s) {
        for (int t = 0; t < n->n_tiles; ++t) {
            if (ended[t]) continue;
            const uint32_t c = cnt[(size_t)(s - w0) * n->n_tiles + t];
            if (c == 0xFFFFFFFFu || p[t] + c > tid[t].size()) {
                *trunc = true;
                ended[t] = 1;
                continue;
            }
            if (s >= s0) {
                const size_t o = out.size();
                for (uint32_t k = 0; k < c; ++k) out.emplace_back((uint32_t)s, tid[t][p[t] + k]);
                std::sort(out.begin() + o, out.end());
            }
            p[t] += c;
        }
    }
    return out;
}

// Adjoint checkpoints: neuron state and input rings at steps k * ckpt.
static void save_checkpoint(cortex_net* n, int k) {
    if (k < 0 || k >= n->n_ckpt) return;
    const int64_t N = n->N;
    const size_t ring_n = (size_t)n->n_tiles * n->R * n->T;
    auto d2d = [&](void* dst, const void* src, size_t bytes) {
        CX_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, n->stream));
    };
    d2d(n->d_ck_U + (size_t)k * N, n->d_U, N * 4);
    d2d(n->d_ck_y1 + (size_t)k * N, n->d_y1, N * 4);
    d2d(n->d_ck_y2 + (size_t)k * N, n->d_y2, N * 4);
    d2d(n->d_ck_r + (size_t)k * N, n->d_r, N * 4);
    d2d(n->d_ck_ring + (size_t)k * ring_n * n->ring_bytes, n->d_ring, ring_n * n->ring_bytes);
}

void restore_checkpoint(cortex_net* n, int k) {
    const int64_t N = n->N;
    const size_t ring_n = (size_t)n->n_tiles * n->R * n->T;
    auto d2d = [&](void* dst, const void* src, size_t bytes) {
        CX_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, n->stream));
    };
    d2d(n->d_U, n->d_ck_U + (size_t)k * N, N * 4);
    d2d(n->d_y1, n->d_ck_y1 + (size_t)k * N, N * 4);
    d2d(n->d_y2, n->d_ck_y2 + (size_t)k * N, N * 4);
    d2d(n->d_r, n->d_ck_r + (size_t)k * N, N * 4);
    d2d(n->d_ring, n->d_ck_ring + (size_t)k * ring_n * n->ring_bytes, ring_n * n->ring_bytes);
}

// Advance the FP32 network, splitting launches at checkpoint steps when the
// adjoint is enabled.  Frozen lists and traces are indexed from the call's
// first step.
void advance_fp32(cortex_net* n, int64_t n_steps, const uint32_t* frz_ids, const uint64_t* frz_ptr,
                  uint64_t frz_n, float* x_trace, float* v_trace) {
    if (n->plan_kind == CORTEX_PLAN_STREAMED) {
        launch_stream_fp32(n, n_steps, frz_ids, frz_ptr, frz_n, x_trace, v_trace);
        return;
    }
    const int64_t first = n->step;
    int64_t left = n_steps;
    while (left > 0) {
        int64_t chunk = left;
        if (n->ckpt > 0) chunk = std::min<int64_t>(left, (n->step / n->ckpt + 1) * n->ckpt - n->step);
        const int64_t off = n->step - first;
        launch_step_fp32(n, chunk, frz_ids, frz_ptr ? frz_ptr + off * n->n_tiles : nullptr, frz_n,
                         x_trace ? x_trace + off * n->N : nullptr, v_trace ? v_trace + off * n->N : nullptr);
        left -= chunk;
        if (n->ckpt > 0 && n->step % n->ckpt == 0) save_checkpoint(n, (int)(n->step / n->ckpt));
    }
}

}  // namespace cortex

using namespace cortex;

#define CX_API_BEGIN try {
#define CX_API_END                                           \
    }                                                        \
    catch (const ::cortex::Error& e) {                       \
        set_error(e.msg);                                    \
        return e.status;                                     \
    }                                                        \
    catch (const std::bad_alloc&) {                          \
        set_error("host allocation failed");                 \
        return CORTEX_ENOMEM;                                \
    }                                                        \
    catch (...) {                                            \
        set_error("unexpected internal error");              \
        return CORTEX_EDEVICE;                               \
    }

// A frozen raster given to a plastic network keeps the refractory period of
// the plastic neurons (consecutive spikes at least n_ref + 1 steps apart),
// as closed-loop spikes do: then no source spikes twice in one window, and
// the plasticity pass updates each synapse at most once per launch.
void cortex::check_plastic_raster(const cortex_net* n, const uint32_t* st, const uint32_t* id, int64_t ns) {
    if (!n->stdp) return;
    std::unordered_map<uint32_t, uint32_t> last;
    for (int64_t q = 0; q < ns; ++q) {
        if ((int64_t)id[q] < n->stdp_lo || (int64_t)id[q] >= n->stdp_hi) continue;
        auto it = last.find(id[q]);
        if (it != last.end())
            require((int64_t)st[q] - (int64_t)it->second >= (int64_t)n->k.n_ref + 1, CORTEX_EINVAL,
                    "a plastic neuron spikes twice within its refractory period in the raster");
        last[id[q]] = st[q];
    }
}

static void require_net(cortex_net* n) {
    require(n != nullptr, CORTEX_EINVAL, "network handle is NULL");
    require(!n->failed, CORTEX_ESTATE, "network failed earlier; destroy it");
}

// The dynamic state of a network, part by part (device buffers), for
// cortex_save_state / cortex_load_state: everything a step reads and writes
// besides the immutable graph.  The staging cursors are zero between
// windows and the staged runs are rebuilt by every window, so neither is
// part of it.
struct StatePart {
    void* p;
    size_t bytes;
};

static std::vector<StatePart> state_parts(cortex_net* n) {
    const size_t N = (size_t)n->N, nt = (size_t)n->n_tiles;
    if (n->spec.precision == CORTEX_FP64_VERIFY) {
        // FP64 verify mode: the state, the spike bits of the last H steps
        // (the pending deliveries) and of the record window, the counters
        return {{n->d_Ud, N * sizeof(double)},
                {n->d_y1d, N * sizeof(double)},
                {n->d_y2d, N * sizeof(double)},
                {n->d_r, N * sizeof(int32_t)},
                {n->d_hist, (size_t)n->H * n->W64 * sizeof(uint64_t)},
                {n->d_raster, (size_t)std::max<int64_t>(1, n->log_steps) * n->W64 * sizeof(uint64_t)},
                {n->d_events, 2 * sizeof(uint64_t)},
                {n->d_err, 4 * sizeof(int32_t)}};
    }
    std::vector<StatePart> v{{n->d_U, N * sizeof(float)},
                             {n->d_y1, N * sizeof(float)},
                             {n->d_y2, N * sizeof(float)},
                             {n->d_r, N * sizeof(int32_t)},
                             {n->d_ring, nt * n->R * n->T * n->ring_bytes}};
    if (n->plan_kind == CORTEX_PLAN_STREAMED) {
        v.push_back({n->d_spk_cnt, (size_t)n->H * n->n_inst * sizeof(uint32_t)});
        v.push_back({n->d_spk_ids, (size_t)n->H * N * sizeof(uint32_t)});
        v.push_back({n->d_clock, 2 * sizeof(int64_t)});
        v.push_back({n->d_kcache, N * sizeof(unsigned long long)});
        if (n->stdp) {
            v.push_back({n->d_seg_state, std::max<uint64_t>(1, n->n_seg) * sizeof(uint64_t)});
            v.push_back({n->d_hist_step, N * kHistLen * sizeof(int32_t)});
            v.push_back({n->d_hist_y, N * kHistLen * sizeof(float)});
            v.push_back({n->d_hist_cnt, N * sizeof(uint32_t)});
            v.push_back({n->d_hist_upto, nt * sizeof(int64_t)});
            // plastic weights, with their records: the order of the synapses
            // inside a segment is not the same in every build, so the
            // weights are restored only together with the records they
            // belong to
            v.push_back({n->d_meta, (size_t)n->E * n->meta_bytes});
            v.push_back({n->d_w, (size_t)n->E * n->w_bytes});
        }
    } else {
        v.push_back({n->d_pub, (size_t)n->H * nt * (n->T + 1) * sizeof(uint64_t)});
    }
    const int64_t per = (n->log_steps + n->k.n_ref) / (n->k.n_ref + 1);
    uint64_t log_ids = 0;
    for (int t = 0; t < n->n_tiles; ++t) log_ids += (uint64_t)n->tile_size[t] * per;
    v.push_back({n->d_log_cnt, (size_t)std::max<int64_t>(1, n->log_steps) * nt * sizeof(uint32_t)});
    v.push_back({n->d_log_ids, std::max<uint64_t>(1, log_ids) * sizeof(uint32_t)});
    v.push_back({n->d_log_pos, nt * sizeof(uint64_t)});
    v.push_back({n->d_events, nt * sizeof(uint64_t)});
    v.push_back({n->d_spikes, nt * sizeof(uint64_t)});
    v.push_back({n->d_err, 4 * sizeof(int32_t)});
    return v;
}

// Header of a saved state: what identifies the network and its plan, and
// the host side of the state.
struct StateHeader {
    uint64_t magic;
    int64_t N, E, step, log_step0, log_steps, bytes;
    int32_t n_tiles, T, R, H, W, ring_bytes, plan_kind, stdp, clock_parity, n_parts;
    uint64_t seed;
};
constexpr uint64_t kStateMagic = 0x31455441545358ull;   // "XSTATE1"

static void state_supported(cortex_net* n) {
    require(n->ckpt == 0, CORTEX_EUNSUPPORTED, "saved states exclude networks with the adjoint enabled");
}

static StateHeader state_header(cortex_net* n, const std::vector<StatePart>& parts) {
    StateHeader h{};
    h.magic = kStateMagic;
    h.N = n->N;
    h.E = n->E;
    h.step = n->step;
    h.log_step0 = n->log_step0;
    h.log_steps = n->log_steps;
    h.n_tiles = n->n_tiles;
    h.T = n->T;
    h.R = n->R;
    h.H = n->H;
    h.W = n->W;
    h.ring_bytes = n->ring_bytes;
    h.plan_kind = n->plan_kind;
    h.stdp = n->stdp ? 1 : 0;
    h.clock_parity = n->clock_parity;
    h.n_parts = (int32_t)parts.size();
    h.seed = n->seed;
    int64_t b = sizeof(StateHeader);
    for (const auto& p : parts) b += (int64_t)p.bytes;
    h.bytes = b;
    return h;
}

extern "C" {

const char* cortex_last_error(void) { return g_error.c_str(); }

int cortex_build_network(const cortex_spec* spec, uint64_t seed, const cortex_device* dev, cortex_net** out) {
    cortex_net* n = nullptr;
    try {
        require(out != nullptr, CORTEX_EINVAL, "out is NULL");
        *out = nullptr;
        validate(spec);
        n = new cortex_net();
        n->spec = *spec;
        n->pops.assign(spec->pops, spec->pops + spec->n_pops);
        n->projs.assign(spec->projs, spec->projs + spec->n_projs);
        n->spec.pops = nullptr;
        n->spec.projs = nullptr;
        if (dev) n->dev = *dev;
        n->stream = static_cast<hipStream_t>(n->dev.stream);
        CX_HIP(hipGetDevice(&n->device));
        hipDeviceProp_t prop;
        CX_HIP(hipGetDeviceProperties(&prop, n->device));
        n->dd.n_cu = prop.multiProcessorCount;
        n->dd.lds_cu = prop.maxSharedMemoryPerMultiProcessor ? prop.maxSharedMemoryPerMultiProcessor : 65536;
        n->dd.thr_cu = prop.maxThreadsPerMultiProcessor ? prop.maxThreadsPerMultiProcessor : 2048;
        n->dd.live = true;
        n->seed = seed;
        build(n);
        *out = n;
        return CORTEX_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        if (n) cortex_destroy(n);
        return e.status;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        if (n) cortex_destroy(n);
        return CORTEX_ENOMEM;
    }
}

int cortex_plan(const cortex_spec* spec, int32_t n_cu, int64_t lds_per_cu, int32_t threads_per_cu,
                int64_t* plan, int32_t n_plan) {
    cortex_net* n = nullptr;
    try {
        require(plan != nullptr && n_plan >= 0, CORTEX_EINVAL, "plan is NULL");
        require(n_cu >= 1 && lds_per_cu >= 1024 && threads_per_cu >= 256, CORTEX_EINVAL, "bad device description");
        validate(spec);
        require(spec->precision == CORTEX_FP32, CORTEX_EINVAL, "plans are made for FP32 networks");
        n = new cortex_net();
        n->spec = *spec;
        n->pops.assign(spec->pops, spec->pops + spec->n_pops);
        n->projs.assign(spec->projs, spec->projs + spec->n_projs);
        n->spec.pops = nullptr;
        n->spec.projs = nullptr;
        n->dd.n_cu = n_cu;
        n->dd.lds_cu = (size_t)lds_per_cu;
        n->dd.thr_cu = threads_per_cu;
        n->dd.live = false;
        n->ckpt = spec->ckpt_every;
        n->k = model_constants(n->spec);
        make_blocks(n);
        host_delay_range(n, &n->dmin, &n->dmax, true);
        plan_fp32(n);
        const int64_t out[] = {n->plan_kind, n->n_tiles, n->T, n->BS, n->NPT, n->W, n->R, n->H, n->chunk,
                               n->ntb_max, (int64_t)n->lds_bytes, n->ring_bytes, n->dmin, n->dmax, n->xcd_map,
                               n->thread_segments, (int64_t)n->stage_cap};
        for (int i = 0; i < n_plan && i < (int)(sizeof out / sizeof out[0]); ++i) plan[i] = out[i];
        delete n;
        return CORTEX_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        delete n;
        return e.status;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        delete n;
        return CORTEX_ENOMEM;
    }
}

int cortex_step(cortex_net* n, int64_t n_steps) {
    CX_API_BEGIN
    require_net(n);
    require(n_steps >= 0, CORTEX_EINVAL, "n_steps must be >= 0");
    if (n->spec.precision == CORTEX_FP64_VERIFY) launch_step_fp64(n, n_steps, nullptr, nullptr, nullptr);
    else advance_fp32(n, n_steps, nullptr, nullptr, 0, nullptr, nullptr);
    return CORTEX_OK;
    CX_API_END
}

int cortex_get_spikes(cortex_net* n, int64_t step0, int64_t step1, uint32_t* steps, uint32_t* ids,
                      int64_t capacity, int64_t* count) {
    CX_API_BEGIN
    require_net(n);
    require(count != nullptr && capacity >= 0 && (capacity == 0 || (steps && ids)), CORTEX_EINVAL,
            "bad output buffers");
    check_device_flag(n);
    bool trunc = false;
    const auto out = collect_spikes(n, step0, step1, &trunc);
    *count = (int64_t)out.size();
    const int64_t m = std::min<int64_t>(capacity, (int64_t)out.size());
    for (int64_t i = 0; i < m; ++i) {
        steps[i] = out[i].first;
        ids[i] = out[i].second;
    }
    if (m < (int64_t)out.size()) trunc = true;
    if (trunc) {
        set_error("spike range truncated (capacity or record window)");
        return CORTEX_ETRUNC;
    }
    return CORTEX_OK;
    CX_API_END
}

int cortex_clear_spikes(cortex_net* n) {
    CX_API_BEGIN
    require_net(n);
    n->log_step0 = n->step;
    if (n->spec.precision != CORTEX_FP64_VERIFY) dev_zero(n, n->d_log_pos, n->n_tiles * sizeof(uint64_t));
    CX_HIP(hipStreamSynchronize(n->stream));
    return CORTEX_OK;
    CX_API_END
}

int cortex_run_frozen(cortex_net* n, const uint32_t* r_steps, const uint32_t* r_ids, int64_t n_spikes,
                      int64_t n_steps, void* x_trace, void* v_trace) {
    CX_API_BEGIN
    require_net(n);
    require(n_steps >= 0 && n_spikes >= 0 && (n_spikes == 0 || (r_steps && r_ids)), CORTEX_EINVAL,
            "bad raster");
    require((x_trace == nullptr) == (v_trace == nullptr), CORTEX_EINVAL, "pass both traces or neither");
    for (int64_t q = 0; q < n_spikes; ++q) {
        require(r_ids[q] < n->N, CORTEX_EINVAL, "raster id out of range");
        require(q == 0 || r_steps[q] > r_steps[q - 1] || (r_steps[q] == r_steps[q - 1] && r_ids[q] > r_ids[q - 1]),
                CORTEX_EINVAL, "raster must be sorted by (step, id) without duplicates");
    }
    if (n_steps == 0) return CORTEX_OK;
    check_plastic_raster(n, r_steps, r_ids, n_spikes);
    if (n->spec.precision == CORTEX_FP64_VERIFY) {
        std::vector<uint64_t> bits((size_t)n_steps * n->W64, 0);
        for (int64_t q = 0; q < n_spikes; ++q) {
            const int64_t s = (int64_t)r_steps[q] - n->step;
            if (s < 0 || s >= n_steps) continue;
            bits[(size_t)s * n->W64 + (r_ids[q] >> 6)] |= 1ull << (r_ids[q] & 63);
        }
        uint64_t* d_bits = dev_alloc_t<uint64_t>(n, bits.size(), true);
        upload(n, d_bits, bits);
        launch_step_fp64(n, n_steps, d_bits, static_cast<double*>(x_trace), static_cast<double*>(v_trace));
    } else {
        std::vector<uint32_t> ids;
        std::vector<uint64_t> ptr;
        std::vector<std::pair<uint32_t, uint32_t>> spikes((size_t)n_spikes);
        for (int64_t q = 0; q < n_spikes; ++q) spikes[q] = {r_steps[q], r_ids[q]};
        frozen_lists_at(n, n->step, spikes, n_steps, ids, ptr);
        uint32_t* d_ids = dev_alloc_t<uint32_t>(n, std::max<size_t>(1, ids.size()), true);
        uint64_t* d_ptr = dev_alloc_t<uint64_t>(n, ptr.size(), true);
        upload(n, d_ids, ids);
        upload(n, d_ptr, ptr);
        advance_fp32(n, n_steps, d_ids, d_ptr, ids.size(), static_cast<float*>(x_trace),
                     static_cast<float*>(v_trace));
    }
    check_device_flag(n);
    free_scratch(n);
    return CORTEX_OK;
    CX_API_END
}

int cortex_backward(cortex_net* n, const float* vstar, float* grad_w, double* loss) {
    CX_API_BEGIN
    require_net(n);
    require(n->spec.precision != CORTEX_FP64_VERIFY, CORTEX_EUNSUPPORTED, "the adjoint runs in FP32 mode");
    require(n->ckpt > 0 && n->plan_kind == CORTEX_PLAN_RESIDENT, CORTEX_ESTATE,
            "adjoint not enabled (ckpt_every = 0 at build)");
    require(vstar != nullptr && grad_w != nullptr && loss != nullptr, CORTEX_EINVAL,
            "vstar, grad_w and loss must not be NULL");
    check_device_flag(n);
    adjoint_backward(n, vstar, grad_w, loss);
    free_scratch(n);
    return CORTEX_OK;
    CX_API_END
}

int cortex_set_weights(cortex_net* n, const float* w_canonical) {
    CX_API_BEGIN
    require_net(n);
    require(w_canonical != nullptr, CORTEX_EINVAL, "w_canonical is NULL");
    require(n->spec.precision != CORTEX_FP64_VERIFY, CORTEX_EUNSUPPORTED, "weights are set in FP32 mode");
    require(n->d_canon != nullptr, CORTEX_ESTATE, "setting weights needs ckpt_every > 0 (canonical order)");
    require(n->step == 0, CORTEX_ESTATE, "weights are set at step 0 (after the build or cortex_reset)");
    check_device_flag(n);
    drop_graph(n);
    set_weights_fp32(n, w_canonical);
    // fixed-point scale from the exact bound of the new weights
    double wmax = 0.0;
    const double bound = max_abs_input(n, &wmax) * (1.0 + 1e-4) + 1e-30;
    const int lg = (int)std::ceil(std::log2(bound));
    if (n->ring_bytes == 8) {
        n->fx = std::max(0, std::min(52, 61 - lg));
        const int fxw = 30 - (int)std::ceil(std::log2(wmax * (1.0 + 1e-6) + 1e-30));
        n->fx_shift = std::max(0, n->fx - std::max(0, fxw));
    } else {
        n->fx = std::max(0, std::min(52, 30 - lg));
        n->fx_shift = 0;
    }
    free_scratch(n);
    return CORTEX_OK;
    CX_API_END
}

int cortex_reset(cortex_net* n) {
    CX_API_BEGIN
    require_net(n);
    if (n->spec.precision == CORTEX_FP64_VERIFY) zero_dynamic_fp64(n);
    else zero_dynamic_fp32(n);
    n->step = 0;
    n->log_step0 = 0;
    CX_HIP(hipStreamSynchronize(n->stream));
    return CORTEX_OK;
    CX_API_END
}

int cortex_state_size(cortex_net* n, int64_t* bytes) {
    CX_API_BEGIN
    require_net(n);
    require(bytes != nullptr, CORTEX_EINVAL, "bytes is NULL");
    state_supported(n);
    const auto parts = state_parts(n);
    *bytes = state_header(n, parts).bytes;
    return CORTEX_OK;
    CX_API_END
}

int cortex_save_state(cortex_net* n, void* host, int64_t bytes) {
    CX_API_BEGIN
    require_net(n);
    require(host != nullptr, CORTEX_EINVAL, "host buffer is NULL");
    state_supported(n);
    check_device_flag(n);
    const auto parts = state_parts(n);
    const StateHeader h = state_header(n, parts);
    require(bytes >= h.bytes, CORTEX_EINVAL, "host buffer smaller than the state");
    CX_HIP(hipStreamSynchronize(n->stream));
    unsigned char* out = static_cast<unsigned char*>(host);
    std::memcpy(out, &h, sizeof h);
    size_t at = sizeof h;
    for (const auto& p : parts) {
        CX_HIP(hipMemcpyAsync(out + at, p.p, p.bytes, hipMemcpyDeviceToHost, n->stream));
        at += p.bytes;
    }
    CX_HIP(hipStreamSynchronize(n->stream));
    return CORTEX_OK;
    CX_API_END
}

int cortex_load_state(cortex_net* n, const void* host, int64_t bytes) {
    CX_API_BEGIN
    require_net(n);
    require(host != nullptr, CORTEX_EINVAL, "host buffer is NULL");
    state_supported(n);
    const auto parts = state_parts(n);
    const StateHeader mine = state_header(n, parts);
    require(bytes >= (int64_t)sizeof(StateHeader), CORTEX_EINVAL, "state buffer too small");
    StateHeader h;
    std::memcpy(&h, host, sizeof h);
    const bool same = h.magic == kStateMagic && h.N == mine.N && h.E == mine.E && h.log_steps == mine.log_steps &&
                      h.n_tiles == mine.n_tiles && h.T == mine.T && h.R == mine.R && h.H == mine.H &&
                      h.W == mine.W && h.ring_bytes == mine.ring_bytes && h.plan_kind == mine.plan_kind &&
                      h.stdp == mine.stdp && h.n_parts == mine.n_parts && h.bytes == mine.bytes &&
                      h.seed == mine.seed;
    require(same, CORTEX_EINVAL, "the state was saved by a network of another spec, seed or plan");
    require(bytes >= h.bytes, CORTEX_EINVAL, "state buffer shorter than its header says");
    CX_HIP(hipStreamSynchronize(n->stream));
    if (n->plan_kind == CORTEX_PLAN_STREAMED) drop_graph(n);
    const unsigned char* in = static_cast<const unsigned char*>(host);
    size_t at = sizeof h;
    for (const auto& p : parts) {
        CX_HIP(hipMemcpyAsync(p.p, in + at, p.bytes, hipMemcpyHostToDevice, n->stream));
        at += p.bytes;
    }
    CX_HIP(hipStreamSynchronize(n->stream));
    n->step = h.step;
    n->log_step0 = h.log_step0;
    n->clock_parity = h.clock_parity;
    return CORTEX_OK;
    CX_API_END
}

int cortex_get_state(cortex_net* n, double* V, int32_t* r, double* y1, double* y2) {
    CX_API_BEGIN
    require_net(n);
    check_device_flag(n);
    const bool fp64 = n->spec.precision == CORTEX_FP64_VERIFY;
    const double EL = n->spec.E_L;
    if (fp64) {
        if (V) { auto u = download(n, n->d_Ud, n->N); for (int64_t i = 0; i < n->N; ++i) V[i] = u[i] + EL; }
        if (y1) { auto u = download(n, n->d_y1d, n->N); std::copy(u.begin(), u.end(), y1); }
        if (y2) { auto u = download(n, n->d_y2d, n->N); std::copy(u.begin(), u.end(), y2); }
    } else {
        if (V) { auto u = download(n, n->d_U, n->N); for (int64_t i = 0; i < n->N; ++i) V[i] = (double)u[i] + EL; }
        if (y1) { auto u = download(n, n->d_y1, n->N); for (int64_t i = 0; i < n->N; ++i) y1[i] = u[i]; }
        if (y2) { auto u = download(n, n->d_y2, n->N); for (int64_t i = 0; i < n->N; ++i) y2[i] = u[i]; }
    }
    if (r) { auto u = download(n, n->d_r, n->N); std::copy(u.begin(), u.end(), r); }
    return CORTEX_OK;
    CX_API_END
}

int cortex_export_graph(cortex_net* n, int64_t* src, int64_t* tgt, double* w, int32_t* d) {
    CX_API_BEGIN
    require_net(n);
    if (n->stdp) check_device_flag(n);   // plastic weights are valid only if no history ran short
    if (n->spec.precision == CORTEX_FP64_VERIFY) {
        auto ptr = download(n, n->d_in_ptr, n->N + 1);
        auto s = download(n, n->d_in_src, n->E);
        auto ww = download(n, n->d_in_w, n->E);
        auto dd = download(n, n->d_in_d, n->E);
        for (int64_t i = 0; i < n->N; ++i)
            for (uint64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
                if (src) src[e] = s[e];
                if (tgt) tgt[e] = i;
                if (w) w[e] = ww[e];
                if (d) d[e] = dd[e];
            }
        return CORTEX_OK;
    }
    auto rs = download(n, n->d_row_start, n->N + 1);
    uint64_t off_len = 0;
    for (int b = 0; b < n->n_inst; ++b) off_len += (uint64_t)n->inst_N[b] * (n->inst_ntiles[b] + 1);
    auto off = download(n, n->d_off_rel, off_len);
    std::vector<uint32_t> meta(n->E);
    std::vector<double> wv(n->E);
    if (n->w_bytes == 2) {
        // packed records: bf16 weight in the high half
        meta = download(n, static_cast<const uint32_t*>(n->d_meta), n->E);
        for (int64_t e = 0; e < n->E; ++e) {
            uint32_t u = meta[e] & 0xFFFF0000u;
            float f;
            std::memcpy(&f, &u, 4);
            wv[e] = f;
            meta[e] &= 0xFFFFu;
        }
    } else if (n->meta_bytes == 2) {
        auto m = download(n, static_cast<const uint16_t*>(n->d_meta), n->E);
        std::copy(m.begin(), m.end(), meta.begin());
    } else {
        meta = download(n, static_cast<const uint32_t*>(n->d_meta), n->E);
    }
    if (n->w_bytes != 2) {
        auto m = download(n, static_cast<const float*>(n->d_w), n->E);
        for (int64_t e = 0; e < n->E; ++e) wv[e] = m[e];
    }
    const uint32_t ts = (uint32_t)n->T;   // record = (delay - dmin) T + target in tile
    for (int b = 0; b < n->n_inst; ++b) {
        const int nt = n->inst_ntiles[b];
        for (int64_t jl = 0; jl < n->inst_N[b]; ++jl) {
            const int64_t j = n->inst_n0[b] + jl;
            const uint64_t ob = n->inst_offbase[b] + (uint64_t)jl * (nt + 1);
            for (int t = 0; t < nt; ++t) {
                for (uint64_t e = rs[j] + off[ob + t]; e < rs[j] + off[ob + t + 1]; ++e) {
                    if (src) src[e] = j;
                    if (tgt) tgt[e] = n->inst_n0[b] + (int64_t)t * n->inst_T[b] + (meta[e] % ts);
                    if (w) w[e] = wv[e];
                    if (d) d[e] = n->dmin + (int32_t)(meta[e] / ts);
                }
            }
        }
    }
    return CORTEX_OK;
    CX_API_END
}

int cortex_export_canonical(cortex_net* n, int64_t* canon) {
    CX_API_BEGIN
    require_net(n);
    require(canon != nullptr, CORTEX_EINVAL, "canon is NULL");
    const uint32_t* src = n->spec.precision == CORTEX_FP64_VERIFY ? n->d_in_canon : n->d_canon;
    require(src != nullptr, CORTEX_ESTATE, "canonical indices need ckpt_every > 0 in FP32 mode");
    auto c = download(n, src, n->E);
    for (int64_t e = 0; e < n->E; ++e) canon[e] = c[e];
    return CORTEX_OK;
    CX_API_END
}

int cortex_export_tiles(cortex_net* n, int64_t* start, int32_t* size, int32_t* instance) {
    CX_API_BEGIN
    require_net(n);
    require(n->spec.precision != CORTEX_FP64_VERIFY, CORTEX_ESTATE, "FP64 networks have no tiles");
    for (int t = 0; t < n->n_tiles; ++t) {
        if (start) start[t] = n->tile_start[t];
        if (size) size[t] = n->tile_size[t];
        if (instance) instance[t] = n->tile_inst[t];
    }
    return CORTEX_OK;
    CX_API_END
}

int cortex_query(cortex_net* n, int what, int64_t* value) {
    CX_API_BEGIN
    require(n != nullptr && value != nullptr, CORTEX_EINVAL, "NULL argument");
    const bool fp64 = n->spec.precision == CORTEX_FP64_VERIFY;
    switch (what) {
        case CORTEX_Q_NEURONS: *value = n->N; break;
        case CORTEX_Q_SYNAPSES: *value = n->E; break;
        case CORTEX_Q_MIN_DELAY: *value = n->dmin; break;
        case CORTEX_Q_MAX_DELAY: *value = n->dmax; break;
        case CORTEX_Q_TILES: *value = n->n_tiles; break;
        case CORTEX_Q_TILE_SIZE: *value = n->T; break;
        case CORTEX_Q_RING_SLOTS: *value = n->R; break;
        case CORTEX_Q_STEP: *value = n->step; break;
        case CORTEX_Q_DEVICE_BYTES: *value = (int64_t)n->dev_bytes; break;
        case CORTEX_Q_EDGE_BYTES: *value = fp64 ? 14 : n->meta_bytes + n->w_bytes; break;
        case CORTEX_Q_BLOCK_SIZE: *value = n->BS; break;
        case CORTEX_Q_LDS_BYTES: *value = (int64_t)n->lds_bytes; break;
        case CORTEX_Q_OFFSET_BYTES: {
            uint64_t off_len = 0;
            for (int b = 0; b < n->n_inst && !fp64; ++b) off_len += (uint64_t)n->inst_N[b] * (n->inst_ntiles[b] + 1);
            *value = (int64_t)off_len * 4;
            break;
        }
        case CORTEX_Q_STEPS_PER_SYNC: *value = fp64 ? 1 : n->W; break;
        case CORTEX_Q_RING_BYTES: *value = fp64 ? 8 : n->ring_bytes; break;
        case CORTEX_Q_PLAN: *value = fp64 ? 0 : n->plan_kind; break;
        case CORTEX_Q_NPT: *value = fp64 ? 0 : n->NPT; break;
        case CORTEX_Q_STAGE_RECORDS: *value = fp64 ? 0 : (int64_t)n->stage_cap; break;
        case CORTEX_Q_STAGE_GROUP: *value = (fp64 || !n->stage_cap) ? 0 : (int64_t)n->stage_group; break;
        case CORTEX_Q_EVENTS:
        case CORTEX_Q_SPIKES: {
            require(!n->failed, CORTEX_ESTATE, "network failed earlier");
            check_device_flag(n);
            if (fp64) {
                auto v = download(n, n->d_events, 2);
                *value = (int64_t)v[what == CORTEX_Q_EVENTS ? 0 : 1];
            } else {
                auto v = download(n, what == CORTEX_Q_EVENTS ? n->d_events : n->d_spikes, n->n_tiles);
                int64_t s = 0;
                for (auto x : v) s += (int64_t)x;
                *value = s;
            }
            break;
        }
        default: throw Error{CORTEX_EINVAL, "unknown query"};
    }
    return CORTEX_OK;
    CX_API_END
}

int cortex_kernel_timing(cortex_net* n, int on) {
    CX_API_BEGIN
    require(n != nullptr, CORTEX_EINVAL, "null network");
    require(n->spec.precision == CORTEX_FP32 && n->plan_kind == CORTEX_PLAN_STREAMED, CORTEX_EUNSUPPORTED,
            "kernel timing is for the streamed FP32 plan");
    if (on && !n->d_ktime) n->d_ktime = dev_alloc_t<KernelTime>(n, 1);
    if (on) {
        // sums cleared, no open interval
        const KernelTime init{};
        CX_HIP(hipMemcpyAsync(n->d_ktime, &init, sizeof init, hipMemcpyHostToDevice, n->stream));
        CX_HIP(hipStreamSynchronize(n->stream));
    }
    if ((on != 0) != n->ktiming) {
        n->ktiming = on != 0;
        drop_graph(n);   // the launches' arguments change
    }
    return CORTEX_OK;
    CX_API_END
}

int cortex_kernel_times(cortex_net* n, double* ms, int32_t* n_windows) {
    CX_API_BEGIN
    require(n != nullptr && ms != nullptr && n_windows != nullptr, CORTEX_EINVAL, "null argument");
    require(n->spec.precision == CORTEX_FP32 && n->plan_kind == CORTEX_PLAN_STREAMED, CORTEX_EUNSUPPORTED,
            "kernel timing is for the streamed FP32 plan");
    ms[0] = ms[1] = 0.0;
    *n_windows = 0;
    if (!n->ktiming || !n->d_ktime) return CORTEX_OK;
    CX_HIP(hipStreamSynchronize(n->stream));
    if (n->graph_stream) CX_HIP(hipStreamSynchronize(n->graph_stream));
    KernelTime kt{};
    CX_HIP(hipMemcpy(&kt, n->d_ktime, sizeof kt, hipMemcpyDeviceToHost));
    int rate_khz = 0;
    CX_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, n->device));
    require(rate_khz > 0, CORTEX_EDEVICE, "device clock rate unknown");
    for (int k = 0; k < 2; ++k)
        ms[k] = kt.count[k] ? (double)kt.sum[k] / (double)kt.count[k] / (double)rate_khz : 0.0;
    *n_windows = (int32_t)std::min<unsigned long long>(kt.count[1], 0x7FFFFFFF);
    return CORTEX_OK;
    CX_API_END
}

void cortex_destroy(cortex_net* n) {
    if (!n) return;
    (void)hipStreamSynchronize(n->stream);
    if (n->graph_stream) (void)hipStreamSynchronize(n->graph_stream);
    if (n->graph_exec) (void)hipGraphExecDestroy(n->graph_exec);
    if (n->fence_in) (void)hipEventDestroy(n->fence_in);
    if (n->fence_out) (void)hipEventDestroy(n->fence_out);
    if (n->graph_stream) (void)hipStreamDestroy(n->graph_stream);
    release(n, n->scratch);
    release(n, n->bufs);
    delete n;
}

}  // extern "C"
