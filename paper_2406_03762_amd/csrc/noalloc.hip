// cortex_run_frozen_noalloc: the frozen-raster run without any device
// allocation, for callers that cannot allocate (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// cortex_run_frozen builds the per-(step, tile) spike lists on the host and
// uploads them into scratch memory it allocates.  This variant copies the raw
// raster into a fixed device array instead and builds the list offsets on
// the device: the raster is sorted by (step, id) and every tile holds a
// contiguous id range, so the list of (step s, tile t) is the raster range
// between the lower bounds of (s, first target of t) and (s, first target
// of t + 1); the ids array is the raster's own.
//
// The fixed array (kScratchBytes, one copy per GPU, kept until the process
// ends) is shared by every call on that GPU: calls that overlap on one GPU
// race, and each call overwrites what the previous one left.
#include <algorithm>
#include <mutex>

#include "internal.hpp"

namespace cortex {
namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).
void* scratch_on(int device) {
    require(device >= 0 && device < kMaxDevices, CORTEX_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        CX_HIP(hipGetDevice(&cur));
        if (cur != device) CX_HIP(hipSetDevice(device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) CX_HIP(hipSetDevice(cur));
        require(e == hipSuccess && p != nullptr, CORTEX_EDEVICE,
                std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    return g_scratch_ptr[device];
}

// ptr[s * n_keys + k] = first raster entry with (step, id) >= (step0 + s,
// keys[k]); ptr[n_steps * n_keys] = first entry with step >= step0 +
// n_steps.  With keys = the tiles' first neurons, [ptr[i], ptr[i + 1]) is
// the list of (step, tile) i.
__global__ void raster_index_kernel(const uint32_t* steps, const uint32_t* ids, int64_t n_spk, int64_t step0,
                                    int64_t n_steps, const int64_t* keys, int n_keys, uint64_t* ptr) {
    const int64_t total = n_steps * n_keys + 1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t key_step, key_id;
        if (i == total - 1) {
            key_step = step0 + n_steps;
            key_id = 0;
        } else {
            key_step = step0 + i / n_keys;
            key_id = keys[i % n_keys];
        }
        int64_t lo = 0, hi = n_spk;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            const int64_t s = steps[mid];
            if (s < key_step || (s == key_step && (int64_t)ids[mid] < key_id)) lo = mid + 1;
            else hi = mid;
        }
        ptr[i] = (uint64_t)lo;
    }
}

}  // namespace

void raster_index(cortex_net* n, const uint32_t* steps, const uint32_t* ids, int64_t n_spk, int64_t step0,
                  int64_t n_steps, const int64_t* keys, int n_keys, uint64_t* ptr) {
    const int64_t total = n_steps * n_keys + 1;
    const int grid = (int)std::min<int64_t>(4096, (total + 255) / 256);
    hipLaunchKernelGGL(raster_index_kernel, dim3(grid), dim3(256), 0, n->stream, steps, ids, n_spk, step0, n_steps,
                       keys, n_keys, ptr);
    CX_HIP(hipGetLastError());
}

}  // namespace cortex

using namespace cortex;

extern "C" int cortex_run_frozen_noalloc(cortex_net* n, const uint32_t* r_steps, const uint32_t* r_ids,
                                         int64_t n_spikes, int64_t n_steps, void* x_trace, void* v_trace) {
    try {
        require(n != nullptr, CORTEX_EINVAL, "network handle is NULL");
        require(!n->failed, CORTEX_ESTATE, "network failed earlier; destroy it");
        require(n->spec.precision == CORTEX_FP32, CORTEX_EUNSUPPORTED, "the allocation-free run is FP32 only");
        require(n_steps >= 0 && n_spikes >= 0 && (n_spikes == 0 || (r_steps && r_ids)), CORTEX_EINVAL,
                "bad raster");
        require((x_trace == nullptr) == (v_trace == nullptr), CORTEX_EINVAL, "pass both traces or neither");
        for (int64_t q = 0; q < n_spikes; ++q) {
            require(r_ids[q] < n->N, CORTEX_EINVAL, "raster id out of range");
            require(q == 0 || r_steps[q] > r_steps[q - 1] ||
                        (r_steps[q] == r_steps[q - 1] && r_ids[q] > r_ids[q - 1]),
                    CORTEX_EINVAL, "raster must be sorted by (step, id) without duplicates");
        }
        if (n_steps == 0) return CORTEX_OK;
        check_plastic_raster(n, r_steps, r_ids, n_spikes);
        // layout: list offsets [n_steps * n_tiles + 1] u64, raster steps and ids u32
        const size_t ptr_bytes = ((size_t)n_steps * n->n_tiles + 1) * sizeof(uint64_t);
        const size_t ras_bytes = (size_t)n_spikes * sizeof(uint32_t);
        const size_t need = ((ptr_bytes + 255) & ~(size_t)255) + 2 * ((ras_bytes + 255) & ~(size_t)255);
        require(need <= kScratchBytes, CORTEX_EINVAL,
                "raster too large for the allocation-free run: needs " + std::to_string(need) +
                    " bytes of its " + std::to_string(kScratchBytes) + "-byte scratch array "
                    "(steps x tiles x 8 + spikes x 8, rounded)");
        unsigned char* base = static_cast<unsigned char*>(scratch_on(n->device));
        uint64_t* d_ptr = reinterpret_cast<uint64_t*>(base);
        uint32_t* d_steps = reinterpret_cast<uint32_t*>(base + ((ptr_bytes + 255) & ~(size_t)255));
        uint32_t* d_ids = reinterpret_cast<uint32_t*>(reinterpret_cast<unsigned char*>(d_steps) +
                                                      ((ras_bytes + 255) & ~(size_t)255));
        if (n_spikes > 0) {
            CX_HIP(hipMemcpyAsync(d_steps, r_steps, ras_bytes, hipMemcpyHostToDevice, n->stream));
            CX_HIP(hipMemcpyAsync(d_ids, r_ids, ras_bytes, hipMemcpyHostToDevice, n->stream));
        }
        raster_index(n, d_steps, d_ids, n_spikes, n->step, n_steps, n->d_tile_start, n->n_tiles, d_ptr);
        advance_fp32(n, n_steps, d_ids, d_ptr, (uint64_t)n_spikes, static_cast<float*>(x_trace),
                     static_cast<float*>(v_trace));
        check_device_flag(n);
        return CORTEX_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (...) {
        set_error("unexpected internal error");
        return CORTEX_EDEVICE;
    }
}
