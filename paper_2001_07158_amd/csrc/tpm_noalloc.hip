// tpm_sieve_noalloc: the sieve of tpm_sieve for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops that must not call hipMalloc).
// Every buffer of the query lives in one fixed block of device memory per GPU, the
// array `scratch` below; the kernels are tpm_sieve's.
//
// In host code `scratch` names a host-side stand-in, not device memory: its device
// address comes from hipGetSymbolAddress, once per device with that device current, and
// only that address is ever passed to kernels.

#include <hip/hip_runtime.h>

#include <mutex>

#include "tpm_internal.h"

using namespace tpm;

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the current device must be dev).
uint8_t *scratch_on(int dev) {
    TPM_REQUIRE(dev >= 0 && dev < kMaxDevices, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        TPM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error{TPM_EDEVICE, "hipGetSymbolAddress returned no address for the scratch"};
        g_scratch_ptr[dev] = (uint8_t *)p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

tpm_status tpm_sieve_noalloc(const tpm_graph *g, const int32_t *multiset, int32_t k, uint64_t seed,
                             uint8_t *per_point, uint8_t *total, uint32_t *error_flags,
                             void *hip_stream) {
    return guarded_call([&]() -> tpm_status {
        TPM_REQUIRE(g != nullptr, "graph must not be NULL");
        TPM_REQUIRE(total != nullptr, "total must not be NULL");
        const Graph &G = g->G;
        DeviceGuard dg(G.device);
        int cur = -1;
        TPM_HIP(hipGetDevice(&cur));
        if (cur != G.device) throw Error{TPM_EDEVICE, "cannot make the graph's device current"};
        uint8_t *base = scratch_on(cur);
        enqueue_sieve_fixed(G, multiset, k, seed, base, kScratchBytes, per_point, total, error_flags,
                            (hipStream_t)hip_stream);
        return TPM_OK;
    });
}

}  // extern "C"
