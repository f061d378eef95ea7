// ebic_evaluate_device_noalloc: the device-pointer evaluation for callers
// that cannot allocate device memory (graph capture, serving loops).
//
// The evaluation's only scratch is one packed 64-bit accumulator per
// candidate (the parts of a candidate spread over several workgroups add
// their row counts there; the last part writes count and fitness and
// zeroes it).  Here those accumulators live in a fixed file-scope device
// array that every GPU holds, at its own address, until the process ends.
// Host code never passes the array's name to a kernel: the name is only a
// host-side stand-in.  The device address is looked up once per device
// with hipGetSymbolAddress (when the first context on that device is
// created) and that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ebic_internal.h"

namespace {

constexpr int32_t kMaxCandidates = EBIC_NOALLOC_MAX_CANDIDATES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned long long scratch[kMaxCandidates];

std::mutex g_mu;
unsigned long long *g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device
hipError_t g_status[kMaxDevices] = {};             // outcome of the lookup, per device
bool g_done[kMaxDevices] = {};

__global__ __launch_bounds__(256) void clear_acc_kernel(unsigned long long *__restrict__ acc,
                                                        int32_t n) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) acc[i] = 0ull;
}

}  // namespace

namespace ebic {

hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_done[device]) return g_status[device];
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_done[device] = true;
    g_status[device] = e;
    if (e == hipSuccess)
        g_scratch[device] = static_cast<unsigned long long *>(p);
    else
        (void)hipGetLastError();   // leave no sticky error for the next call
    return e;
}

}  // namespace ebic

extern "C" ebic_status ebic_evaluate_device_noalloc(ebic_ctx *ctx, const int32_t *d_offsets,
                                                    const int32_t *d_cols, int32_t P,
                                                    int64_t n_entries, const ebic_params *params,
                                                    uint64_t *d_masks, int32_t *d_counts,
                                                    double *d_fitness, void *hip_stream) {
    if (!ctx) return ebic::fail_status(nullptr, EBIC_E_ARG, "ctx is null");
    if (P > kMaxCandidates)
        return ebic::fail_status(ctx, EBIC_E_RANGE,
                                 "P exceeds EBIC_NOALLOC_MAX_CANDIDATES (65536)");
    unsigned long long *acc = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (ctx->device >= 0 && ctx->device < kMaxDevices) acc = g_scratch[ctx->device];
    }
    if (!acc)
        return ebic::fail_status(ctx, EBIC_E_DEVICE,
                                 "no-allocation scratch array unavailable on this device "
                                 "(hipGetSymbolAddress failed)");
    if (P > 0 && params && params->struct_size >= sizeof(ebic_params)) {
        // Clear what this call's accumulators must start from (a kernel,
        // not a memset node, so the call can be captured in a graph).
        if (hipSetDevice(ctx->device) != hipSuccess)
            return ebic::fail_status(ctx, EBIC_E_DEVICE, "hipSetDevice failed");
        hipStream_t s = static_cast<hipStream_t>(hip_stream);
        hipLaunchKernelGGL(clear_acc_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s,
                           acc, P);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return ebic::fail_status(ctx, EBIC_E_DEVICE, hipGetErrorString(e));
    }
    return ebic::evaluate_device_impl(ctx, d_offsets, d_cols, P, n_entries, params, d_masks,
                                      d_counts, d_fitness, hip_stream, acc);
}
