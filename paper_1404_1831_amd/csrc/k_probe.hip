// Measurement probe: the rate of random 4-byte LDS reads from 256-entry
// tables, the access pattern of the scans' table lookups (one table per PQ
// subspace, a code byte as the index), over the whole chip. It is a
// denominator for the scans' LDS roof, not part of the search.
#include <hip/hip_runtime.h>

#include "fbpq.h"

namespace {

constexpr int kProbeNT = 256;
constexpr int kProbeTabs = 16;

__global__ __launch_bounds__(kProbeNT) void k_probe_lds(int iters, float *out)
{
    __shared__ float tab[kProbeTabs * 256];
    for (int i = threadIdx.x; i < kProbeTabs * 256; i += kProbeNT) tab[i] = (float)(i & 1023);
    __syncthreads();
    uint32_t x = 0x9e3779b9u * (uint32_t)(blockIdx.x * kProbeNT + threadIdx.x + 1);
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int g = 0; g < kProbeTabs / 4; ++g) {
            x ^= x << 13;
            x ^= x >> 17;
            x ^= x << 5;
#pragma unroll
            for (int b = 0; b < 4; ++b) acc += tab[(g * 4 + b) * 256 + ((x >> (8 * b)) & 255)];
        }
    }
    if (acc == -1.f) out[0] = acc;  // never true: keeps the reads
}

}  // namespace

extern "C" int fbpq_probe_lds_gather(int device, double *lookups_per_s)
{
    if (!lookups_per_s) return FBPQ_E_INVALID;
    if (hipSetDevice(device) != hipSuccess) {
        (void)hipGetLastError();
        return FBPQ_E_DEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || ncu < 1)
        ncu = 256;
    const int blocks = ncu * 8, iters = 2048;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float *out = nullptr;
    int rc = FBPQ_OK;
    float ms = 0.f;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess || hipMalloc(&out, sizeof(float)) != hipSuccess) {
        rc = FBPQ_E_DEVICE;
    } else {
        hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(kProbeNT), 0, st, iters, out);  // warm
        (void)hipEventRecord(e0, st);
        hipLaunchKernelGGL(k_probe_lds, dim3(blocks), dim3(kProbeNT), 0, st, iters, out);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f)
            rc = FBPQ_E_DEVICE;
    }
    if (rc == FBPQ_OK) *lookups_per_s = (double)blocks * kProbeNT * iters * kProbeTabs / (ms * 1e-3);
    (void)hipGetLastError();
    if (out) (void)hipFree(out);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    return rc;
}
