// apd_probe.hip -- issue-rate probe of the vector ALU, the ceiling against
// which the assignment kernels are measured.
//
// Each thread runs eight independent register chains of one instruction
// kind, each instruction reading registers that no other chain writes, so
// that neither dependencies nor shared operands limit the rate; the grid puts
// eight waves on every SIMD.  The result is the sustained number of VALU lane
// operations per second (instructions x 64 lanes / time).
#include "../../include/apd.h"

#include <hip/hip_runtime.h>

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeWavesPerSimd = 8;

template <int OP>
__global__ __launch_bounds__(kProbeThreads) void k_probe_valu(float *out, int iters, float a0, float b0) {
    float a[8], b[8], x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = a0 + (float)(threadIdx.x + k) * 1e-7f;
        b[k] = b0 + (float)k * 1e-3f;
        x[k] = (float)k;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float p = a[(k + 1 + r) & 7], q = b[(k + 3 + r) & 7];
                if (OP == 0) x[k] = fmaf(x[k], p, q);   // fused multiply-add
                if (OP == 1) x[k] = x[k] + p;           // add
            }
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k] + a[k];
    out[blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" apd_status apd_measure_valu_rate(int32_t device, int32_t op, double *lane_ops_per_s) {
    if (!lane_ops_per_s || op < 0 || op > 1) return APD_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return APD_ERR_DEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1)
        return APD_ERR_DEVICE;
    // a block is 4 waves, one per SIMD of a compute unit
    const int blocks = cus * kProbeWavesPerSimd;
    const int iters = 20000;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * kProbeThreads) != hipSuccess) return APD_ERR_OOM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    apd_status st = APD_OK;
    float ms = 0.0f;
    auto launch = [&](int it) {
        if (op == 0) hipLaunchKernelGGL(k_probe_valu<0>, dim3(blocks), dim3(kProbeThreads), 0, 0, out, it, 1.0f, 0.0f);
        if (op == 1) hipLaunchKernelGGL(k_probe_valu<1>, dim3(blocks), dim3(kProbeThreads), 0, 0, out, it, 1e-9f, 0.0f);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        st = APD_ERR_DEVICE;
    } else {
        launch(16);  // first launch: code load
        if (hipDeviceSynchronize() != hipSuccess || hipEventRecord(e0, 0) != hipSuccess) st = APD_ERR_DEVICE;
        if (st == APD_OK) {
            launch(iters);
            if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f)
                st = APD_ERR_DEVICE;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (st != APD_OK) {
        (void)hipGetLastError();
        return st;
    }
    const double lane_ops = (double)blocks * kProbeThreads * (double)iters * 32.0;
    *lane_ops_per_s = lane_ops / ((double)ms * 1e-3);
    return APD_OK;
}
