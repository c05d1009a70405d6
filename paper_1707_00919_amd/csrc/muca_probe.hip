// muca_probe.hip -- issue-rate probes of the gfx950 vector ALU, for the
// integer roof the sweep kernels are measured against.
//
// Each lane advances eight independent chains of one instruction kind for a
// given number of iterations, so a wave always has independent work to issue
// and the SIMD's issue rate, not the instruction's latency, sets the time.  The
// instruction kinds are those of the chain step and of Philox4x32-10: a 32-bit
// add, a three-input xor (v_bitop3_b32), the low and the high 32 bits of a
// 32 x 32 product, and the 32 x 32 + 64 -> 64 multiply-add.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "muca.h"

namespace {

constexpr int kChains = 8;

// One step of chain a; n is the neighbouring chain's value, b and c are
// kernel arguments.  The add, the xor and the low product take n as an
// operand so that the compiler cannot fold a chain's steps into one.
template <int OP>
__device__ __forceinline__ uint32_t probe_op(uint32_t a, uint32_t n, uint32_t b, uint32_t c)
{
    if constexpr (OP == MUCA_PROBE_ADD)
        return a + n;
    else if constexpr (OP == MUCA_PROBE_XOR3)
        return __builtin_amdgcn_bitop3_b32(a, n, c, 0x96);
    else if constexpr (OP == MUCA_PROBE_MUL_LO)
        return a * n;
    else if constexpr (OP == MUCA_PROBE_MUL_HI)
        return __umulhi(a, b);
    else
        return (uint32_t)(((uint64_t)a * b + (uint64_t)c) >> 32);
}

template <int OP>
__global__ __launch_bounds__(256) void probe_kernel(uint32_t* out, uint32_t iterations, uint32_t b, uint32_t c)
{
    uint32_t x[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        x[j] = threadIdx.x * 2654435761u + (uint32_t)j * 40503u + blockIdx.x;
    for (uint32_t it = 0; it < iterations; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int j = 0; j < kChains; ++j)
                x[j] = probe_op<OP>(x[j], x[(j + 1) % kChains], b, c);
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        acc ^= x[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

template <int OP>
hipError_t launch_probe(uint32_t blocks, uint32_t* out, uint32_t iterations, hipStream_t s)
{
    hipLaunchKernelGGL(probe_kernel<OP>, dim3(blocks), dim3(256), 0, s, out, iterations, 0x9E3779B9u, 0x7F4A7C15u);
    return hipGetLastError();
}

}  // namespace

extern "C" int muca_probe_issue_rate(uint32_t op, uint32_t waves_per_simd, uint32_t iterations, double* ms,
                                     uint64_t* lane_ops)
{
    if (!ms || !lane_ops || op > MUCA_PROBE_MAD_U64 || waves_per_simd == 0 || waves_per_simd > 8 ||
        iterations == 0 || iterations > (1u << 24))
        return MUCA_ERR_INVALID_ARG;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return MUCA_ERR_DEVICE;
    // a workgroup of 256 threads is four waves, one per SIMD of a CU
    const uint32_t blocks = (uint32_t)cus * waves_per_simd;
    uint32_t* out = nullptr;
    if (hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return MUCA_ERR_OUT_OF_MEMORY;
    }
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MUCA_OK;
    float t = 0.0f;
    auto launch = [&](uint32_t iters) -> hipError_t {
        switch (op) {
        case MUCA_PROBE_ADD: return launch_probe<MUCA_PROBE_ADD>(blocks, out, iters, s);
        case MUCA_PROBE_XOR3: return launch_probe<MUCA_PROBE_XOR3>(blocks, out, iters, s);
        case MUCA_PROBE_MUL_LO: return launch_probe<MUCA_PROBE_MUL_LO>(blocks, out, iters, s);
        case MUCA_PROBE_MUL_HI: return launch_probe<MUCA_PROBE_MUL_HI>(blocks, out, iters, s);
        default: return launch_probe<MUCA_PROBE_MAD_U64>(blocks, out, iters, s);
        }
    };
    if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess || launch(16) != hipSuccess ||
        hipEventRecord(e0, s) != hipSuccess || launch(iterations) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        rc = MUCA_ERR_DEVICE;
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (s)
        (void)hipStreamDestroy(s);
    (void)hipFree(out);
    if (rc != MUCA_OK)
        return rc;
    *ms = t;
    *lane_ops = (uint64_t)blocks * 256u * iterations * 8u * kChains;
    return MUCA_OK;
}
