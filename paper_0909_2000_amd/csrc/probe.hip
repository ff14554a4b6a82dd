// A measurement helper, not part of the method: the sustained rate of packed
// 16-bit VALU operations on the device, against which the seaweed kernels'
// rates are reported.  Every lane advances eight independent chains of
// v_pk_max_u16 (two 16-bit operations per lane and instruction), so no
// instruction waits for the one before it, over enough waves to fill every
// SIMD of every CU.  The second operand is a scalar register, so each
// instruction reads a single vector register.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlcs {
namespace {

#define WLCS_PEAK_ROUND                \
    "v_pk_max_u16 %0, %0, %8\n\t"      \
    "v_pk_max_u16 %1, %1, %8\n\t"      \
    "v_pk_max_u16 %2, %2, %8\n\t"      \
    "v_pk_max_u16 %3, %3, %8\n\t"      \
    "v_pk_max_u16 %4, %4, %8\n\t"      \
    "v_pk_max_u16 %5, %5, %8\n\t"      \
    "v_pk_max_u16 %6, %6, %8\n\t"      \
    "v_pk_max_u16 %7, %7, %8\n\t"

__global__ __launch_bounds__(256) void valu_peak_kernel(uint32_t* __restrict__ out, int32_t iters) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    uint32_t a0 = t, a1 = t ^ 0x11111111u, a2 = t ^ 0x22222222u, a3 = t ^ 0x33333333u;
    uint32_t a4 = t ^ 0x44444444u, a5 = t ^ 0x55555555u, a6 = t ^ 0x66666666u, a7 = t ^ 0x77777777u;
    const uint32_t b = __builtin_amdgcn_readfirstlane(blockIdx.x * 0x9E3779B9u);
    for (int32_t i = 0; i < iters; ++i) {
        // 64 instructions per iteration
        asm volatile(WLCS_PEAK_ROUND WLCS_PEAK_ROUND WLCS_PEAK_ROUND WLCS_PEAK_ROUND WLCS_PEAK_ROUND
                         WLCS_PEAK_ROUND WLCS_PEAK_ROUND WLCS_PEAK_ROUND
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                     : "s"(b));
    }
    out[t] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;  // keeps the chains alive
}
#undef WLCS_PEAK_ROUND

}  // namespace

// blocks x 256 threads; element operations per launch: blocks * 256 * iters * 64 * 2
hipError_t launch_valu_peak(uint32_t* out, int32_t blocks, int32_t iters, hipStream_t stream) {
    hipLaunchKernelGGL(valu_peak_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, out, iters);
    return hipGetLastError();
}

}  // namespace wlcs
