// A measurement helper, not part of the method: the sustained rate of packed
// 16-bit VALU operations on the device, against which the seaweed kernels'
// rates are reported.  Every lane advances eight independent chains of
// v_pk_max_u16 (two 16-bit operations per lane and instruction), so no
// instruction waits for the one before it, over enough waves to fill every
// SIMD of every CU.  The second operand is a scalar register, so each
// instruction reads a single vector register.
//
// The second helper measures the issue rate of wave64 VALU instructions with
// a chosen number of waves resident on every SIMD: one workgroup of 256 k
// threads per CU puts k waves on each of its four SIMDs at once.  Each wave
// runs rounds of one kind of instruction stream: packed 16-bit, plain 32-bit
// or three-input bitwise instructions on eight independent accumulators, or
// the seaweed cell down a column of eight rows (each cell waits for the label
// the cell above sends down, the dependency of the plot kernels).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "packed.hpp"

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

namespace {

#define WLCS_ISSUE_ROUND(OP)                                                                        \
    asm volatile(OP " %0, %0, %8\n\t" OP " %1, %1, %8\n\t" OP " %2, %2, %8\n\t" OP " %3, %3, %8\n\t" \
                 OP " %4, %4, %8\n\t" OP " %5, %5, %8\n\t" OP " %6, %6, %8\n\t" OP " %7, %7, %8"      \
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)          \
                 : "v"(b))

#define WLCS_ISSUE_ROUND3(OP)                                                                        \
    asm volatile(OP " %0, %0, %8, %9 bitop3:0x96\n\t" OP " %1, %1, %8, %9 bitop3:0x96\n\t"          \
                 OP " %2, %2, %8, %9 bitop3:0x96\n\t" OP " %3, %3, %8, %9 bitop3:0x96\n\t"          \
                 OP " %4, %4, %8, %9 bitop3:0x96\n\t" OP " %5, %5, %8, %9 bitop3:0x96\n\t"          \
                 OP " %6, %6, %8, %9 bitop3:0x96\n\t" OP " %7, %7, %8, %9 bitop3:0x96"                \
                 : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)          \
                 : "v"(b), "v"(t))

// The seaweed cell with Z formed by v_xor_b32 instead of v_pk_add_u16: x and
// y codes equal for equal letters, x's code repeated in both halves of its own
// register (a register per row instead of per two rows).  Probe only.
__device__ __forceinline__ uint32_t xor_cell(uint32_t& s, uint32_t t, uint32_t xr, uint32_t y) {
    uint32_t down;
    asm volatile(
        "v_xor_b32 %1, %3, %4\n\t"
        "v_pk_min_u16 %1, %2, %1\n\t"
        "v_pk_max_u16 %1, %0, %1\n\t"
        "v_bitop3_b32 %0, %0, %2, %1 bitop3:0x96"
        : "+v"(s), "=&v"(down)
        : "v"(t), "v"(xr), "s"(y));
    return down;
}

// The seaweed cell as first written, its right label by two v_xor_b32 (five
// instructions).  Probe only.
template <int HI>
__device__ __forceinline__ uint32_t two_xor_cell(uint32_t& s, uint32_t t, uint32_t x, uint32_t y) {
    uint32_t down;
    if (HI)
        asm volatile(
            "v_pk_add_u16 %1, %3, %4 op_sel:[1,0]\n\t"
            "v_pk_min_u16 %1, %2, %1\n\t"
            "v_pk_max_u16 %1, %0, %1\n\t"
            "v_xor_b32 %0, %0, %2\n\t"
            "v_xor_b32 %0, %0, %1"
            : "+v"(s), "=&v"(down)
            : "v"(t), "v"(x), "s"(y));
    else
        asm volatile(
            "v_pk_add_u16 %1, %3, %4 op_sel_hi:[0,1]\n\t"
            "v_pk_min_u16 %1, %2, %1\n\t"
            "v_pk_max_u16 %1, %0, %1\n\t"
            "v_xor_b32 %0, %0, %2\n\t"
            "v_xor_b32 %0, %0, %1"
            : "+v"(s), "=&v"(down)
            : "v"(t), "v"(x), "s"(y));
    return down;
}

// KIND 0: 16 v_pk_max_u16 per round, KIND 1: 16 v_xor_b32, KIND 2: eight
// seaweed cells (32 instructions) down one column, KIND 3: the same with Z by
// v_xor_b32 (xor_cell, 32), KIND 4: the same with two_xor_cell (40), KIND 5:
// 16 v_bitop3_b32.
template <int KIND>
__global__ __launch_bounds__(1024) void valu_issue_kernel(uint32_t* __restrict__ out, int32_t iters) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t a0 = t, a1 = t ^ 0x11111111u, a2 = t ^ 0x22222222u, a3 = t ^ 0x33333333u;
    uint32_t a4 = t ^ 0x44444444u, a5 = t ^ 0x55555555u, a6 = t ^ 0x66666666u, a7 = t ^ 0x77777777u;
    const uint32_t b = t * 0x9E3779B9u;
    for (int32_t i = 0; i < iters; ++i) {
        if constexpr (KIND == 0) {
            WLCS_ISSUE_ROUND("v_pk_max_u16");
            WLCS_ISSUE_ROUND("v_pk_max_u16");
        } else if constexpr (KIND == 1) {
            WLCS_ISSUE_ROUND("v_xor_b32");
            WLCS_ISSUE_ROUND("v_xor_b32");
        } else if constexpr (KIND == 5) {
            WLCS_ISSUE_ROUND3("v_bitop3_b32");
            WLCS_ISSUE_ROUND3("v_bitop3_b32");
        } else if constexpr (KIND == 4) {
            const uint32_t y = (uint32_t)__builtin_amdgcn_readfirstlane(i * 0x00010001);
            uint32_t d = (uint32_t)__builtin_amdgcn_readfirstlane(i);
            d = two_xor_cell<0>(a0, d, b, y);
            d = two_xor_cell<1>(a1, d, b, y);
            d = two_xor_cell<0>(a2, d, t, y);
            d = two_xor_cell<1>(a3, d, t, y);
            d = two_xor_cell<0>(a4, d, b, y);
            d = two_xor_cell<1>(a5, d, b, y);
            d = two_xor_cell<0>(a6, d, t, y);
            d = two_xor_cell<1>(a7, d, t, y);
            a0 ^= d & 1u;
        } else if constexpr (KIND == 3) {
            const uint32_t y = (uint32_t)__builtin_amdgcn_readfirstlane(i * 0x00010001);
            uint32_t d = (uint32_t)__builtin_amdgcn_readfirstlane(i);
            d = xor_cell(a0, d, b, y);
            d = xor_cell(a1, d, t, y);
            d = xor_cell(a2, d, b, y);
            d = xor_cell(a3, d, t, y);
            d = xor_cell(a4, d, b, y);
            d = xor_cell(a5, d, t, y);
            d = xor_cell(a6, d, b, y);
            d = xor_cell(a7, d, t, y);
            a0 ^= d & 1u;
        } else {
            // labels a0..a7 of eight rows, their letters in two registers,
            // the column's letter (uniform) and top label from the round
            const uint32_t y = (uint32_t)__builtin_amdgcn_readfirstlane(i * 0x00010001);
            uint32_t d = wlcs::seaweed_cell_top(a0, (uint32_t)__builtin_amdgcn_readfirstlane(i), b, y);
            d = wlcs::seaweed_cell<1>(a1, d, b, y);
            d = wlcs::seaweed_cell<0>(a2, d, t, y);
            d = wlcs::seaweed_cell<1>(a3, d, t, y);
            d = wlcs::seaweed_cell<0>(a4, d, b, y);
            d = wlcs::seaweed_cell<1>(a5, d, b, y);
            d = wlcs::seaweed_cell<0>(a6, d, t, y);
            d = wlcs::seaweed_cell<1>(a7, d, t, y);
            a0 ^= d & 1u;  // keeps the column's exit alive
        }
    }
    out[t] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}
#undef WLCS_ISSUE_ROUND
#undef WLCS_ISSUE_ROUND3

}  // namespace

// blocks x (256 k) threads; wave64 VALU instructions per wave and round:
// 16 (kinds 0, 1, 5), 32 (kinds 2, 3) or 40 (kind 4)
hipError_t launch_valu_issue(uint32_t* out, int32_t kind, int32_t blocks, int32_t k, int32_t iters,
                             hipStream_t stream) {
    const dim3 grid((uint32_t)blocks), block((uint32_t)(256 * k));
    if (kind == 0)
        hipLaunchKernelGGL(valu_issue_kernel<0>, grid, block, 0, stream, out, iters);
    else if (kind == 1)
        hipLaunchKernelGGL(valu_issue_kernel<1>, grid, block, 0, stream, out, iters);
    else if (kind == 2)
        hipLaunchKernelGGL(valu_issue_kernel<2>, grid, block, 0, stream, out, iters);
    else if (kind == 3)
        hipLaunchKernelGGL(valu_issue_kernel<3>, grid, block, 0, stream, out, iters);
    else if (kind == 4)
        hipLaunchKernelGGL(valu_issue_kernel<4>, grid, block, 0, stream, out, iters);
    else
        hipLaunchKernelGGL(valu_issue_kernel<5>, grid, block, 0, stream, out, iters);
    return hipGetLastError();
}

}  // namespace wlcs
