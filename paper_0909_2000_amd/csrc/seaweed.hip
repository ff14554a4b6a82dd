// Windowed seaweed combing for alignment plots on gfx950.
//
// Method (Krusche & Tiskin, Theorem 3.1): for each x-window x[i..i+w) comb the
// strip of height w and width n of the alignment dag (Section 2) column by
// column.  A seaweed starts at the top of every column and at the left of every
// row; in each cell the seaweed arriving from the left (s) and the one arriving
// from the top (t) either turn (match cell, or a mismatch cell whose pair has
// crossed before) or cross (mismatch cell, not crossed yet).  Labelling
// seaweeds by start column, with left starts below all top starts, a match
// cell sends s down and t right, a mismatch cell sends max(s, t) down and
// min(s, t) right.  By Theorem 2.1 the LLCS of the x-window and the y-window
// starting at j is w minus the number of seaweeds that start at the top of
// columns j..j+w-1 and leave the bottom inside the same columns; the count
// slides along y in O(1) per column.
//
// GPU mapping (one 64-lane wavefront per workgroup; strips of 65..128 rows
// are split over two waves and strips of 129..255 rows over a chain of four,
// see seaweed_kernel_rsplit and seaweed_kernel_wide):
//  * lane = strip: the 64 lanes of a wave comb 64 consecutive x-windows, so
//    the y letter of the current column is the same for every lane (it arrives
//    through scalar loads, one column ahead) and the x letters of each lane's
//    w rows sit in registers.  The w labels of the seaweeds travelling right
//    (one per row) stay in VGPRs for the whole tile.
//  * two tiles per lane: each 32-bit register holds two 16-bit labels, the
//    low half for tile A of the strip and the high half for tile B (a
//    disjoint y range), so every instruction of the cell advances two cells.
//  * the cell in four instructions: Z = f(x) + g(y) is 0 on a match and
//    >= 1024 on a mismatch (letter codes of kernels.hpp), labels are < 1024,
//        down  = max(s, min(t, Z))          (match: s; mismatch: max(s, t))
//        right = s ^ t ^ down               (the other of the two, in one
//                                            three-input v_bitop3_b32)
//    The x code of a row is read from one half of a shared register through
//    the op_sel modifiers of v_pk_add_u16.
//  * labels are start columns relative to a moving origin and are clamped at
//    0 every kRebase windows: a monotone relabelling commutes with the
//    max/min of the cell, and a seaweed that started before the oldest open
//    window can no longer be counted (the span bound behind Propositions 3.3
//    and 3.4), so 10 bits suffice for any w <= 255.
//  * y tiles: every x-window is combed afresh from the first column of each
//    tile of T windows (T + w - 1 columns); windows starting inside the tile
//    only depend on columns from the tile start on.
//  * the count: the exit at column l with start s counts for the windows
//    l-w+1..s when its span l - s is below w.  A running total per tile adds
//    each such exit and removes it again at window s + 1 through a ring of
//    pending marks (one bit per start column) kept in LDS.  This replaces the
//    paper's min-heap, which deletes at most one seaweed per column.
//  * output: per 4 windows the two W bytes of each tile are packed into
//    dwords and staged in LDS; every 32 windows each lane stores its strip's
//    32 bytes per tile (16-byte or 4-byte stores when the row stride allows,
//    else the block is transposed through LDS into coalesced byte stores),
//    plus the bitmap word and the uint16 indel distances when requested.
//  * strided and sparse plots (the step size of Section 3, the dot plot of
//    Section 1): every x-window at a multiple of hx is a strip (hx x codes
//    between strips), every window is combed and counted, and each flushed
//    block stores only its windows at multiples of hy, and/or appends the
//    windows at or above the threshold to a list of dots.
#include "seaweed_unit.hpp"

namespace wlcs {
namespace {

template <int WC, bool EXACT, int WS, bool SP, bool DL = false>
__global__ __launch_bounds__(64, DL ? min_waves_per_simd_dl(WC) : min_waves_per_simd(WC)) void seaweed_kernel(
                                                                              const uint16_t* __restrict__ xf,
                                                                              const uint32_t* __restrict__ yg32,
                                                                              uint8_t* __restrict__ out,
                                                                              uint32_t* __restrict__ bm32,
                                                                              uint16_t* __restrict__ indel,
                                                                              DotRec* __restrict__ dots,
                                                                              unsigned long long* __restrict__ dot_count,
                                                                              Geom g,
                                                                              const uint32_t* __restrict__ gate) {
    if constexpr (SP) {
        if (gate && *gate == 0u) return;  // a launch kept only in case an earlier pass asks for it
    }
    __shared__ uint32_t ring[ring_words(WC) * 64];
    __shared__ uint32_t stage[stage_dwords(WC, WS)];
    // pair-major order: the last tile pair of every strip block (usually
    // shorter: the plot's width is rarely a multiple of two tiles) comes last
    // and fills the tail of the launch
    const int64_t nblocks = (g.rows + 63) / 64;
    const int64_t unit = blockIdx.x;
    const int pr = (int)(unit / nblocks);
    const int64_t sb = unit - (int64_t)pr * nblocks;
    comb_unit<WC, EXACT, WS, SP, DL>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr, ring, stage);
}

// Score plots of more than kDlSplitRows rows: two waves per strip (the upper
// and the lower pair slots, see comb_unit), one unit per workgroup of 128.
template <int WC>
__global__ __launch_bounds__(128, min_waves_per_simd_dl_split(WC)) void seaweed_kernel_split(
    const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32, uint8_t* __restrict__ out,
    uint32_t* __restrict__ bm32, uint16_t* __restrict__ indel, DotRec* __restrict__ dots,
    unsigned long long* __restrict__ dot_count, Geom g) {
    __shared__ uint32_t ring[ring_words(WC) * 64];
    __shared__ uint32_t stage[stage_dwords(WC, 2)];
    __shared__ uint32_t hand[kDlHandDwords];
    const int64_t nblocks = (g.rows + 63) / 64;
    const int64_t unit = blockIdx.x;
    const int pr = (int)(unit / nblocks);
    const int64_t sb = unit - (int64_t)pr * nblocks;
    if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0)
        comb_unit<WC, false, 2, false, true, 1>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr, ring, stage,
                                                 hand);
    else
        comb_unit<WC, false, 2, false, true, 2>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr, ring, stage,
                                                 hand);
}

// Plots in the 128-row class: two waves per strip (the upper and the lower
// half of the rows, see comb_unit), one unit per workgroup of 128.
template <int WC, bool EXACT, bool SP>
__global__ __launch_bounds__(128, min_waves_per_simd_split(WC)) void seaweed_kernel_rsplit(
    const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32, uint8_t* __restrict__ out,
    uint32_t* __restrict__ bm32, uint16_t* __restrict__ indel, DotRec* __restrict__ dots,
    unsigned long long* __restrict__ dot_count, Geom g, const uint32_t* __restrict__ gate) {
    if constexpr (SP) {
        if (gate && *gate == 0u) return;
    }
    __shared__ uint32_t ring[ring_words(WC) * 64];
    __shared__ uint32_t stage[stage_dwords(WC, 1)];
    __shared__ uint32_t hand[kDlHandDwords];
    const int64_t nblocks = (g.rows + 63) / 64;
    const int64_t unit = blockIdx.x;
    const int pr = (int)(unit / nblocks);
    const int64_t sb = unit - (int64_t)pr * nblocks;
    if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0)
        comb_unit<WC, EXACT, 1, SP, false, 1>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr, ring, stage,
                                               hand);
    else
        comb_unit<WC, EXACT, 1, SP, false, 2>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr, ring, stage,
                                               hand);
}

// Plots in the 256-row class: a chain of kWideWaves waves per strip
// (wide_rows), one unit per workgroup.
template <bool SP>
__global__ __launch_bounds__(64 * kWideWaves, 3) void seaweed_kernel_wide(
    const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32, uint8_t* __restrict__ out,
    uint32_t* __restrict__ bm32, uint16_t* __restrict__ indel, DotRec* __restrict__ dots,
    unsigned long long* __restrict__ dot_count, Geom g, const uint32_t* __restrict__ gate) {
    static_assert(kWideWaves == 4, "one case per wave of the chain");
    if constexpr (SP) {
        if (gate && *gate == 0u) return;
    }
    __shared__ uint32_t ring[ring_words(256) * 64];
    __shared__ uint32_t stage[stage_dwords(256, 1)];
    __shared__ uint32_t hand[(kWideWaves - 1) * kDlHandDwords];
    const int64_t nblocks = (g.rows + 63) / 64;
    const int64_t unit = blockIdx.x;
    const int pr = (int)(unit / nblocks);
    const int64_t sb = unit - (int64_t)pr * nblocks;
    switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
        case 0:
            comb_unit<256, false, 1, SP, false, 1, kWideWaves>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr,
                                                               ring, stage, hand);
            break;
        case 1:
            comb_unit<256, false, 1, SP, false, 2, kWideWaves>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr,
                                                               ring, stage, hand);
            break;
        case 2:
            comb_unit<256, false, 1, SP, false, 3, kWideWaves>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr,
                                                               ring, stage, hand);
            break;
        default:
            comb_unit<256, false, 1, SP, false, 4, kWideWaves>(xf, yg32, out, bm32, indel, dots, dot_count, g, sb, pr,
                                                               ring, stage, hand);
            break;
    }
}

__global__ void zero_u64(unsigned long long* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

template <int WC, int WS, bool SP>
void launch_ws(const PlotArgs& a, const Geom& g, uint32_t units, hipStream_t stream) {
    const uint32_t* yg32 = (const uint32_t*)a.yg;
    if constexpr (WS == 1 && WC == 256) {
        hipLaunchKernelGGL((seaweed_kernel_wide<SP>), dim3(units), dim3(64 * kWideWaves), 0, stream, a.xf, yg32,
                           a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g, a.gate);
    } else if constexpr (WS == 1 && general_split(WC)) {
        if (a.w == WC)
            hipLaunchKernelGGL((seaweed_kernel_rsplit<WC, true, SP>), dim3(units), dim3(128), 0, stream, a.xf, yg32,
                               a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g, a.gate);
        else
            hipLaunchKernelGGL((seaweed_kernel_rsplit<WC, false, SP>), dim3(units), dim3(128), 0, stream, a.xf, yg32,
                               a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g, a.gate);
    } else {
        if constexpr (WC < 256) {  // windows are at most 255 long: none fills the 256-row class
            if (a.w == WC) {
                hipLaunchKernelGGL((seaweed_kernel<WC, true, WS, SP>), dim3(units), dim3(64), 0, stream, a.xf, yg32,
                                   a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g, a.gate);
                return;
            }
        }
        hipLaunchKernelGGL((seaweed_kernel<WC, false, WS, SP>), dim3(units), dim3(64), 0, stream, a.xf, yg32,
                           a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g, a.gate);
    }
}

// score plots: the separator schedule in the class of the window rounded up
// to 2 * kDlSlots rows
template <int WC>
hipError_t launch_dl(const PlotArgs& a, hipStream_t stream) {
    const int64_t nblocks = (a.rows + 63) / 64;
    const int64_t units = nblocks * a.npairs;
    if (units <= 0) return hipSuccess;
    if (units > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const Geom g = geom_of(a);
    if constexpr (dl_split(WC))
        hipLaunchKernelGGL((seaweed_kernel_split<WC>), dim3((uint32_t)units), dim3(128), 0, stream, a.xf,
                           (const uint32_t*)a.yg, a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g);
    else
        hipLaunchKernelGGL((seaweed_kernel<WC, false, 2, false, true>), dim3((uint32_t)units), dim3(64), 0, stream,
                           a.xf, (const uint32_t*)a.yg, a.wlcs, a.bitmap32, a.indel, a.dots, a.dot_count, g, a.gate);
    return hipGetLastError();
}

// the class wc (a multiple of 2 * kDlSlots up to 256) picks its kernel
template <int WC>
hipError_t dispatch_dl(const PlotArgs& a, int wc, hipStream_t stream) {
    if constexpr (WC >= 256) {
        return launch_dl<256>(a, stream);
    } else {
        if (wc <= WC) return launch_dl<WC>(a, stream);
        return dispatch_dl<WC + 2 * kDlSlots>(a, wc, stream);
    }
}

template <int WC>
hipError_t launch_wc(const PlotArgs& a, hipStream_t stream) {
    const int64_t nblocks = (a.rows + 63) / 64;
    const int64_t units = nblocks * a.npairs;
    if (units <= 0) return hipSuccess;
    if (units > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const Geom g = geom_of(a);
    if (a.hy > 1 || a.dot_count)
        launch_ws<WC, 1, true>(a, g, (uint32_t)units, stream);
    else
        launch_ws<WC, 1, false>(a, g, (uint32_t)units, stream);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u64, dim3(1), dim3(64), 0, stream, p);
    return hipGetLastError();
}

hipError_t launch_seaweed(const PlotArgs& a, hipStream_t stream) {
    if (a.ws == 2) {  // blown-up strings: even window, separator rows and columns
        if (a.w % 2 || a.w < 2 || a.w > 256) return hipErrorInvalidValue;
        return dispatch_dl<2 * kDlSlots>(a, (a.w + 2 * kDlSlots - 1) / (2 * kDlSlots) * (2 * kDlSlots), stream);
    }
    switch (w_class(a.w)) {
        case 16: return launch_wc<16>(a, stream);
        case 32: return launch_wc<32>(a, stream);
        case 64: return launch_wc<64>(a, stream);
        case 128: return launch_wc<128>(a, stream);
        default: return launch_wc<256>(a, stream);
    }
}

}  // namespace wlcs
