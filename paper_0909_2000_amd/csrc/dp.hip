// Plain per-window dynamic program on gfx950: the paper's O(m n w^2)
// baseline (Section 2), every window pair solved independently by
//     L[p][q] = L[p-1][q-1] + 1                 if x letter == y letter
//             = max(L[p-1][q], L[p][q-1])       otherwise.
// Because L[p-1][q], L[p][q-1] <= L[p-1][q-1] + 1, the recurrence equals
// max(L[p-1][q], L[p][q-1], L[p-1][q-1] + [match]); with the letter codes of
// kernels.hpp the match term is a saturating subtract of Z from L[p-1][q-1]+1.
//
// Mapping: lane = x-window (64 strips per wave), two y-windows per lane in the
// 16-bit halves; the DP column over the w rows lives in registers and is swept
// across the w columns of the y-window, whose letters are wave-uniform.
// Also here: the stand-alone epilogue (bitmap, indel) used by this path and
// the letter-encoding kernel shared by both paths.
#include "kernels.hpp"
#include "packed.hpp"

namespace wlcs {
namespace {

constexpr int kDpChunk = 64;  // y-windows per half per unit

template <int WC, bool EXACT>
__global__ __launch_bounds__(64) void dp_kernel(const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32,
                                                uint8_t* __restrict__ wout, int64_t ldo, int64_t rows, int64_t cols,
                                                int32_t wrt, int32_t nchunks, int64_t xstride, int64_t hy) {
    const int lane = threadIdx.x;
    const int64_t unit = blockIdx.x;
    const int64_t sb = unit / nchunks;
    const int cp = (int)(unit - sb * nchunks);
    const int64_t s = sb * 64 + lane;
    const int64_t jA0 = (int64_t)cp * 2 * kDpChunk, jB0 = jA0 + kDpChunk;
    const int w = EXACT ? WC : wrt;
    const uint32_t one2 = 0x00010001u;

    // output (s, j) compares the x-window at s * xstride with the y-window
    // at j * hy; lanes and windows past the end compute copies of the last
    // ones, which are never stored
    uint32_t xc[WC / 2];
    {
        const uint16_t* xp = xf + (s < rows ? s : rows - 1) * xstride;
#pragma unroll
        for (int j = 0; j < WC / 2; ++j) xc[j] = (uint32_t)xp[2 * j] | ((uint32_t)xp[2 * j + 1] << 16);
    }
    for (int jj = 0; jj < kDpChunk; ++jj) {
        const int64_t jA = jA0 + jj, jB = jB0 + jj;
        if (jA >= cols) break;
        const int64_t yA = jA * hy, yB = (jB < cols ? jB : cols - 1) * hy;
        uint32_t col[WC];  // col[p] = L[p+1][q-1], both windows
#pragma unroll
        for (int p = 0; p < WC; ++p) col[p] = 0;
        for (int q = 0; q < w; ++q) {
            const uint32_t Y = u16_at(yg32, yA + q) | (u16_at(yg32, yB + q) << 16);
            uint32_t up = 0, diag = 0;  // L[p][q], L[p][q-1]
#pragma unroll
            for (int p = 0; p < WC; ++p) {
                if (EXACT || p < w) {
                    const uint32_t left = col[p];
                    const uint32_t v = (p & 1) ? dp_cell<1>(up, left, diag, xc[p >> 1], Y, one2)
                                               : dp_cell<0>(up, left, diag, xc[p >> 1], Y, one2);
                    diag = left;
                    col[p] = v;
                    up = v;
                }
            }
        }
        uint32_t res = 0;
#pragma unroll
        for (int p = 0; p < WC; ++p)
            if (p == w - 1) res = col[p];
        if (s < rows) {
            wout[s * ldo + jA] = (uint8_t)(res & 0xFFu);
            if (jB < cols) wout[s * ldo + jB] = (uint8_t)(res >> 16);
        }
    }
}

// bitmap, indel and dot list from a finished plot; one wave per 64 windows of
// a row.  Dots (entries >= threshold) are appended with one vector atomic per
// wave that has any; entry (r, j) is the window pair (r * xstride, j * hy).
__global__ __launch_bounds__(256) void epilogue_kernel(const uint8_t* __restrict__ plot, int64_t ld,
                                                       int64_t rows, int64_t cols, int32_t w,
                                                       uint32_t* __restrict__ bitmap32, int64_t ldw32,
                                                       int32_t threshold, uint16_t* __restrict__ indel,
                                                       int64_t ld_indel, DotRec* __restrict__ dots, int64_t dot_cap,
                                                       unsigned long long* __restrict__ dot_count, int64_t xstride,
                                                       int64_t hy) {
    const int64_t words = (cols + 63) / 64;
    const int64_t gw = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (gw >= rows * words) return;  // whole wave exits together
    const int lane = threadIdx.x & 63;
    const int64_t r = gw / words, q = gw - r * words;
    const int64_t j = q * 64 + lane;
    const bool in = j < cols;
    const int v = in ? plot[r * ld + j] : 0;
    if (indel && in) indel[r * ld_indel + j] = (uint16_t)(2 * w - 2 * v);
    if (bitmap32 || dot_count) {
        const uint64_t bal = __ballot(in && v >= threshold);
        if (bitmap32 && lane == 0) {
            bitmap32[r * ldw32 + 2 * q] = (uint32_t)bal;
            bitmap32[r * ldw32 + 2 * q + 1] = (uint32_t)(bal >> 32);
        }
        if (dot_count && bal) {  // uniform
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(dot_count, (unsigned long long)__popcll(bal));
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)base, 0);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(base >> 32), 0);
            const unsigned long long k = (((unsigned long long)hi << 32) | lo) + __popcll(bal & ((1ull << lane) - 1ull));
            if (dots && in && v >= threshold && k < (unsigned long long)dot_cap) {
                uint32_t* rec = (uint32_t*)(dots + k);
                rec[0] = (uint32_t)(r * xstride);
                rec[1] = (uint32_t)(j * hy);
                rec[2] = (uint32_t)v | ((uint32_t)(2 * w - 2 * v) << 16);
            }
        }
    }
}

template <int WC>
hipError_t dp_wc(const PlotArgs& a, uint8_t* wout, int64_t ldo, hipStream_t stream) {
    const int64_t nblocks = (a.rows + 63) / 64;
    const int64_t nchunks = (a.cols + 2 * kDpChunk - 1) / (2 * kDpChunk);
    const int64_t units = nblocks * nchunks;
    if (units <= 0) return hipSuccess;
    if (units > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const uint32_t* yg32 = (const uint32_t*)a.yg;
    if (a.w == WC)
        hipLaunchKernelGGL((dp_kernel<WC, true>), dim3((uint32_t)units), dim3(64), 0, stream, a.xf, yg32, wout, ldo,
                           a.rows, a.cols, a.w, (int32_t)nchunks, a.xstride, a.hy);
    else
        hipLaunchKernelGGL((dp_kernel<WC, false>), dim3((uint32_t)units), dim3(64), 0, stream, a.xf, yg32, wout,
                           ldo, a.rows, a.cols, a.w, (int32_t)nchunks, a.xstride, a.hy);
    return hipGetLastError();
}

struct Map256 {
    uint8_t m[256];
};

// Letters -> codes.  With a separator code (sep >= 0) the string is first
// blown up as in Section 2's reduction of the alignment score: the separator
// letter goes before every letter, so code i of the output belongs to
// separator (i even) or letter i/2 (i odd).
__global__ void encode_kernel(const uint8_t* __restrict__ raw, int64_t len, Map256 map, int x_side, int sep,
                              uint16_t* __restrict__ out, int64_t out_len) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < out_len;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t c;
        if (sep < 0) c = i < len ? map.m[raw[i]] : 0u;
        else c = i < 2 * len ? ((i & 1) ? map.m[raw[i >> 1]] : (uint32_t)sep) : 0u;
        out[i] = x_side ? f_code(c) : g_code(c);
    }
}

}  // namespace

hipError_t launch_dp(const PlotArgs& a, hipStream_t stream) {
    // the DP writes the plot first; epilogues (if any) read it back
    uint8_t* wout = a.wlcs;
    int64_t ldo = a.ld;
    hipError_t e = hipSuccess;
    const bool epi = a.bitmap32 || a.indel || a.dot_count;
    if (!wout) {
        e = hipMallocAsync((void**)&wout, (size_t)(a.rows * a.cols), stream);
        if (e != hipSuccess) return e;
        ldo = a.cols;
    }
    switch (w_class(a.w)) {
        case 16: e = dp_wc<16>(a, wout, ldo, stream); break;
        case 32: e = dp_wc<32>(a, wout, ldo, stream); break;
        case 64: e = dp_wc<64>(a, wout, ldo, stream); break;
        case 128: e = dp_wc<128>(a, wout, ldo, stream); break;
        default: e = dp_wc<256>(a, wout, ldo, stream); break;
    }
    if (e == hipSuccess && epi) e = launch_epilogue(a, wout, ldo, stream);
    if (!a.wlcs) {
        hipError_t e2 = hipFreeAsync(wout, stream);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

hipError_t launch_epilogue(const PlotArgs& a, const uint8_t* wout, int64_t ldo, hipStream_t stream) {
    if (!a.bitmap32 && !a.indel && !a.dot_count) return hipSuccess;
    const int64_t waves = a.rows * ((a.cols + 63) / 64);
    const int64_t blocks = (waves + 3) / 4;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFFll) return hipErrorInvalidValue;
    hipLaunchKernelGGL(epilogue_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, wout, ldo, a.rows, a.cols,
                       a.w, a.bitmap32, a.ld_words32, a.threshold, a.indel, a.ld_indel, a.dots, a.dot_cap,
                       a.dot_count, a.xstride, a.hy);
    return hipGetLastError();
}

hipError_t launch_encode(const uint8_t* raw, int64_t len, const uint8_t* map256, int x_side, uint16_t* out,
                         int64_t out_len, hipStream_t stream, int sep) {
    if (out_len <= 0) return hipSuccess;
    Map256 m;
    for (int i = 0; i < 256; ++i) m.m[i] = map256[i];
    int64_t blocks = (out_len + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(encode_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, raw, len, m, x_side, sep,
                       out, out_len);
    return hipGetLastError();
}

}  // namespace wlcs
