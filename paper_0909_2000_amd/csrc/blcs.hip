// Bit-parallel LCS per window pair on gfx950: the BLCS baseline of the
// paper's experiments (Section 4 compares against Crochemore et al.'s
// bit-vector LCS, 2001).
//
// For a fixed x-window a (|a| = w) and a y-window b, a w-bit vector V starts
// with every bit set and takes, for each letter b_q in turn,
//     U = V & M[b_q],    V = (V + U) | (V - U),
// where bit p of M[c] is set iff a_p = c.  LLCS(a, b) is then the number of
// zero bits among the low w bits of V.  Bits above w never reach the low
// ones (carries and borrows only travel upwards), so the vector is kept in
// whole 32-bit words and the high bits are simply ignored at the end.
//
// Mapping: lane = x-window (64 per wave), so the y letter of a step is
// wave-uniform; each lane's letter masks M[c] (NW words each) sit in LDS, one
// column per lane.  A step costs 4 VALU instructions per word (and, add with
// carry, subtract with borrow, or) plus the mask read; a window pair costs w
// steps.  Windows run in chunks of the y range per workgroup; two windows are
// advanced together so that their dependency chains interleave.
#include "kernels.hpp"
#include "packed.hpp"

namespace wlcs {
namespace {

constexpr int kBlcsChunk = 256;  // y-windows per unit

// One step of the recurrence on an NW-word vector.
template <int NW>
__device__ __forceinline__ void blcs_step(uint32_t (&v)[NW], const uint32_t* m) {
    uint32_t carry = 0, borrow = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t u = v[k] & m[k];
        uint32_t co, bo;
        const uint32_t sum = __builtin_addc(v[k], u, carry, &co);
        const uint32_t dif = __builtin_subc(v[k], u, borrow, &bo);
        carry = co;
        borrow = bo;
        v[k] = sum | dif;
    }
}

template <int NW>
__device__ __forceinline__ uint32_t zeros_low(const uint32_t (&v)[NW], int w) {
    uint32_t ones = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int bits = w - 32 * k;
        const uint32_t mask = bits >= 32 ? 0xFFFFFFFFu : (bits > 0 ? (1u << bits) - 1u : 0u);
        ones += (uint32_t)__popc(v[k] & mask);
    }
    return (uint32_t)w - ones;
}

template <int NW>
__global__ __launch_bounds__(64) void blcs_kernel(const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32,
                                                  uint8_t* __restrict__ out, int64_t ld, int64_t rows, int64_t cols,
                                                  int32_t w, int32_t sigma, int32_t nchunks, int64_t xstride,
                                                  int64_t hy) {
    extern __shared__ uint32_t masks[];  // [sigma][NW][64 lanes]
    const int lane = threadIdx.x;
    const int64_t unit = blockIdx.x;
    const int64_t sb = unit / nchunks;
    const int64_t ch = unit - sb * nchunks;
    const int64_t s = sb * 64 + lane;
    const int64_t sx = s < rows ? s : rows - 1;  // lanes past the last strip copy the last one

    // this lane's masks: bit p of word k of M[c] <=> x letter 32k + p is c
    for (int c = 0; c < sigma; ++c)
#pragma unroll
        for (int k = 0; k < NW; ++k) masks[(c * NW + k) * 64 + lane] = 0u;
    const uint16_t* xp = xf + sx * xstride;
    for (int p = 0; p < w; ++p) {
        const uint32_t c = (uint32_t)xp[p] >> kCodeShift;
        masks[(c * NW + (p >> 5)) * 64 + lane] |= 1u << (p & 31);
    }

    const const_u32p y = as_const(yg32);
    auto ycode = [&](int64_t q) -> uint32_t {  // letter code of y at q (wave-uniform)
        const uint32_t g = (y[q >> 1] >> ((uint32_t)(q & 1) * 16u)) & 0xFFFFu;
        return (64u - (g >> kCodeShift)) & 63u;
    };
    const int64_t j0 = ch * kBlcsChunk;
    const int64_t j1 = j0 + kBlcsChunk < cols ? j0 + kBlcsChunk : cols;
    for (int64_t j = j0; j < j1; j += 2) {
        const bool two = j + 1 < j1;  // uniform
        const int64_t ya = j * hy, yb = (two ? j + 1 : j) * hy;
        uint32_t va[NW], vb[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) va[k] = vb[k] = 0xFFFFFFFFu;
#pragma unroll 2
        for (int q = 0; q < w; ++q) {
            const uint32_t ca = __builtin_amdgcn_readfirstlane(ycode(ya + q));
            const uint32_t cb = __builtin_amdgcn_readfirstlane(ycode(yb + q));
            uint32_t ma[NW], mb[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                ma[k] = masks[(ca * NW + k) * 64 + lane];
                mb[k] = masks[(cb * NW + k) * 64 + lane];
            }
            blcs_step<NW>(va, ma);
            blcs_step<NW>(vb, mb);
        }
        if (s < rows) {
            out[s * ld + j] = (uint8_t)zeros_low<NW>(va, w);
            if (two) out[s * ld + j + 1] = (uint8_t)zeros_low<NW>(vb, w);
        }
    }
}

template <int NW>
hipError_t blcs_nw(const PlotArgs& a, uint8_t* wout, int64_t ldo, hipStream_t stream) {
    const int64_t nblocks = (a.rows + 63) / 64;
    const int64_t nchunks = (a.cols + kBlcsChunk - 1) / kBlcsChunk;
    const int64_t units = nblocks * nchunks;
    if (units <= 0) return hipSuccess;
    if (units > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const size_t lds = (size_t)a.sigma * NW * 64 * sizeof(uint32_t);  // <= 63 * 8 * 256 bytes
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)blcs_kernel<NW>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((blcs_kernel<NW>), dim3((uint32_t)units), dim3(64), lds, stream, a.xf,
                       (const uint32_t*)a.yg, wout, ldo, a.rows, a.cols, a.w, a.sigma, (int32_t)nchunks,
                       a.xstride, a.hy);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blcs(const PlotArgs& a, hipStream_t stream) {
    // the plot is written first; epilogues (if any) read it back
    uint8_t* wout = a.wlcs;
    int64_t ldo = a.ld;
    hipError_t e = hipSuccess;
    if (!wout) {
        e = hipMallocAsync((void**)&wout, (size_t)(a.rows * a.cols), stream);
        if (e != hipSuccess) return e;
        ldo = a.cols;
    }
    const int nw = (a.w + 31) / 32;
    e = nw <= 1 ? blcs_nw<1>(a, wout, ldo, stream)
        : nw <= 2 ? blcs_nw<2>(a, wout, ldo, stream)
        : nw <= 4 ? blcs_nw<4>(a, wout, ldo, stream)
                  : blcs_nw<8>(a, wout, ldo, stream);
    if (e == hipSuccess) e = launch_epilogue(a, wout, ldo, stream);
    if (!a.wlcs) {
        const hipError_t e2 = hipFreeAsync(wout, stream);
        if (e == hipSuccess) e = e2;
    }
    return e;
}

}  // namespace wlcs
