// Exact threshold filter for dot lists: the dots (window pairs with
// WLCS >= T) of a plot without combing every strip.
//
// Moving an x-window by one letter drops one letter and adds one, so its LLCS
// with any y-window changes by at most one: |WLCS(i + d, j) - WLCS(i, j)| <=
// |d|.  The host runtime therefore combs only the probe strips -- every h-th
// x-window, starting at half the remainder of (rows - 1) / h so that no row
// lies more than floor(h / 2) rows from a probe -- with the seaweed kernel,
// listing their entries at the lowered threshold T - floor(h / 2).  Every
// other row i has a designated nearest probe p (the lower one on ties), and a
// dot (i, j) implies WLCS(p, j) >= T - |i - p|, so p has listed (p, j).  The kernel below takes each listed probe entry (p, j, v):
// probe entries with v >= T are dots as they stand, and every row i whose
// designated probe is p with v + |i - p| >= T is a candidate, evaluated
// exactly and listed if it reaches T.  Each window pair is considered from one
// probe only, so the list has no duplicates, and no dot is missed.
//
// Candidates are evaluated with the bit-parallel LCS (Crochemore et al.,
// the recurrence of blcs.hip): the candidates of one probe entry share the
// y-window, so each lane builds that window's letter masks once (in LDS, one
// column per lane) and runs the w-step recurrence over the letters of each
// candidate x-window.  Both windows' codes are read 32 at a time into
// registers with 17 aligned 32-bit loads, so the steps wait on LDS only.
//
// If the probe entries exceed the probe list, the kernel lists nothing and
// raises a flag instead; a gated launch of the plain dot list over every strip
// (which returns at once unless the flag is up) then gives the exact list.
#include <algorithm>

#include "kernels.hpp"
#include "packed.hpp"

namespace wlcs {
namespace {

template <int NW>
__device__ __forceinline__ void bl_step(uint32_t (&v)[NW], const uint32_t* m) {
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

// Codes per register chunk of a window (two 16-bit codes per register).
constexpr int kChunk = 32;

// kChunk 16-bit codes starting at element pos of a16, two per register (code
// 2k in the low half of c[k]), read as kChunk / 2 + 1 aligned 32-bit loads:
// an odd start is realigned per lane with v_alignbit.  Reads elements up to
// pos + kChunk + 1.
__device__ __forceinline__ void load_chunk(const uint16_t* __restrict__ a16, int64_t pos, uint32_t (&c)[kChunk / 2]) {
    const uint32_t* wp = (const uint32_t*)(a16 + (pos & ~(int64_t)1));
    const uint32_t sh = (uint32_t)(pos & 1) * 16u;
    uint32_t prev = wp[0];
#pragma unroll
    for (int k = 0; k < kChunk / 2; ++k) {
        const uint32_t next = wp[k + 1];
        c[k] = __builtin_amdgcn_alignbit(next, prev, sh);
        prev = next;
    }
}

// Append one dot to the caller's list (counted past the capacity).
__device__ __forceinline__ void append(DotRec* dots, int64_t cap, unsigned long long* count, int64_t i, int64_t j,
                                       uint32_t v, int w) {
    const unsigned long long k = atomicAdd(count, 1ull);
    if (dots && k < (unsigned long long)cap) {
        uint32_t* rec = (uint32_t*)(dots + k);
        rec[0] = (uint32_t)i;
        rec[1] = (uint32_t)j;
        rec[2] = v | ((uint32_t)(2 * w - 2 * (int)v) << 16);
    }
}

template <int NW>
__global__ __launch_bounds__(64) void candidates_kernel(const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32,
                                                        const DotRec* __restrict__ probe, int64_t probe_cap,
                                                        const unsigned long long* __restrict__ probe_count,
                                                        int64_t rows, int64_t first, int32_t w, int32_t sigma,
                                                        int32_t h,
                                                        int32_t threshold, DotRec* __restrict__ dots, int64_t dot_cap,
                                                        unsigned long long* __restrict__ dot_count,
                                                        uint32_t* __restrict__ fallback) {
    extern __shared__ uint32_t masks[];  // [sigma][NW][64 lanes]
    const int lane = threadIdx.x;
    const unsigned long long n = *probe_count;
    if (n > (unsigned long long)probe_cap) {  // some probe entries were not stored
        if (blockIdx.x == 0 && lane == 0) *fallback = 1u;
        return;
    }
    const int H = h / 2;
    const int64_t last = first + (rows - 1 - first) / h * h;  // the last probe row
    const int64_t stride = (int64_t)gridDim.x * 64;
    for (int64_t e = (int64_t)blockIdx.x * 64 + lane; e < (int64_t)n; e += stride) {
        const DotRec r = probe[e];
        const int64_t p = r.i, j = r.j;
        const int v = r.wlcs;
        if (v >= threshold) append(dots, dot_cap, dot_count, p, j, (uint32_t)v, w);
        if (v + H < threshold) continue;  // no row within reach can get there
        // letter masks of the y-window at j: bit q of word k of M[c] <=> y[j + 32k + q] is c
        for (int c = 0; c < sigma; ++c)
#pragma unroll
            for (int k = 0; k < NW; ++k) masks[(c * NW + k) * 64 + lane] = 0u;
#pragma unroll
        for (int k = 0; k < NW; ++k) {  // one chunk of 32 letters per mask word
            uint32_t yc[kChunk / 2];
            load_chunk((const uint16_t*)yg32, j + kChunk * k, yc);
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                if (kChunk * k + q >= w) break;  // uniform
                const uint32_t g = (yc[q >> 1] >> ((q & 1) * 16)) & 0xFFFFu;
                const uint32_t c = (64u - (g >> kCodeShift)) & 63u;
                masks[(c * NW + k) * 64 + lane] |= 1u << q;
            }
        }
        for (int d = -H; d <= H; ++d) {
            const int64_t i = p + d;
            if (d == 0 || i < 0 || i >= rows) continue;
            // the designated probe of row i (a probe row is its own, so it
            // is never a candidate of another probe)
            int64_t near;
            if (i <= first) {
                near = first;
            } else if (i >= last) {
                near = last;
            } else {
                const int64_t lo = first + (i - first) / h * h;
                near = i - lo <= lo + h - i ? lo : lo + h;
            }
            if (near != p || v + (d < 0 ? -d : d) < threshold) continue;
            uint32_t vec[NW];
#pragma unroll
            for (int k = 0; k < NW; ++k) vec[k] = 0xFFFFFFFFu;
            for (int a0 = 0; a0 < w; a0 += kChunk) {  // the x-window's letters, a chunk at a time
                uint32_t xc[kChunk / 2];
                load_chunk(xf, i + a0, xc);
#pragma unroll
                for (int a = 0; a < kChunk; ++a) {
                    if (a0 + a >= w) break;  // uniform
                    const uint32_t c = ((xc[a >> 1] >> ((a & 1) * 16)) & 0xFFFFu) >> kCodeShift;
                    uint32_t m[NW];
#pragma unroll
                    for (int k = 0; k < NW; ++k) m[k] = masks[(c * NW + k) * 64 + lane];
                    bl_step<NW>(vec, m);
                }
            }
            uint32_t ones = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k) {
                const int bits = w - 32 * k;
                const uint32_t mask = bits >= 32 ? 0xFFFFFFFFu : (bits > 0 ? (1u << bits) - 1u : 0u);
                ones += (uint32_t)__popc(vec[k] & mask);
            }
            const uint32_t val = (uint32_t)w - ones;
            if ((int)val >= threshold) append(dots, dot_cap, dot_count, i, j, val, w);
        }
    }
}

// The grid: every single-wave workgroup that fits on the device at once (the
// letter masks take sigma x NW words of LDS per lane, the registers allow up
// to eight waves per SIMD), at most 32 per CU.  A candidate's steps wait on
// LDS and on each other: with one wave per SIMD the VALU stood idle four
// cycles in five.  The entries are split evenly over the grid, so no
// workgroup of it may wait for another to finish.
template <int NW>
hipError_t candidates_nw(const FilterArgs& f, hipStream_t stream) {
    const size_t lds = (size_t)f.sigma * NW * 64 * sizeof(uint32_t);  // <= 63 * 8 * 256 bytes
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)candidates_kernel<NW>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)candidates_kernel<NW>, 64, lds);
    if (e != hipSuccess) return e;
    const int64_t grid = (int64_t)std::max(1, std::min(per_cu, 32)) * f.cus;
    hipLaunchKernelGGL((candidates_kernel<NW>), dim3((uint32_t)grid), dim3(64), lds, stream, f.xf,
                       (const uint32_t*)f.yg, f.probe, f.probe_cap, f.probe_count, f.rows, f.first, f.w, f.sigma, f.h,
                       f.threshold, f.dots, f.dot_cap, f.dot_count, f.fallback);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_candidates(const FilterArgs& f, hipStream_t stream) {
    if (f.cus <= 0) return hipSuccess;
    switch ((f.w + 31) / 32) {
        case 1: return candidates_nw<1>(f, stream);
        case 2: return candidates_nw<2>(f, stream);
        case 3: return candidates_nw<3>(f, stream);
        case 4: return candidates_nw<4>(f, stream);
        case 5: return candidates_nw<5>(f, stream);
        case 6: return candidates_nw<6>(f, stream);
        case 7: return candidates_nw<7>(f, stream);
        default: return candidates_nw<8>(f, stream);
    }
}

}  // namespace wlcs
