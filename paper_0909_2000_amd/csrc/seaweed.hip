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
// GPU mapping (one 64-lane wavefront per workgroup):
//  * lane = strip: the 64 lanes of a wave comb 64 consecutive x-windows, so
//    the y letter of the current column is the same for every lane (it arrives
//    through scalar loads, one column ahead) and the x letters of each lane's
//    w rows sit in registers.  The w labels of the seaweeds travelling right
//    (one per row) stay in VGPRs for the whole tile.
//  * two tiles per lane: each 32-bit register holds two 16-bit labels, the
//    low half for tile A of the strip and the high half for tile B (a
//    disjoint y range), so every instruction of the cell advances two cells.
//  * the cell in five packed operations: Z = f(x) + g(y) is 0 on a match and
//    >= 1024 on a mismatch (letter codes of kernels.hpp), labels are < 1024,
//        down  = max(s, min(t, Z))          (match: s; mismatch: max(s, t))
//        right = s ^ t ^ down               (the other of the two)
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
#include "kernels.hpp"
#include "packed.hpp"

namespace wlcs {
namespace {

constexpr int kStagePitch = 9;  // dwords per lane row of the staging buffer (8 + 1 pad)

template <int WC, bool EXACT>
__global__ __launch_bounds__(64) void seaweed_kernel(const uint16_t* __restrict__ xf,
                                                     const uint32_t* __restrict__ yg32,
                                                     uint8_t* __restrict__ out,
                                                     uint32_t* __restrict__ bm32,
                                                     uint16_t* __restrict__ indel, Geom g) {
    constexpr int RW = WC <= 128 ? 16 : 32;  // ring words of 16 start columns each
    __shared__ uint32_t ring[RW * 64];
    __shared__ uint32_t stage[2 * 64 * kStagePitch];

    const int lane = threadIdx.x;
    const int64_t unit = blockIdx.x;
    const int64_t sb = unit / g.npairs;
    const int pr = (int)(unit - sb * g.npairs);
    const int64_t s0 = sb * 64;
    const int64_t tA = (int64_t)(2 * pr) * g.tile;
    const int64_t tB = tA + g.tile;
    const int w = EXACT ? WC : g.w;

    // x letters of this lane's strip, two rows per register
    uint32_t xc[WC / 2];
    {
        const uint16_t* xp = xf + s0 + lane;
#pragma unroll
        for (int j = 0; j < WC / 2; ++j) xc[j] = (uint32_t)xp[2 * j] | ((uint32_t)xp[2 * j + 1] << 16);
    }
    uint32_t h[WC];
#pragma unroll
    for (int k = 0; k < WC; ++k) h[k] = 0;
#pragma unroll
    for (int q = 0; q < RW; ++q) ring[q * 64 + lane] = 0;

    const int64_t restA = g.cols - tA;  // > 0: every launched unit has a non-empty tile A
    const int64_t nA = (restA + 63) / 64 * 64;
    const int nproc = (int)(nA < g.tile ? nA : g.tile);

    int32_t org = -w;   // the seaweed starting at tile column l carries label l - org + 1
    uint32_t cur2 = 0;  // seaweeds counted for the current window, both tiles
    uint32_t ring_pf = 0;
    const uint32_t w2 = pk_rep(w);

    auto yload = [&](int l) -> uint32_t { return u16_at(yg32, tA + l) | (u16_at(yg32, tB + l) << 16); };
    uint32_t ynext = yload(0);

    // Comb column l (tile-relative) through the w rows and update the sliding
    // count; returns w - count for the window starting at l - w + 1.
    auto column = [&](int l) -> uint32_t {
        const uint32_t Y = ynext;
        ynext = yload(l + 1);
        uint32_t t = pk_rep(l - org + 1);
#pragma unroll
        for (int k = 0; k < WC; ++k) {
            if (EXACT || k < w) {
                t = (k & 1) ? seaweed_cell<1>(h[k], t, xc[k >> 1], Y) : seaweed_cell<0>(h[k], t, xc[k >> 1], Y);
            }
        }
        // consume the mark of start column l - w (prefetched after the
        // previous column's marks were set)
        uint32_t f2 = 0;
        const int pc = l - w;
        if (pc >= 0) {
            f2 = (ring_pf >> (pc & 15)) & 0x00010001u;
            if ((pc & 15) == 15) ring[((pc >> 4) & (RW - 1)) * 64 + lane] = 0;
        }
        // p = start - (l - w + 1) lies in [0, w) iff the exit's span is below w
        const uint32_t p2 = pk_sub(t, pk_rep(l - org + 2 - w));
        const uint32_t v2 = pk_min(pk_sub_sat(w2, p2), 0x00010001u);
        const uint32_t pos2 = pk_add(p2, pk_rep(l - w + 1));
        const uint32_t bit2 = pk_shl(v2, pos2);
        const uint32_t wlo = (pos2 >> 4) & (RW - 1), whi = (pos2 >> 20) & (RW - 1);
        atomicOr(&ring[wlo * 64 + lane], bit2 & 0xFFFFu);
        atomicOr(&ring[whi * 64 + lane], bit2 & 0xFFFF0000u);
        cur2 = pk_sub(pk_add(cur2, v2), f2);
        if (pc + 1 >= 0) ring_pf = ring[(((pc + 1) >> 4) & (RW - 1)) * 64 + lane];
        return pk_sub(w2, cur2);
    };

    // warm-up columns: no window is complete yet
    for (int l = 0; l < w - 1; ++l) (void)column(l);

    const uint32_t bm_words = (uint32_t)(((g.cols + 63) >> 6) * 2);
    for (int jb = 0; jb < nproc; jb += 32) {
#pragma unroll 1
        for (int gi = 0; gi < 8; ++gi) {
            const int jj = jb + 4 * gi;
            if (jj > 0 && (jj % kRebase) == 0) {
                const int32_t norg = jj - 1;  // (column jj + w - 1) - w
                const uint32_t d2 = pk_rep(norg - org);
#pragma unroll
                for (int k = 0; k < WC; ++k) h[k] = pk_sub_sat(h[k], d2);
                org = norg;
            }
            const int l = jj + w - 1;
            const uint32_t r0 = column(l);
            const uint32_t r1 = column(l + 1);
            const uint32_t r2 = column(l + 2);
            const uint32_t r3 = column(l + 3);
            const uint32_t wa = (r0 & 0xFFu) | ((r1 & 0xFFu) << 8) | ((r2 & 0xFFu) << 16) | ((r3 & 0xFFu) << 24);
            const uint32_t wb = ((r0 >> 16) & 0xFFu) | (((r1 >> 16) & 0xFFu) << 8) |
                                (((r2 >> 16) & 0xFFu) << 16) | (((r3 >> 16) & 0xFFu) << 24);
            stage[lane * kStagePitch + gi] = wa;
            stage[64 * kStagePitch + lane * kStagePitch + gi] = wb;
        }
        __syncthreads();
        const int64_t s = s0 + lane;  // this lane's strip
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            const int64_t ts = half ? tB : tA;
            const int64_t te = ts + g.tile < g.cols ? ts + g.tile : g.cols;
            const int64_t j0 = ts + jb;
            // windows of this block inside the tile (0 for the padding block
            // that completes the last bitmap word, or past the end of y)
            const int nvalid = (int)(te - j0 < 32 ? (te - j0 > 0 ? te - j0 : 0) : 32);
            if (nvalid == 0 && (uint32_t)(j0 >> 5) >= bm_words) continue;  // uniform
            uint32_t d[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) d[k] = stage[half * 64 * kStagePitch + lane * kStagePitch + k];
            if (out && g.wmode > 0 && nvalid > 0) {
                if (s < g.rows) {
                    uint8_t* row = out + s * g.ld + j0;
                    if (nvalid == 32) {
                        if (g.wmode == 2) {
                            ((uint4*)row)[0] = make_uint4(d[0], d[1], d[2], d[3]);
                            ((uint4*)row)[1] = make_uint4(d[4], d[5], d[6], d[7]);
                        } else {
#pragma unroll
                            for (int k = 0; k < 8; ++k) ((uint32_t*)row)[k] = d[k];
                        }
                    } else {
                        for (int b = 0; b < nvalid; ++b) row[b] = (uint8_t)(d[b >> 2] >> (8 * (b & 3)));
                    }
                }
            }
            if (bm32 && s < g.rows && (uint32_t)(j0 >> 5) < bm_words) {
                uint32_t bits = 0;
#pragma unroll
                for (int b = 0; b < 32; ++b)
                    bits |= (uint32_t)((int)((d[b >> 2] >> (8 * (b & 3))) & 0xFFu) >= g.threshold) << b;
                if (nvalid < 32) bits &= nvalid ? (0xFFFFFFFFu >> (32 - nvalid)) : 0u;
                bm32[s * g.ld_words32 + (j0 >> 5)] = bits;
            }
            if (((out && g.wmode == 0) || indel) && nvalid > 0) {
                // transposed: lanes cover 32 windows of two strips per step
                const int q = lane & 31;
                const uint8_t* sbytes = (const uint8_t*)stage;
#pragma unroll 4
                for (int it = 0; it < 32; ++it) {
                    const int r = 2 * it + (lane >> 5);
                    const int64_t sr = s0 + r;
                    const uint32_t v = sbytes[(half * 64 * kStagePitch + r * kStagePitch) * 4 + q];
                    if (sr < g.rows && q < nvalid) {
                        if (out && g.wmode == 0) out[sr * g.ld + j0 + q] = (uint8_t)v;
                        if (indel) indel[sr * g.ld_indel + j0 + q] = (uint16_t)(2 * w - 2 * (int)v);
                    }
                }
            }
        }
        __syncthreads();
    }
}

template <int WC>
hipError_t launch_wc(const PlotArgs& a, hipStream_t stream) {
    const int64_t nblocks = (a.rows + 63) / 64;
    const int64_t units = nblocks * a.npairs;
    if (units <= 0) return hipSuccess;
    if (units > 0x7FFFFFFFll) return hipErrorInvalidValue;
    const Geom g = geom_of(a);
    const uint32_t* yg32 = (const uint32_t*)a.yg;
    if (a.w == WC)
        hipLaunchKernelGGL((seaweed_kernel<WC, true>), dim3((uint32_t)units), dim3(64), 0, stream, a.xf, yg32,
                           a.wlcs, a.bitmap32, a.indel, g);
    else
        hipLaunchKernelGGL((seaweed_kernel<WC, false>), dim3((uint32_t)units), dim3(64), 0, stream, a.xf, yg32,
                           a.wlcs, a.bitmap32, a.indel, g);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_seaweed(const PlotArgs& a, hipStream_t stream) {
    switch (w_class(a.w)) {
        case 16: return launch_wc<16>(a, stream);
        case 32: return launch_wc<32>(a, stream);
        case 64: return launch_wc<64>(a, stream);
        case 128: return launch_wc<128>(a, stream);
        default: return launch_wc<256>(a, stream);
    }
}

}  // namespace wlcs
