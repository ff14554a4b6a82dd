// One unit of the windowed seaweed plot: 64 consecutive strips (x-windows)
// against two y-tiles, combed, counted and stored.  Shared by the single-plot
// kernel (seaweed.hip) and the persistent batched kernel (batch.hip); the
// method and the mapping are described at the top of seaweed.hip.
#pragma once

#include <type_traits>

#include "kernels.hpp"
#include "packed.hpp"

namespace wlcs {

// dwords per lane row of the staging buffer (one per 4 windows, plus a pad
// dword that spreads the lanes over the LDS banks)
constexpr int stage_pitch(int wc, int ws = 1) { return flush_windows(wc, ws) / 4 + 1; }

// Per byte: x - b (mod 256) for b <= 127 in every byte, without borrows
// between the bytes.
__device__ __forceinline__ uint32_t sub_bytes(uint32_t x, uint32_t b4) {
    const uint32_t H = 0x80808080u;
    return ((x | H) - b4) ^ ((x ^ ~b4) & H);
}
// One 32-bit word of a strip's bitmap: bit b is set iff byte b % 4 of
// d[b / 4] is at least the threshold T, for bytes below 128.  k4 holds
// 128 - T (T clamped to [0, 128]) in every byte: v + 128 - T keeps bit 7 iff
// v >= T, with no carry between the bytes.  v_dot4_u32_u8 weighs the four
// bit-7 flags of a dword by 1, 2, 4, 8 (16 .. 128 for the second dword of an
// eight-window chunk), which gives 128 times a byte of the word.
__device__ __forceinline__ uint32_t bitmap_word(const uint32_t* d, uint32_t k4) {
    auto chunk = [&](int i, uint32_t acc) -> uint32_t {  // 128 x windows 8i .. 8i + 7, plus acc
        const uint32_t a = (d[2 * i] + k4) & 0x80808080u, b = (d[2 * i + 1] + k4) & 0x80808080u;
        return __builtin_amdgcn_udot4(b, 0x80402010u, __builtin_amdgcn_udot4(a, 0x08040201u, acc, false), false);
    };
    const uint32_t lo = chunk(0, chunk(1, 0u) << 8);  // 128 x bits 0..15
    const uint32_t hi = chunk(2, chunk(3, 0u) << 8);  // 128 x bits 16..31
    return (lo >> 7) | (hi << 9);
}

// LDS ring words (16 start columns each) per lane: the ring must cover the
// w + 1 start columns that can be pending at once, with a margin that keeps
// the word being cleared apart from the newest marks.
constexpr int ring_words(int wc) { return wc <= 128 ? 16 : 32; }
constexpr int stage_dwords(int wc, int ws = 1) { return 2 * 64 * stage_pitch(wc, ws); }
// Stores of a strided plot for one flushed block: window j0 + b of strip
// s0 + r sits in byte b of row r of the staged block (stride pitch dwords).
// Output column c holds the window c * hy; the lanes of the wave cover the
// block's output columns of one strip at a time, so the stores of a strip are
// contiguous.
__device__ __forceinline__ void strided_stores(uint8_t* __restrict__ out, uint16_t* __restrict__ indel,
                                               const Geom& g, int64_t s0, int64_t j0, int nk, int w,
                                               const uint8_t* staged, int pitch) {
    if (nk <= 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t hy = g.hy;
    const int64_t c_lo = (j0 + hy - 1) / hy;
    const int nout = (int)((j0 + nk + hy - 1) / hy - c_lo);  // <= 64
    if (nout <= 0) return;
    const bool act = lane < nout;
    const int64_t c = c_lo + lane;
    const int b = act ? (int)(c * hy - j0) : 0;
    const int64_t rest = g.rows - s0;
    const int nrows = rest < 64 ? (int)rest : 64;
#pragma unroll 1
    for (int r = 0; r < nrows; ++r) {
        const int64_t s = s0 + r;
        const uint32_t v = staged[r * pitch * 4 + b];
        if (act) {
            if (out) out[s * g.ld + c] = (uint8_t)v;
            if (indel) indel[s * g.ld_indel + c] = (uint16_t)(2 * w - 2 * (int)v);
        }
    }
}

// Flags of the four staged windows of dword d (byte i = window 4q + i): bit
// 8i + 7 is set iff the window's value is at least the threshold.  SMALL
// (every value below 128, windows of at most 127 letters): per byte,
// (v | 0x80) - T keeps bit 7 iff v >= T, with no borrow between the bytes for
// T <= 128 (t4 = T in every byte).  Otherwise the bytes are split into the
// even and the odd pair of 16-bit lanes, where (v | 0x8000) - T keeps bit 15
// iff v >= T for any v <= 255 and T <= 256 (t2 = T in both halves).
template <bool SMALL>
__device__ __forceinline__ uint32_t dot_flags(uint32_t d, uint32_t t4, uint32_t t2) {
    if (SMALL) return ((d | 0x80808080u) - t4) & 0x80808080u;
    const uint32_t e = d & 0x00FF00FFu, o = (d >> 8) & 0x00FF00FFu;
    const uint32_t fe = ((e | 0x80008000u) - t2) & 0x80008000u;
    const uint32_t fo = ((o | 0x80008000u) - t2) & 0x80008000u;
    return (fe >> 8) | fo;
}

// The dots (windows with WLCS >= threshold, at output positions) of one
// flushed block, listed by the lane that owns each strip: lane r flags the
// staged windows of strip s0 + r (a dword per four windows, `row`) and counts
// them; a scan of the counts over the wave gives each lane its offset, one
// atomic add reserves a run of slots for the whole block (so that a dense list
// does not serialise on the counter), and each lane writes its records in
// window order, the strips one after another.  The block's output positions
// (bit b: window j0 + b is an output; every window for hy = 1, every hy-th
// for hy > 1) are the same for every lane.  The counter keeps counting past
// dot_cap; records beyond it are not written.
template <int FL, bool SMALL>
__device__ __forceinline__ void list_dots(DotRec* __restrict__ dots, unsigned long long* __restrict__ dot_count,
                                          const Geom& g, int64_t s0, int64_t j0, int nk, int w,
                                          const uint32_t* row) {
    static_assert(FL <= 64, "one 64-bit mask of output positions per block");
    if (nk <= 0 || g.threshold > w) return;  // uniform
    const int lane = threadIdx.x & 63;
    uint64_t obits;  // wave-uniform
    if (g.hy == 1) {
        obits = nk >= 64 ? ~0ull : (1ull << nk) - 1ull;
    } else {
        obits = 0;
        const int64_t c_lo = (j0 + g.hy - 1) / g.hy;
        for (int64_t b = c_lo * g.hy - j0; b < nk; b += g.hy) obits |= 1ull << b;
    }
    const uint32_t t = (uint32_t)(g.threshold > 0 ? g.threshold : 0);
    const uint32_t t4 = t * 0x01010101u, t2 = t * 0x00010001u;
    // byte-form output mask of dword q: bit 8i + 7 for each output window 4q + i
    auto omask = [&](int q) -> uint32_t {
        const uint32_t nib = (uint32_t)(obits >> (4 * q)) & 0xFu;
        return ((nib * 0x00204081u) & 0x01010101u) << 7;
    };
    uint32_t cnt = 0;
    if (s0 + lane < g.rows) {  // a lane past the last strip holds a copy
#pragma unroll
        for (int q = 0; q < FL / 4; ++q) cnt += (uint32_t)__popc(dot_flags<SMALL>(row[q], t4, t2) & omask(q));
    }
    uint32_t incl = cnt;  // inclusive scan of the counts over the lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, d);
        if (lane >= d) incl += y;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63);  // wave-uniform
    if (total == 0) return;
    unsigned long long base0 = 0;
    if (lane == 0) base0 = atomicAdd(dot_count, (unsigned long long)total);
    const unsigned long long base =
        (((unsigned long long)__builtin_amdgcn_readlane((uint32_t)(base0 >> 32), 0) << 32) |
         __builtin_amdgcn_readlane((uint32_t)base0, 0)) + (incl - cnt);
    const unsigned long long cap = (unsigned long long)g.dot_cap;
    if (!dots || cnt == 0 || base >= cap) return;
    unsigned long long k = base;
    const uint32_t ii = (uint32_t)(g.x0 + (s0 + lane) * g.xstride);
#pragma unroll 1
    for (int q = 0; q < FL / 4 && k < cap; ++q) {
        const uint32_t d = row[q];
        uint32_t m = dot_flags<SMALL>(d, t4, t2) & omask(q);
        while (m != 0 && k < cap) {
            const int bit = __builtin_ctz(m);  // 8i + 7
            m &= m - 1u;
            const uint32_t v = (d >> (bit - 7)) & 0xFFu;
            uint32_t* rec = (uint32_t*)(dots + k);
            rec[0] = ii;
            rec[1] = (uint32_t)(j0 + 4 * q + (bit >> 3));
            rec[2] = v | ((uint32_t)(2 * w - 2 * (int)v) << 16);
            ++k;
        }
    }
}

// SP: the strided / sparse variant (store every g.hy-th window and list the
// dots of the windows at or above the threshold; WS = 1 only).
// DL: the score-plot schedule for strings blown up with a separator before
// every letter (WS = 2; Section 2's reduction of the alignment score).  Rows
// alternate separator, letter, separator, ...; so do the columns (tile starts
// are even).  In a separator column every separator row matches and every
// letter row mismatches, so the pair of rows (2r, 2r + 1) sends the larger of
// its two labels down to row 2r + 2 (or out of the strip) and keeps the
// smaller one, and the new top seaweed enters row 0: one max and one min per
// pair, with no chain down the column.  In a letter column the separator row
// is a mismatch (min/max) and the letter row the general cell.  One top-down
// pass combs a separator column and the letter column after it together: at
// each pair slot the separator column's max is carried to the next slot
// instead of being written there (fused_slot).  Two passes run at once, one
// slot apart, so that two independent chains share the instruction stream.
// The strip has WC / 2 pair slots; a window of w / 2 < WC / 2 pairs leaves the
// top WC / 2 - w / 2 (< kDlSlots) slots unused.
//
// PART: 0 combs the whole strip in one wave.  With two waves per strip, PART
// 1 (the upper wave) combs the upper rows (DL: pair slots) and hands the
// labels leaving its last row to PART 2 (the lower wave) through `hand` in
// LDS, four per group of columns (DL: per pair of passes); PART 2 combs the
// lower rows one group behind, counts and stores.  Both waves meet at one
// workgroup barrier per group (the upper after writing, the lower before
// reading), and the same sequence of groups in both makes the barriers match.
// NPART > 2 (the 256-row class, see wide_rows): a chain of NPART waves, wave
// PART taking its rows of the strip from the one above through its own pair
// of hand-over buffers, PART - 1 groups behind the first; every wave ends each
// group with the workgroup barrier, after PART - 1 barriers before its first
// group and NPART - PART after its last, so the counts match.
template <int WC, bool EXACT, int WS = 1, bool SP = false, bool DL = false, int PART = 0, int NPART = 2>
__device__ __forceinline__ void comb_unit(const uint16_t* __restrict__ xf, const uint32_t* __restrict__ yg32,
                                          uint8_t* __restrict__ out, uint32_t* __restrict__ bm32,
                                          uint16_t* __restrict__ indel, DotRec* __restrict__ dots,
                                          unsigned long long* __restrict__ dot_count, const Geom& g, int64_t sb,
                                          int pr, uint32_t* __restrict__ ring, uint32_t* __restrict__ stage,
                                          uint32_t* __restrict__ hand = nullptr) {
    static_assert(!SP || WS == 1, "strided and sparse plots store single windows");
    static_assert(!DL || (WS == 2 && !EXACT && WC % (2 * kDlSlots) == 0), "the score-plot schedule");
    // the chain of waves of the 256-row class
    constexpr bool WIDE = !DL && PART != 0 && NPART > 2;
    static_assert(PART == 0 || (DL ? dl_split(WC) : (WS == 1 && (general_split(WC) || WIDE))),
                  "two waves per strip: score plots above kDlSplitRows rows, other plots of 128 rows");
    static_assert(!WIDE || (WC == 256 && !EXACT && PART <= NPART && NPART == kWideWaves), "the 256-row chain");
    static_assert(NPART == 2 || WIDE, "a chain of more than two waves is the 256-row class");
    constexpr bool UPPER = PART != 0 && PART < NPART;  // combs only: no count, no stores
    constexpr int RW = ring_words(WC);
    constexpr int FL = flush_windows(WC, WS);
    constexpr int PITCH = stage_pitch(WC, WS);
    constexpr int FO = FL / WS;  // outputs per flushed block
    const int lane = threadIdx.x & 63;
    const int64_t s0 = sb * 64;
    int64_t tA;  // first window of tile A
    const int64_t tlen = pair_tile(g.cols, g.tile, g.tile2, g.nbig, pr, &tA);  // windows per tile of this pair
    const int64_t tB = tA + tlen;
    const int w = EXACT ? WC : g.w;

    // Rows.  A window shorter than its class runs in a strip padded at the
    // top to wpad = w rounded up to 8 rows (pad_rows, wide_pad_rows): the pad
    // rows hold a code that no y letter has, so every cell there is a
    // mismatch whose left-boundary label (0) stays put while each seaweed
    // from the top (label >= 1) passes straight down -- the padded strip has
    // the same exits as the strip of height w.  Rows from wpad on are skipped
    // 8 at a time by one uniform branch, so no cell carries a test of its
    // own.
    const int pad = (EXACT || DL) ? 0 : (WIDE ? wide_pad_rows(w) : pad_rows(w)) - w;
    const int wpad = (EXACT || DL) ? WC : w + pad;
    constexpr int NP = WC / 2;                 // DL: pair slots
    const int ppad = DL ? NP - w / 2 : 0;      // DL: unused slots at the top (< kDlSlots)
    // DL: this wave's pair slots, S0 .. S0 + NS - 1 of the strip
    constexpr int S0 = (DL && PART == 2) ? dl_upper_slots(WC) : 0;
    constexpr int NS = (!DL || PART == 0) ? NP : PART == 1 ? dl_upper_slots(WC) : NP - dl_upper_slots(WC);
    static_assert(!DL || (NS % 2 == 0 && S0 >= (PART == 2 ? kDlSlots : 0)), "slot split");
    // general: this wave's rows, R0 .. R0 + NR - 1 of the strip (WIDE: NR
    // is the capacity, the wave's rows are r0 .. r0 + nrw - 1)
    constexpr int R0 = (!DL && !WIDE && PART == 2) ? WC / 2 : 0;
    constexpr int NR = WIDE ? kWideRowsPerWave : (DL || PART == 0) ? WC : WC / 2;
    constexpr int HN = DL ? 2 * NS : NR;       // labels held by this wave
    int r0 = R0, nrw = NR;
    if constexpr (WIDE) wide_rows(w, PART - 1, &r0, &nrw);
    constexpr bool TOP = PART <= 1;            // this wave holds row 0 of the strip
    // x letters of this lane's strip, two rows per register (lanes past the
    // last strip comb a copy of the last one; their results are never stored);
    // DL: the letters of this wave's letter rows only, two slots per register
    constexpr int NXC = DL ? NS / 2 : NR / 2;
    uint32_t xc[NXC];
    {
        const int64_t sx = s0 + lane < g.rows ? s0 + lane : g.rows - 1;
        const uint16_t* xp = xf + sx * g.xstride;
        constexpr uint32_t PADF = f_code(kPadCode);
#pragma unroll
        for (int j = 0; j < NXC; ++j) {
            uint32_t lo, hi;
            if (DL) {  // slot r holds letter r - ppad, at row 2 (r - ppad) + 1 of the strip
                const int i0 = S0 + 2 * j - ppad, i1 = S0 + 2 * j + 1 - ppad;
                lo = i0 >= 0 ? (uint32_t)xp[2 * i0 + 1] : PADF;
                hi = i1 >= 0 ? (uint32_t)xp[2 * i1 + 1] : PADF;
            } else {
                const int i0 = r0 + 2 * j - pad, i1 = r0 + 2 * j + 1 - pad;
                lo = (EXACT || i0 >= 0) ? (uint32_t)xp[EXACT ? R0 + 2 * j : i0] : PADF;
                hi = (EXACT || i1 >= 0) ? (uint32_t)xp[EXACT ? R0 + 2 * j + 1 : i1] : PADF;
            }
            xc[j] = lo | (hi << 16);
        }
    }
    uint32_t h[HN];
#pragma unroll
    for (int k = 0; k < HN; ++k) h[k] = 0;
    if constexpr (!UPPER && (DL || WC > 32)) {  // the LDS ring of pending marks (longer windows)
#pragma unroll
        for (int q = 0; q < RW; ++q) ring[q * 64 + lane] = 0;
    }

    const int64_t restA = g.cols - tA;  // > 0: every launched unit has a non-empty tile A
    const int64_t nA = (restA + 63) / 64 * 64;
    const int nproc = (int)(nA < tlen ? nA : tlen);

    int32_t org = -w;   // the seaweed starting at tile column l carries label l - org + 1
    uint32_t rem2 = pk_rep(w);  // w minus the seaweeds counted for the current window, both tiles
    uint32_t ring_pf = 0;
    const uint32_t w2 = pk_rep(w);
    constexpr int RB = RW == 16 ? 4 : 5;  // log2 of the ring words per lane
    uint32_t* const ring_lane = ring + lane;

    // y codes of the two tiles (tile starts are multiples of 64, so both
    // bases are dword aligned); the codes are read-only and the index is
    // wave-uniform, so the loads and the unpacking stay on the scalar unit
    const const_u32p yA = as_const(yg32 + (tA >> 1));
    const const_u32p yB = as_const(yg32 + (tB >> 1));
    auto yload = [&](int l) -> uint32_t {
        const int q = __builtin_amdgcn_readfirstlane(l >> 1);
        const uint32_t sh = (uint32_t)__builtin_amdgcn_readfirstlane(l & 1) * 16u;
        const uint32_t a = yA[q], b = yB[q];
        return __builtin_amdgcn_readfirstlane(((a >> sh) & 0xFFFFu) | (((b >> sh) & 0xFFFFu) << 16));
    };
    const uint32_t one2 = 0x00010001u;
    uint32_t ynext = DL ? 0u : yload(0);

    // Windows of at most 32 letters keep the pending marks in registers
    // instead of the LDS ring: bit q of a tile's mask marks the start column
    // (l - w + 1) + q of the current window l - w + 1.  Moving to the next
    // column takes bit 0 out (that start column leaves the window: the mark
    // consumed) and shifts the rest down by one.  Up to 16 letters the masks
    // of both tiles share one register, a 16-bit half each; up to 32 each
    // tile has a register of its own.
    constexpr bool RMASK = !DL && WC <= 32;
    uint32_t m2 = 0, mA = 0, mB = 0;

    // The sliding count after column l (tile-relative), from the packed label
    // t leaving its bottom; returns w - count for the window starting at
    // l - w + 1.
    auto count = [&](int l, uint32_t t) -> uint32_t {
        // consume the mark of start column l - w (ring: prefetched after the
        // previous column's marks were set)
        uint32_t f2 = 0;
        const int pc = l - w;
        if constexpr (RMASK && WC <= 16) {
            f2 = m2 & one2;
        } else if constexpr (RMASK) {
            f2 = __builtin_amdgcn_perm(mB, mA, 0x0c040c00u) & one2;  // bit 0 of each mask
        } else if (pc >= 0) {
            f2 = (ring_pf >> (pc & 15)) & 0x00010001u;
            if ((pc & 15) == 15) ring_lane[((pc >> 4) & (RW - 1)) * 64] = 0;
        }
        uint32_t p2 = 0, v2;
        if constexpr (RMASK) {
            // p = start - (l - w + 1) lies in [0, w) iff the exit's span is below w
            p2 = pk_sub(t, pk_rep(l - org + 2 - w));
            v2 = pk_below(w2, p2, one2);
        } else {
            // the same test on the label: the exit's seaweed started in the
            // window iff t >= label(l - w + 1) = l - w + 2 - org (>= 2 here)
            v2 = pk_above(t, pk_rep(l - w + 1 - org), one2);
        }
        if constexpr (RMASK && WC <= 16) {
            m2 = pk_shr1(m2) | pk_lshl(p2, v2);  // p < w <= 16 wherever v = 1
        } else if constexpr (RMASK) {
            mA = (mA >> 1) | ((v2 & 0xFFFFu) << (p2 & 31u));  // p < w <= 32 wherever v = 1
            mB = (mB >> 1) | ((v2 >> 16) << ((p2 >> 16) & 31u));
        } else {
            const uint32_t pos2 = pk_add(t, pk_rep(org - 1));  // the start column: label + org - 1
            const uint32_t bit2 = pk_lshl(pos2, v2);
            // ring word of each mark: bits 4.. of its start column
            const uint32_t wlo = bfe<4, RB>(pos2), whi = bfe<20, RB>(pos2);
            atomicOr(&ring_lane[wlo * 64], bit2 & 0xFFFFu);
            atomicOr(&ring_lane[whi * 64], bit2 & 0xFFFF0000u);
        }
        rem2 = pk_add(pk_sub(rem2, v2), f2);
        if constexpr (!RMASK) {
            if (pc + 1 >= 0) ring_pf = ring_lane[(((pc + 1) >> 4) & (RW - 1)) * 64];
        }
        return rem2;
    };

    // Comb column l (tile-relative) through this wave's rows (general
    // schedule); returns the label leaving the last of them.  The upper rows
    // start from the column's top label, the lower ones from t_in (the label
    // the upper wave handed over).
    auto comb_rows = [&](int l, uint32_t t_in) -> uint32_t {
        const uint32_t Y = ynext;
        ynext = yload(l + 1);
        uint32_t t = t_in;
        if constexpr (TOP) t = seaweed_cell_top(h[0], pk_rep(l - org + 1), xc[0], Y);
#pragma unroll
        for (int k = TOP ? 1 : 0; k < NR; ++k) {
            // uniform, once per block of rows past the fewest a wave holds
            if constexpr (WIDE) {
                if (wide_stops_at_row(k, nrw)) break;
            } else {
                if (!EXACT && stops_at_row(WC, R0 + k, wpad)) break;
            }
            t = (k & 1) ? seaweed_cell<1>(h[k], t, xc[k >> 1], Y) : seaweed_cell<0>(h[k], t, xc[k >> 1], Y);
        }
        return t;
    };
    // One column through the whole strip; returns the count.
    auto column = [&](int l) -> uint32_t { return count(l, comb_rows(l, 0u)); };
    // Two waves per strip: columns l0 .. l0 + n - 1 (n <= 4, uniform).  The
    // upper wave hands the four exits over and returns nothing; the lower
    // wave returns the counts (of the columns there are) in r[].  (One wave
    // per strip combs column by column: grouping its columns would inline four
    // copies of a whole strip per call site, which at 256 rows no longer
    // unrolls and puts the label arrays in scratch memory.)
    int hand_buf_g = 0;
    auto group = [&](int l0, int n, uint32_t (&r)[4]) {
        if constexpr (WIDE) {
            // this wave's pair of buffers from the wave above, and to the one
            // below (kDlHandDwords per link: two buffers of four columns of
            // 64 lanes)
            const int hb = (hand_buf_g & 1) * (kDlHandDwords / 2) + lane;
            const uint32_t* const hin = hand + (TOP ? 0 : (PART - 2) * kDlHandDwords) + hb;
            uint32_t* const hout = hand + (UPPER ? (PART - 1) * kDlHandDwords : 0) + hb;
            ++hand_buf_g;
            uint32_t t_in[4] = {0u, 0u, 0u, 0u};
            if constexpr (!TOP) {
#pragma unroll
                for (int i = 0; i < 4; ++i) t_in[i] = hin[i * 64];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (i < n) {
                    const uint32_t t = comb_rows(l0 + i, t_in[i]);
                    if constexpr (UPPER)
                        hout[i * 64] = t;
                    else
                        r[i] = count(l0 + i, t);
                }
            }
            __syncthreads();
        } else if constexpr (PART != 0) {
            uint32_t* const hb = hand + (hand_buf_g & 1) * 256 + lane;
            ++hand_buf_g;
            if constexpr (UPPER) {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (i < n) hb[i * 64] = comb_rows(l0 + i, 0u);
                __syncthreads();
            } else {
                __syncthreads();
                uint32_t t_in[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) t_in[i] = hb[i * 64];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (i < n) r[i] = count(l0 + i, comb_rows(l0 + i, t_in[i]));
            }
        }
    };

    // DL: a pass down the pair slots combs the separator column c - 1 and
    // the letter column c (c odd) together; two passes (c and c + 2) run at
    // once, the second one slot behind the first, which leaves every slot of
    // the first pass done before the second reads it.  The y codes of the
    // letter columns are loaded one call ahead.  Returns the counts after
    // columns c, c + 1 and c + 2 (the last two of a pair of passes only).
    uint32_t yq0 = 0, yq1 = 0;
    if constexpr (DL) {
        yq0 = yload(1);
        yq1 = yload(3);
    }
    int hand_buf = 0;  // DL split: pairs of passes so far (picks the hand-over buffer)
    struct Counts { uint32_t c0, c1, c2; };
    auto passes = [&](int c, auto two_t) -> Counts {
        constexpr bool TWO = decltype(two_t)::value;
        const uint32_t YP = yq0, YQ = yq1;
        if (TWO) {
            yq0 = yload(c + 4);
            yq1 = yload(c + 6);
        } else {
            yq0 = yq1;
            yq1 = yload(c + 4);
        }
        uint32_t pcar = pk_rep(c - org), pt = pk_rep(c + 1 - org);
        uint32_t qcar = pk_rep(c + 2 - org), qt = pk_rep(c + 3 - org);
        uint32_t* const hb = hand + (hand_buf & 1) * 256 + lane;  // DL split: this pair of passes' hand-over
        if constexpr (PART == 2) {
            // the labels leaving the upper wave's last slot in these passes
            __syncthreads();
            pcar = hb[0];
            pt = hb[64];
            qcar = hb[128];
            qt = hb[192];
        }
        // The unused top slots (their letter is the pad code, which matches
        // nothing) run the same steps: the letter column's label, the largest
        // of all, passes through them unchanged, and after each of them the
        // separator column's carry is raised to its own top label (larger
        // than every label the slot holds), so that both columns enter the
        // first used slot with their top labels.
        const uint32_t sP = pcar, sQ = qcar;
        // step k: pass P at slot k, pass Q at slot k - 1 (this wave's slots)
        auto step = [&](int k, bool q_on) {
            const int kp = k < NS ? k : NS - 1, kq = k >= 1 ? k - 1 : 0;
            if (k < NS && q_on) {
                if (k & 1)
                    fused_slot2<1>(h[2 * kp], h[2 * kp + 1], pt, pcar, xc[kp >> 1], YP, h[2 * kq], h[2 * kq + 1],
                                   qt, qcar, xc[kq >> 1], YQ);
                else
                    fused_slot2<0>(h[2 * kp], h[2 * kp + 1], pt, pcar, xc[kp >> 1], YP, h[2 * kq], h[2 * kq + 1],
                                   qt, qcar, xc[kq >> 1], YQ);
            } else if (k < NS) {
                pcar = (k & 1) ? fused_slot<1>(h[2 * kp], h[2 * kp + 1], pt, pcar, xc[kp >> 1], YP)
                               : fused_slot<0>(h[2 * kp], h[2 * kp + 1], pt, pcar, xc[kp >> 1], YP);
            } else if (q_on) {
                qcar = (kq & 1) ? fused_slot<1>(h[2 * kq], h[2 * kq + 1], qt, qcar, xc[kq >> 1], YQ)
                                : fused_slot<0>(h[2 * kq], h[2 * kq + 1], qt, qcar, xc[kq >> 1], YQ);
            }
            if (S0 + k < kDlSlots && k < NS) pcar = pk_max(pcar, k < ppad ? sP : 0u);
            if (q_on && S0 + kq < kDlSlots) qcar = pk_max(qcar, kq < ppad ? sQ : 0u);
        };
#pragma unroll
        for (int k = 0; k <= NS; ++k) step(k, TWO && k >= 1);
        ++hand_buf;
        if constexpr (UPPER) {
            hb[0] = pcar;
            hb[64] = pt;
            hb[128] = qcar;
            hb[192] = qt;
            __syncthreads();
            return Counts{0u, 0u, 0u};
        }
        (void)count(c - 1, pcar);
        Counts r;
        r.c0 = count(c, pt);
        if (TWO) {
            r.c1 = count(c + 1, qcar);
            r.c2 = count(c + 2, qt);
        } else {
            r.c1 = r.c2 = r.c0;
        }
        return r;
    };

    using P0 = std::integral_constant<bool, false>;
    using P1 = std::integral_constant<bool, true>;
    // warm-up columns: no window is complete yet (DL: w is even, so the
    // w - 1 warm-up columns 0 .. w - 2 end on a separator column, which the
    // first pass of the main loop combs)
    if constexpr (DL) {
        int c = 1;
        for (; c + 2 <= w - 3; c += 4) (void)passes(c, P1{});
        if (c <= w - 3) (void)passes(c, P0{});
    } else if constexpr (PART == 0) {
        for (int l = 0; l < w - 1; ++l) (void)column(l);
    } else {
        if constexpr (WIDE) {
            for (int q = 1; q < PART; ++q) __syncthreads();  // the chain fills: one group per wave above
        }
        uint32_t r[4];
        for (int l = 0; l < w - 1; l += 4) group(l, w - 1 - l < 4 ? w - 1 - l : 4, r);
    }

    // The staging block is this wave's alone: with two waves per strip the
    // lower wave orders its LDS accesses without a workgroup barrier (the
    // upper wave does not store).
    auto stage_sync = [&]() {
        if constexpr (PART == 0) {
            __syncthreads();
        } else {
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    };
    const uint32_t bm_words = (uint32_t)(((g.ocols + 63) >> 6) * 2);
    for (int jb = 0; jb < nproc; jb += FL) {
#pragma unroll 1
        for (int gi = 0; gi < FL / 4; ++gi) {
            const int jj = jb + 4 * gi;
            if (jj > 0 && (jj % kRebase) == 0) {
                const int32_t norg = jj - 1;  // (column jj + w - 1) - w
                const uint32_t d2 = pk_rep(norg - org);
#pragma unroll
                for (int k = 0; k < HN; ++k) h[k] = pk_sub_sat(h[k], d2);
                org = norg;
            }
            const int l = jj + w - 1;  // DL: odd (w even, jj a multiple of 4)
            uint32_t r0, r1, r2, r3;
            if constexpr (DL) {
                // columns l - 1 .. l + 2; the window after column l + 3
                // (odd, never stored) takes r2's place
                const Counts r = passes(l, P1{});
                r0 = r.c0;
                r1 = r.c1;
                r2 = r3 = r.c2;
            } else if constexpr (PART == 0) {
                r0 = column(l);
                r1 = column(l + 1);
                r2 = column(l + 2);
                r3 = column(l + 3);
            } else {
                uint32_t r[4] = {0u, 0u, 0u, 0u};
                group(l, 4, r);
                r0 = r[0];
                r1 = r[1];
                r2 = r[2];
                r3 = r[3];
            }
            if constexpr (!UPPER) {
                // bytes 0 (tile A) and 2 (tile B) of the four results, gathered
                // into one dword per tile: r0.b0 r0.b2 r1.b0 r1.b2, then the
                // same for r2, r3, then the even and the odd bytes of the two
                const uint32_t t01 = __builtin_amdgcn_perm(r1, r0, 0x06040200u);
                const uint32_t t23 = __builtin_amdgcn_perm(r3, r2, 0x06040200u);
                const uint32_t wa = __builtin_amdgcn_perm(t23, t01, 0x06040200u);
                const uint32_t wb = __builtin_amdgcn_perm(t23, t01, 0x07050301u);
                stage[lane * PITCH + gi] = wa;
                stage[64 * PITCH + lane * PITCH + gi] = wb;
            }
        }
        if constexpr (UPPER) continue;  // the lower wave stores
        stage_sync();
        // this lane's strip (for windows of at most 32 letters, at four
        // waves per SIMD, an opaque copy per flush: the row addresses
        // derived from it are then formed here instead of being held in
        // registers through the combing, which spilled them)
        int64_t s = s0 + lane;
        if constexpr (WC <= 32) asm volatile("" : "+v"(s));
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            const int64_t ts = half ? tB : tA;
            const int64_t te = ts + tlen < g.cols ? ts + tlen : g.cols;
            const int64_t j0 = ts + jb;   // first (combed) window of the block
            const int64_t o0 = j0 / WS;   // its output column
            // windows of this block inside the tile (0 for the padding block
            // that completes the last bitmap word, or past the end of y);
            // with WS = 2 only the even ones are outputs
            const int nk = (int)(te - j0 < FL ? (te - j0 > 0 ? te - j0 : 0) : FL);
            if (SP) {
                const uint32_t* sblock = stage + half * 64 * PITCH;
                if (g.hy > 1 && (out || indel))
                    strided_stores(out, indel, g, s0, j0, nk, w, (const uint8_t*)sblock, PITCH);
                if (dot_count) list_dots<FL, (WC <= 64)>(dots, dot_count, g, s0, j0, nk, w, sblock + lane * PITCH);
                if (g.hy > 1) continue;  // uniform
            }
            const int nvalid = (nk + WS - 1) / WS;
            if (nvalid == 0 && (uint32_t)(o0 >> 5) >= bm_words) continue;  // uniform
            uint32_t d[FO / 4];
#pragma unroll
            for (int k = 0; k < FO / 4; ++k) {
                if (WS == 1) {
                    d[k] = stage[half * 64 * PITCH + lane * PITCH + k];
                } else {  // keep bytes 0 and 2 of two staged dwords
                    const uint32_t a = stage[half * 64 * PITCH + lane * PITCH + 2 * k];
                    const uint32_t b = stage[half * 64 * PITCH + lane * PITCH + 2 * k + 1];
                    d[k] = (a & 0xFFu) | ((a >> 8) & 0xFF00u) | ((b & 0xFFu) << 16) | ((b << 8) & 0xFF000000u);
                }
            }
            if (bm32 && s < g.rows) {
                const int kt = 128 - g.threshold;
                const uint32_t k4 = (uint32_t)(kt < 0 ? 0 : kt > 128 ? 128 : kt) * 0x01010101u;
#pragma unroll
                for (int sub = 0; sub < FO / 32; ++sub) {
                    const uint32_t wi = (uint32_t)(o0 >> 5) + sub;
                    if (wi < bm_words) {
                        const int nv = nvalid - 32 * sub;
                        uint32_t bits = 0;
                        if constexpr (WC <= 64) {  // values at most 64
                            bits = bitmap_word(d + 8 * sub, k4);
                        } else {
#pragma unroll
                            for (int b = 0; b < 32; ++b)
                                bits |= (uint32_t)((int)((d[8 * sub + (b >> 2)] >> (8 * (b & 3))) & 0xFFu) >=
                                                   g.threshold)
                                        << b;
                        }
                        if (nv < 32) bits &= nv > 0 ? (0xFFFFFFFFu >> (32 - nv)) : 0u;
                        bm32[s * g.ld_words32 + wi] = bits;
                    }
                }
            }
            if (g.bias) {
#pragma unroll
                for (int k = 0; k < FO / 4; ++k) d[k] = sub_bytes(d[k], (uint32_t)g.bias * 0x01010101u);
            }
            const int pmode = g.wmode & 3;
            if (out && pmode > 0 && nvalid > 0) {
                if (s < g.rows) {
                    uint8_t* row = out + s * g.ld + o0;
                    if (nvalid == FO) {
                        if (pmode == 2) {
#pragma unroll
                            for (int k = 0; k < FO / 16; ++k)
                                ((uint4*)row)[k] = make_uint4(d[4 * k], d[4 * k + 1], d[4 * k + 2], d[4 * k + 3]);
                        } else {
#pragma unroll
                            for (int k = 0; k < FO / 4; ++k) ((uint32_t*)row)[k] = d[k];
                        }
                    } else {  // a partial block: from the staged row (d cannot be indexed at run time)
                        const uint8_t* ob = (const uint8_t*)(stage + half * 64 * PITCH + lane * PITCH);
                        for (int b = 0; b < nvalid; ++b) row[b] = (uint8_t)(ob[b * WS] - (uint32_t)g.bias);
                    }
                }
            }
            if (WS == 1 && indel && (g.wmode & kIndelRows16) && nvalid > 0 && s < g.rows) {
                // this strip's indel distances 2w - 2v, read again from its
                // staged row: four per 8-byte store (two u16 lanes per dword,
                // the bytes spread by v_perm)
                const uint32_t* own = stage + half * 64 * PITCH + lane * PITCH;
                uint16_t* irow = indel + s * g.ld_indel + o0;
                if (nvalid == FO) {
                    const uint32_t w2x2 = (uint32_t)(2 * w) * 0x00010001u;
#pragma unroll 2
                    for (int k = 0; k < FO / 4; ++k) {
                        const uint32_t v = own[k];
                        const uint32_t lo = __builtin_amdgcn_perm(0u, v, 0x0c010c00u);  // bytes 0, 1
                        const uint32_t hi = __builtin_amdgcn_perm(0u, v, 0x0c030c02u);  // bytes 2, 3
                        ((uint2*)irow)[k] = make_uint2(pk_sub(w2x2, pk_add(lo, lo)), pk_sub(w2x2, pk_add(hi, hi)));
                    }
                } else {
                    const uint8_t* ob = (const uint8_t*)own;
                    for (int b = 0; b < nvalid; ++b) irow[b] = (uint16_t)(2 * w - 2 * (int)ob[b]);
                }
            }
            const bool indel_t = indel && (WS != 1 || !(g.wmode & kIndelRows16));
            if (((out && pmode == 0) || indel_t) && nvalid > 0) {
                // transposed: the lanes cover FO outputs of 64 / FO strips per step
                constexpr int RPI = 64 / FO;
                const int q = lane % FO;
                const uint8_t* sbytes = (const uint8_t*)stage;
#pragma unroll 4
                for (int it = 0; it < 64 / RPI; ++it) {
                    const int r = RPI * it + lane / FO;
                    const int64_t sr = s0 + r;
                    const uint32_t v = sbytes[(half * 64 * PITCH + r * PITCH) * 4 + q * WS];
                    if (sr < g.rows && q < nvalid) {
                        if (out && pmode == 0) out[sr * g.ld + o0 + q] = (uint8_t)(v - (uint32_t)g.bias);
                        if (indel_t) indel[sr * g.ld_indel + o0 + q] = (uint16_t)(2 * w - 2 * (int)v);
                    }
                }
            }
        }
        stage_sync();
    }
    if constexpr (WIDE) {
        for (int q = PART; q < NPART; ++q) __syncthreads();  // the chain drains: one group per wave below
    }
}

}  // namespace wlcs
