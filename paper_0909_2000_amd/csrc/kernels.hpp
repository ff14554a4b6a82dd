// Internal interface between the host runtime and the gfx950 kernels.
//
// Letter codes.  Every letter of the alphabet gets a code c in [0, 63).  The
// kernels never compare letters directly: x letters are stored as
// f(c) = c << 10 and y letters as g(c) = ((64 - c) mod 64) << 10, so that the
// 16-bit sum f(a) + g(b) is 0 when a == b and at least 1024 otherwise.  With
// seaweed labels kept below 1024, one packed add gives a value Z that sits
// below every label on a match and above every label on a mismatch, which
// turns the seaweed cell into max/min operations (seaweed.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlcs {

constexpr int kCodeShift = 10;
constexpr uint16_t f_code(uint32_t c) { return (uint16_t)(c << kCodeShift); }
constexpr uint16_t g_code(uint32_t c) { return (uint16_t)(((64u - c) & 63u) << kCodeShift); }
// A code no letter gets: an x row of it mismatches every y letter (padding
// rows of the strip, seaweed_unit.hpp).
constexpr uint32_t kPadCode = 63;

// Windows between two relabellings of the seaweed labels (a multiple of 32).
constexpr int kRebase = 512;

// Geom::wmode bit: the indel rows start 16 bytes apart (each lane stores its
// strip's indel values with 16-byte stores).
constexpr int32_t kIndelRows16 = 4;

// One plot's worth of kernel arguments (host side).
// One dot of a sparse plot: window starts, WLCS and indel distance (the
// wlcs_dot record of the C ABI).
struct DotRec {
    uint32_t i, j;
    uint16_t wlcs, indel;
};
static_assert(sizeof(DotRec) == 12, "dot record layout");

struct PlotArgs {
    int64_t xstride = 1;     // x codes between consecutive strips
    int64_t x0 = 0;          // x-window of the first strip (dot records count from it)
    const uint32_t* gate = nullptr;  // strided / sparse plots: if set, run only when *gate != 0
    int32_t ws = 1;          // store every ws-th combed window (1 or 2)
    int32_t bias = 0;        // subtracted from every stored value
    int64_t hy = 1;          // strided plots: output column c is the window c * hy
    int32_t sigma = 64;      // letters of the alphabet (the BLCS baseline keeps a mask per letter)
    DotRec* dots = nullptr;  // sparse output (may be null while counting)
    int64_t dot_cap = 0;
    unsigned long long* dot_count = nullptr;  // non-null: list the dots
    const uint16_t* xf;      // f-codes of x, padded (see host runtime)
    const uint16_t* yg;      // g-codes of y, padded
    int64_t rows;            // x-windows (strips)
    int64_t cols;            // y-windows
    int32_t w;
    int32_t tile;            // y-windows per tile, multiple of 64 (the long tiles)
    int32_t npairs;          // tile pairs per block of 64 strips
    int32_t tile2 = 0;       // y-windows per tile after the first nbig pairs (0: tile)
    int32_t nbig = 0;        // leading tile pairs of `tile` windows
    int32_t threshold;
    uint8_t* wlcs;           // may be null
    int64_t ld;
    uint32_t* bitmap32;      // uint64 words addressed as little-endian u32 halves; may be null
    int64_t ld_words32;      // row stride in u32 units (2 * ld_words)
    uint16_t* indel;         // may be null
    int64_t ld_indel;
};

// The pointer-free part, passed by value to the kernels (the pointers travel
// as separate __restrict__ parameters so that uniform loads become scalar).
struct Geom {
    int64_t rows, cols, ld, ld_words32, ld_indel;
    int64_t ocols;     // output columns (cols / ws: only every ws-th combed window is stored)
    int64_t xstride;   // x codes between consecutive strips (1: every x-window)
    int32_t w, tile, npairs, threshold;
    int32_t tile2, nbig;  // pairs from nbig on have tiles of tile2 windows
    int32_t wmode;     // bits 0-1, plot stores: 2 = 16-byte rows, 1 = 4-byte rows, 0 = bytes;
                       // bit 2 (kIndelRows16): indel rows start 16 bytes apart (16-byte stores)
    int32_t bias;      // subtracted from every stored value (0..127)
    int64_t hy;        // strided plots: output column c is the window c * hy
    int64_t dot_cap;   // dot records the sparse output holds
    int64_t x0;        // x-window of strip 0 (the dot records' i is x0 + strip * xstride)
};

// Tile pairs along a row of cols windows: the first nbig pairs have tiles of
// `tile` windows, the later ones tiles of tile2 (one length if tile2 ==
// tile); the last pair's remaining windows are split evenly (in whole blocks
// of 64) between its two tiles, so that both halves of every register carry
// work there too.  Returns the windows per tile of pair pr; tile A of the pair
// starts at *start, tile B right after it.
__host__ __device__ inline int64_t pair_tile(int64_t cols, int64_t tile, int64_t tile2, int64_t nbig, int64_t pr,
                                             int64_t* start) {
    const bool big = pr < nbig;
    const int64_t t = big ? tile : tile2;
    const int64_t a = big ? 2 * pr * tile : 2 * nbig * tile + 2 * (pr - nbig) * tile2;
    *start = a;
    const int64_t rest = cols - a;
    const int64_t half = ((rest + 1) / 2 + 63) / 64 * 64;
    return half < t ? half : t;
}

inline Geom geom_of(const PlotArgs& a) {
    Geom g;
    g.rows = a.rows;
    g.cols = a.cols;
    g.ld = a.ld;
    g.ld_words32 = a.ld_words32;
    g.ld_indel = a.ld_indel;
    g.w = a.w;
    g.tile = a.tile;
    g.npairs = a.npairs;
    g.tile2 = a.tile2 > 0 ? a.tile2 : a.tile;
    g.nbig = a.tile2 > 0 ? a.nbig : 0;
    g.threshold = a.threshold;
    g.ocols = a.ws == 2 ? a.cols / 2 : a.cols;
    g.xstride = a.xstride;
    g.bias = a.bias;
    g.hy = a.hy;
    g.dot_cap = a.dot_cap;
    g.x0 = a.x0;
    const uintptr_t base = (uintptr_t)a.wlcs;
    g.wmode = (a.ld % 16 == 0 && base % 16 == 0) ? 2 : (a.ld % 4 == 0 && base % 4 == 0) ? 1 : 0;
    if (a.ld_indel % 8 == 0 && (uintptr_t)a.indel % 16 == 0) g.wmode |= kIndelRows16;
    return g;
}

// One entry of the batched kernel's job table.
struct JobDesc {
    const uint16_t* xf;
    const uint32_t* yg32;
    uint8_t* out;
    uint32_t* bm32;
    uint16_t* indel;
    DotRec* dots;
    unsigned long long* dot_count;
    Geom g;
    int64_t unit0;    // index of the entry's first unit in its group's unit list
    int32_t variant;  // per-unit code path (batch_variant)
    int32_t pr0;      // the entry's first tile pair (a job's last pair is an entry of its own)
};

// Windows staged per lane before a flush: 64 (64-byte row segments) where
// the LDS budget allows it at the class's occupancy, else 32; 64 whenever only
// every second window is stored (ws = 2), so a block still fills 32 outputs.
constexpr int flush_windows(int wc, int ws = 1) { return (wc >= 64 || ws == 2) ? 64 : 32; }
// Occupancy each window class is compiled for (waves per SIMD): the w labels
// and w/2 code registers per lane plus the flush temporaries must fit.
constexpr int min_waves_per_simd(int wc) { return wc <= 32 ? 4 : wc <= 64 ? 3 : wc <= 128 ? 2 : 1; }
// Score-plot classes (the separator schedule of the seaweed kernel).  Waves
// per SIMD a class of wc rows is compiled for when one wave holds the whole
// strip: its wc labels and the codes of its wc / 2 letter rows (wc / 4
// registers) must fit.
constexpr int min_waves_per_simd_dl(int wc) { return wc <= 64 ? 3 : wc <= 128 ? 2 : 1; }
// Score-plot classes come in steps of this many pair slots (2 rows each), so a
// window leaves fewer than kDlSlots slots of its class unused.
constexpr int kDlSlots = 4;
// Score-plot classes above this many rows split every strip over two waves of
// one workgroup (the upper and the lower pair slots), so that each wave's
// labels and codes fit three (two above 208 rows) waves per SIMD instead of
// one.
constexpr int kDlSplitRows = 128;
constexpr bool dl_split(int wc) { return wc > kDlSplitRows; }
// Pair slots of the upper wave: a little over half, since the lower wave also
// counts and stores (a multiple of kDlSlots, so unused slots stay in it).
constexpr int dl_upper_slots(int wc) { return (wc / 4 + 2 + kDlSlots - 1) / kDlSlots * kDlSlots; }
constexpr int min_waves_per_simd_dl_split(int wc) { return wc <= 208 ? 3 : 2; }
// LDS of the hand-over between the two waves: two buffers of four labels
// per lane
constexpr int kDlHandDwords = 2 * 4 * 64;
// Plots in the 128-row class split every strip over two waves as well (the
// upper and the lower half of the rows): one wave holding 128 rows needs all
// 256 registers (two waves per SIMD), a half fits three.  (Halves of the
// 256-row class spill inside the column loop at two waves per SIMD and ran
// slower than one wave holding the whole strip.)
constexpr bool general_split(int wc) { return wc == 128; }
constexpr int min_waves_per_simd_split(int wc) { return wc <= 128 ? 3 : 2; }
// Plots in the 256-row class (windows of 129..255 letters) chain four waves
// down every strip, each holding at most 64 rows (one wave holding the strip
// needs its labels in accumulation registers, at one wave per SIMD; chains of
// three waves measured slower and less steady from run to run).  The strip
// is padded at the top to wpad = w rounded up to 8 rows, and its rows are
// dealt out to the waves in blocks of 8, the earlier waves taking the extra
// blocks (the last wave also counts and stores): every wave gets 32 to 64
// rows.
constexpr int kWideWaves = 4;
constexpr int kWideRowsPerWave = 64;
constexpr int kWideRowBlock = 8;
constexpr int kWideMinRows = 32;
__host__ __device__ constexpr int wide_pad_rows(int w) { return (w + kWideRowBlock - 1) / kWideRowBlock * kWideRowBlock; }
// Rows of the strip a window shorter than its class is combed in (padded at
// the top with rows that match nothing): w rounded up to a block of
// kPadRowBlock rows, the rows past it skipped one block at a time.
constexpr int kPadRowBlock = 8;
__host__ __device__ constexpr int pad_rows(int w) { return (w + kPadRowBlock - 1) / kPadRowBlock * kPadRowBlock; }
// The fewest rows a window of class wc is combed in (class 16 holds windows
// of 1..16 letters, every larger class those longer than half of it): no row
// below it is ever skipped.
__host__ __device__ constexpr int min_pad_rows(int wc) { return pad_rows(wc <= 16 ? 1 : wc / 2 + 1); }
// Whether a window shorter than class wc, combed in wpad rows, stops before
// row r of the strip: tested once per block of rows from the fewest rows a
// window of the class is combed in.
__host__ __device__ constexpr bool stops_at_row(int wc, int r, int wpad) {
    return r >= min_pad_rows(wc) && r % kPadRowBlock == 0 && r >= wpad;
}
// The same for row k of a wave of the 256-row chain holding nrw rows.
__host__ __device__ constexpr bool wide_stops_at_row(int k, int nrw) {
    return k >= kWideMinRows && k % kWideRowBlock == 0 && k >= nrw;
}
// rows [*r0, *r0 + *nr) of the padded strip go to wave q (0-based) of the chain
__host__ __device__ inline void wide_rows(int w, int q, int* r0, int* nr) {
    const int blocks = wide_pad_rows(w) / kWideRowBlock;
    const int base = blocks / kWideWaves, extra = blocks % kWideWaves;
    *r0 = kWideRowBlock * (q * base + (q < extra ? q : extra));
    *nr = kWideRowBlock * (base + (q < extra ? 1 : 0));
}

// Window capacity class of a window length: 16, 32, 64, 128 or 256.
inline int w_class(int w) { return w <= 16 ? 16 : w <= 32 ? 32 : w <= 64 ? 64 : w <= 128 ? 128 : 256; }

hipError_t launch_encode(const uint8_t* raw, int64_t len, const uint8_t* map256, int x_side,
                         uint16_t* out, int64_t out_len, hipStream_t stream, int sep = -1);
hipError_t launch_seaweed(const PlotArgs& a, hipStream_t stream);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream);
hipError_t launch_dp(const PlotArgs& a, hipStream_t stream);
hipError_t launch_blcs(const PlotArgs& a, hipStream_t stream);
// bitmap, indel and dot list of a finished plot (at wout, row stride ldo)
hipError_t launch_epilogue(const PlotArgs& a, const uint8_t* wout, int64_t ldo, hipStream_t stream);
// Per-unit code paths of the batched kernels: a window class, and whether
// the window fills it (exact) or is shorter (padded strip).
enum BatchVariant {
    kBatch16, kBatch16Short, kBatch32, kBatch32Short,  // group 0
    kBatch64, kBatch64Short,                           // group 1
    kBatch128, kBatch128Short,                         // group 2 (two waves per strip)
};
constexpr int kBatchGroups = 3;
constexpr int batch_group(int variant) { return variant <= kBatch32Short ? 0 : variant <= kBatch64Short ? 1 : 2; }
constexpr int kBatchMaxW = 128;            // longer windows leave the batched kernels
// the code path of a window w <= kBatchMaxW
inline int batch_variant(int w) {
    switch (w_class(w)) {
        case 16: return w == 16 ? kBatch16 : kBatch16Short;
        case 32: return w == 32 ? kBatch32 : kBatch32Short;
        case 64: return w == 64 ? kBatch64 : kBatch64Short;
        default: return w == 128 ? kBatch128 : kBatch128Short;
    }
}
// waves per SIMD the one-wave groups are compiled for (their largest class)
constexpr int group_waves_per_simd(int grp) { return grp == 0 ? min_waves_per_simd(32) : min_waves_per_simd(64); }
// resident waves per CU of a group's kernel (the default persistent grid)
inline int batch_waves_per_cu(int group) {
    const int per_simd = group == 0   ? group_waves_per_simd(0)
                         : group == 1 ? group_waves_per_simd(1)
                                      : min_waves_per_simd_split(128);
    return 4 * per_simd;  // four SIMDs per CU
}
// One group's persistent launch over its njobs table entries (unit0 counted
// from the group's first unit), grid workgroups (group 2: two waves each).
// sparse: some job stores strided windows or lists dots (the kernel variant
// with those flushes).  The counter is zeroed first by a kernel of its own.
hipError_t launch_batch(int group, const JobDesc* jobs_dev, int32_t njobs, int64_t total_units,
                        unsigned long long* counter, int32_t grid, bool sparse, hipStream_t stream);
// *ptrs[k] = 0 for k < n
hipError_t launch_zero_each(unsigned long long* const* ptrs, int32_t n, hipStream_t stream);

// The exact threshold filter for dot lists (filter.hip): from the probe
// strips' listed entries (every h-th x-window from `first`, listed at
// threshold - h / 2), the dots of every row.  If the probe list overflowed,
// nothing is listed and *fallback is set.
struct FilterArgs {
    const uint16_t* xf;  // f-codes of x
    const uint16_t* yg;  // g-codes of y
    const DotRec* probe;
    int64_t probe_cap;
    const unsigned long long* probe_count;
    int64_t rows;        // x-windows of the plot
    int64_t first;       // the first probe row (the probes are first, first + h, ...)
    int32_t w, sigma, h, threshold;
    DotRec* dots;        // the caller's list (may be null while counting)
    int64_t dot_cap;
    unsigned long long* dot_count;
    uint32_t* fallback;
    int32_t cus;         // CUs of the device: the grid is every workgroup of 64 lanes that fits on them at
                         // once, at most 32 per CU (the kernel strides over the entries)
};
hipError_t launch_candidates(const FilterArgs& f, hipStream_t stream);

// The fixed device scratch of the allocation-free batch (batch.hip): its
// size, and its address on `device` (looked up once per device, with that
// device current).
constexpr size_t kNoAllocScratchBytes = 1u << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int device, uint8_t** ptr);
// Copy `bytes` (a multiple of 4) host bytes to device memory dst in stream
// order, carried in the arguments of small kernels (kUploadChunkWords dwords
// each): the host bytes may be reused on return.
constexpr int kUploadChunkWords = 960;
hipError_t launch_upload(uint8_t* dst, const uint8_t* src, size_t bytes, hipStream_t stream);

}  // namespace wlcs
