// Host runtime of the alignment-plot library: the C ABI declared in
// include/wlcs.h.  Validates arguments before anything is enqueued, stages the
// host strings through pinned buffers, and enqueues the encoding kernel and the
// plot kernels on the caller's stream.  Per-call device scratch is taken with
// stream-ordered allocation, so calls on different streams never share it.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/wlcs.h"
#include "kernels.hpp"

#include "runtime.hpp"

namespace wlcs {
// probe.hip: blocks x 256 threads of independent packed 16-bit VALU chains
hipError_t launch_valu_peak(uint32_t* out, int32_t blocks, int32_t iters, hipStream_t stream);
hipError_t launch_valu_issue(uint32_t* out, int32_t kind, int32_t blocks, int32_t k, int32_t iters,
                             hipStream_t stream);
}  // namespace wlcs

using wlcs_rt::kMaxSlots;
using wlcs_rt::Slot;
using wlcs_rt::TileRule;

namespace {

// Append a tiling rule (later rules win).  A rule for exactly the same range
// replaces the earlier one, so setting a range again never fills the table.
int add_rule(TileRule* rules, int& nrules, TileRule r) {
    int k = 0;
    for (int i = 0; i < nrules; ++i)
        if (!(rules[i].lo == r.lo && rules[i].hi == r.hi)) rules[k++] = rules[i];
    nrules = k;
    if (nrules == 16) return WLCS_ENOMEM;
    rules[nrules++] = r;
    return WLCS_OK;
}

// Switch to the context's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = (prev == dev) || (hipSetDevice(dev) == hipSuccess);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int fail(wlcs_ctx* ctx, hipError_t e) {
    if (ctx) ctx->last_hip = (int)e;
    return e == hipErrorOutOfMemory ? WLCS_ENOMEM : WLCS_EHIP;
}

int64_t n_windows(int64_t len, int32_t w, bool full) {
    const int64_t k = len - w + (full ? 1 : 0);
    return k > 0 ? k : 0;
}

// Units (64 strips, one tile pair) resident per SIMD for the single-plot
// kernel of a window class, as the tile model counts them: its waves per SIMD
// (the register budget; LDS allows 4 more at 8.7 KB per wave for the
// 32-window flush and 3 at 12.8 KB for the 64-window one).  A score-plot
// class that splits a strip over two waves counts one unit per SIMD: its
// waves fit 2 or 3 per SIMD, but the tilings measured fastest on the GPU are
// the ones the model picks with one.  The 256-row class chains four waves per
// unit at three waves per SIMD: 0.75 units per SIMD, which puts the model's
// choices next to the tilings measured fastest (wlcs_tune_plot) on 30,000 x
// 30,000 protein plots.
double units_per_simd(int wc, int ws, int w) {
    if (ws == 2) {  // score plots: the separator schedule, classes of 8 rows
        const int dc = (wc + 7) / 8 * 8;
        return wlcs::dl_split(dc) ? 1.0 : (double)wlcs::min_waves_per_simd_dl(dc);
    }
    if (wc == 256) return 3.0 / wlcs::kWideWaves;
    const int regs = wc <= 32 ? 4 : wc == 64 ? 3 : wc == 128 ? 2 : 1;
    const int lds = wc >= 64 ? 3 : 4;
    return std::min(regs, lds);
}

// Units (workgroups) that fit on one CU at once.
int units_per_cu(int wc, int ws, int w) {
    if (ws == 2) {
        const int dc = (wc + 7) / 8 * 8;
        return wlcs::dl_split(dc) ? 4 * wlcs::min_waves_per_simd_dl_split(dc) / 2 : 4 * wlcs::min_waves_per_simd_dl(dc);
    }
    return (int)(4 * units_per_simd(wc, ws, w));
}

// Tile pairs of a row of cols windows with long tiles of `tile` windows for
// at most nbig_max leading pairs (never past the row's end) and tiles of tile2
// after them.
void set_tiles(wlcs::PlotArgs& a, int64_t cols, int32_t tile, int32_t tile2, int64_t nbig_max) {
    const int64_t nbig = tile2 == tile ? 0 : std::max<int64_t>(0, std::min<int64_t>(nbig_max, cols / (2 * (int64_t)tile)));
    const int64_t rest = cols - 2 * nbig * tile;
    a.tile = tile;
    a.tile2 = tile2;
    a.nbig = (int32_t)nbig;
    a.npairs = (int32_t)(nbig + (rest + 2 * (int64_t)tile2 - 1) / (2 * (int64_t)tile2));
}

// Greedy list scheduling of units over `slots` equal slots, in launch order:
// each unit starts on the slot that frees first.  The slots are kept as levels
// (free time, number of slots); k units of d columns each are placed level by
// level, a whole level at a time.
struct SlotLevels {
    std::vector<std::pair<int64_t, int64_t>> lv;  // ascending free time
    explicit SlotLevels(int64_t slots) : lv{{0, slots}} {}
    void add(int64_t t, int64_t c) {
        if (c <= 0) return;
        auto it = std::lower_bound(lv.begin(), lv.end(), std::make_pair(t, (int64_t)0));
        if (it != lv.end() && it->first == t)
            it->second += c;
        else
            lv.insert(it, {t, c});
    }
    void place(int64_t k, int64_t d) {
        while (k > 0) {
            const int64_t tau = lv[0].first, c = lv[0].second;
            lv.erase(lv.begin());
            if (lv.empty() || k < c * ((lv[0].first - tau + d - 1) / d)) {
                // the units run out before this level reaches the next one
                const int64_t r = k / c, q = k % c;
                add(tau + r * d, c - q);
                add(tau + (r + 1) * d, q);
                return;
            }
            const int64_t n = (lv[0].first - tau + d - 1) / d;  // rounds until the next level
            k -= c * n;
            add(tau + n * d, c);
        }
    }
    int64_t makespan() const { return lv.back().first; }
};

// Time (in combed columns per slot) of a plot's units under a tiling.
int64_t tiling_makespan(const wlcs::PlotArgs& a, int64_t nblocks, int64_t cols, int32_t w, int64_t slots) {
    SlotLevels s(slots);
    const int64_t t2 = a.tile2 > 0 ? a.tile2 : a.tile;
    const int64_t nbig = a.tile2 > 0 ? a.nbig : 0;
    const int64_t n2 = a.npairs - nbig;
    if (nbig > 0) s.place(nbig * nblocks, a.tile + w - 1);
    if (n2 > 1) s.place((n2 - 1) * nblocks, t2 + w - 1);
    if (n2 > 0) {
        int64_t start;
        const int64_t last = wlcs::pair_tile(cols, a.tile, t2, nbig, a.npairs - 1, &start);
        s.place(nblocks, last + w - 1);
    }
    return s.makespan();
}

// Tiles for the seaweed kernel.  A unit (64 strips, one tile pair) combs
// tlen + w - 1 columns; the units start in launch order on the wave slots of
// the SIMDs as these free up.  Long tiles waste little on the w - 1 columns
// that each tile combs before its first complete window; short ones keep the
// launch's tail short.  So the pairs of every strip block may start with long
// tiles and end with short ones.  Every candidate (one length, or two with a
// few counts of long pairs) is scored by the finishing time of a greedy list
// schedule of its units over SIMDs x resident units equal slots; the fastest
// wins (the longer tiles on ties).  A context rule (wlcs_ctx_set_tile or
// wlcs_ctx_set_tiles) overrides the choice, and a tiling measured for the
// shape (wlcs_tune_plot) overrides the model.
// The choice for a shape is kept in a small cache of the context.
void choose_tiles(wlcs_ctx* ctx, wlcs::PlotArgs& a, int64_t rows, int64_t cols, int32_t w, int ws = 1) {
    for (int r = ctx->nrules - 1; r >= 0; --r) {
        const TileRule& R = ctx->rules[r];
        if (w >= R.lo && w <= R.hi) {
            set_tiles(a, cols, R.tile, R.tile2 > 0 ? R.tile2 : R.tile, R.nbig);
            return;
        }
    }
    if (const wlcs_rt::TileChoice* c = wlcs_rt::find_tuned(ctx, rows, cols, w, ws)) {
        set_tiles(a, cols, c->tile, c->tile2 > 0 ? c->tile2 : c->tile, c->nbig);
        return;
    }
    for (const wlcs_rt::TileChoice& c : ctx->tile_cache) {
        if (c.rows == rows && c.cols == cols && c.w == w && c.ws == ws) {
            a.tile = c.tile;
            a.tile2 = c.tile2;
            a.nbig = c.nbig;
            a.npairs = c.npairs;
            return;
        }
    }
    static const int32_t cand[] = {64, 128, 192, 256, 384, 512, 768, 1024, 1280, 1536, 2048, 2560, 3072, 4096, 6144, 8192, 12288, 16384};
    const int64_t nblocks = (rows + 63) / 64;
    const int wcl = ws == 2 ? w : wlcs::w_class(w);
    const int64_t slots = (int64_t)(4.0 * ctx->cus * units_per_simd(wcl, ws, w));
    // long tiles only with about as many long units as fit on the GPU at once
    // (at least 85%): then every CU starts (nearly) full of long units,
    // whichever CUs the units land on.  With far fewer, some CUs can end up
    // with several long units and others with none, and the launch waits for
    // the former (measured: 64% of the resident units gave launches of either
    // 4.4 or 5.7 ms; 91-92% gave steady times).
    const int64_t resident = (int64_t)ctx->cus * units_per_cu(wcl, ws, w);
    const int64_t cap = std::max<int64_t>(64, (cols + 63) / 64 * 64);
    int64_t best_t = INT64_MAX;
    wlcs::PlotArgs best = a;
    auto consider = [&](int32_t t, int32_t t2, int64_t nbig) {
        wlcs::PlotArgs c = a;
        set_tiles(c, cols, t, t2, nbig);
        const int64_t mk = tiling_makespan(c, nblocks, cols, w, slots);
        if (mk <= best_t) {
            best_t = mk;
            best = c;
        }
    };
    for (int32_t t : cand) {
        if (t > cap && t > 64) break;
        consider(t, t, 0);
        const int64_t nb_max = cols / (2 * (int64_t)t);
        for (int32_t t2 : cand) {
            if (t2 >= t) break;
            for (int64_t nb = std::max<int64_t>(1, nb_max - 7); nb <= nb_max; ++nb)
                if (20 * nb * nblocks >= 17 * resident) consider(t, t2, nb);
        }
    }
    a.tile = best.tile;
    a.tile2 = best.tile2;
    a.nbig = best.nbig;
    a.npairs = best.npairs;
    wlcs_rt::TileChoice& slot = ctx->tile_cache[ctx->tile_cache_next];
    ctx->tile_cache_next = (ctx->tile_cache_next + 1) % wlcs_rt::kTileCache;
    slot.rows = rows;
    slot.cols = cols;
    slot.w = w;
    slot.ws = ws;
    slot.tile = a.tile;
    slot.tile2 = a.tile2;
    slot.nbig = a.nbig;
    slot.npairs = a.npairs;
}

// One tile length (the DP and BLCS paths, the batched kernel).
void uniform_tiles(wlcs::PlotArgs& a, int64_t cols, int32_t tile) { set_tiles(a, cols, tile, tile, 0); }

struct Prepared {
    int64_t rows = 0, cols = 0;
    uint16_t* xf = nullptr;
    uint16_t* yg = nullptr;
};

int validate(const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, int32_t w, const uint8_t* alphabet,
             int32_t sigma, uint8_t map[256]) {
    if (w < 1 || w > WLCS_MAX_W) return WLCS_ERANGE;
    if (m < 0 || n < 0 || m > WLCS_MAX_LEN || n > WLCS_MAX_LEN) return WLCS_ERANGE;
    if (!alphabet || sigma < 1 || sigma > WLCS_MAX_SIGMA) return WLCS_EALPHABET;
    memset(map, 0xFF, 256);
    for (int c = 0; c < sigma; ++c) {
        if (map[alphabet[c]] != 0xFF) return WLCS_EALPHABET;  // repeated letter
        map[alphabet[c]] = (uint8_t)c;
    }
    if ((m > 0 && !x) || (n > 0 && !y)) return WLCS_EINVAL;
    for (int64_t i = 0; i < m; ++i)
        if (map[x[i]] == 0xFF) return WLCS_EALPHABET;
    for (int64_t i = 0; i < n; ++i)
        if (map[y[i]] == 0xFF) return WLCS_EALPHABET;
    return WLCS_OK;
}

// Copy `bytes` host bytes to device memory dst on `stream` through one of the
// context's pinned slots (the host buffer may be reused on return).
// A pinned staging slot of at least `bytes` (with a device buffer as large
// when `device`) whose last work has completed: the first idle one from the
// rotation (a query, no wait), else a new one while fewer than kMaxSlots
// exist, else the next one in turn after its work is done.  So work queued
// behind other work on a busy stream does not hold the host back while slots
// are to be had, and no device memory is allocated or freed per call
// (a stream-ordered free costs the host about half a millisecond while the
// stream has work queued).  Capacities grow in powers of two from 1 MiB
// (each growth frees the old buffers, and freeing device memory waits for the
// device).
int acquire_slot(wlcs_ctx* ctx, size_t bytes, Slot*& out, bool device = false) {
    out = nullptr;
    Slot* pick = nullptr;
    for (int k = 0; k < ctx->nslots && !pick; ++k) {
        Slot& sl = ctx->slots[(ctx->next_slot + k) % ctx->nslots];
        if (!sl.pending) {
            pick = &sl;
            break;
        }
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipSuccess) {
            sl.pending = false;
            pick = &sl;
        } else if (q != hipErrorNotReady) {
            return fail(ctx, q);
        }
    }
    hipError_t e;
    if (!pick && ctx->nslots < kMaxSlots) {
        Slot& sl = ctx->slots[ctx->nslots];
        if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) return fail(ctx, e);
        ++ctx->nslots;
        pick = &sl;
    }
    if (!pick) {
        Slot& sl = ctx->slots[ctx->next_slot % ctx->nslots];
        if ((e = hipEventSynchronize(sl.done)) != hipSuccess) return fail(ctx, e);
        sl.pending = false;
        pick = &sl;
    }
    ctx->next_slot = (int)(pick - ctx->slots + 1) % ctx->nslots;
    size_t cap = 1 << 20;
    while (cap < bytes) cap <<= 1;
    if (pick->cap < bytes) {
        if (pick->buf) (void)hipHostFree(pick->buf);
        pick->buf = nullptr;
        pick->cap = 0;
        if ((e = hipHostMalloc((void**)&pick->buf, cap, hipHostMallocDefault)) != hipSuccess) return fail(ctx, e);
        pick->cap = cap;
    }
    if (device && pick->dcap < bytes) {
        if (pick->dbuf) (void)hipFree(pick->dbuf);
        pick->dbuf = nullptr;
        pick->dcap = 0;
        if ((e = hipMalloc((void**)&pick->dbuf, cap)) != hipSuccess) return fail(ctx, e);
        pick->dcap = cap;
    }
    out = pick;
    return WLCS_OK;
}

int stage_copy(wlcs_ctx* ctx, const void* src, size_t bytes, void* dst, hipStream_t stream) {
    if (bytes == 0) return WLCS_OK;
    Slot* slot = nullptr;
    int st = acquire_slot(ctx, bytes, slot);
    if (st != WLCS_OK) return st;
    Slot& sl = *slot;
    hipError_t e;
    memcpy(sl.buf, src, bytes);
    if ((e = hipMemcpyAsync(dst, sl.buf, bytes, hipMemcpyHostToDevice, stream)) != hipSuccess) return fail(ctx, e);
    if ((e = hipEventRecord(sl.done, stream)) != hipSuccess) return fail(ctx, e);
    sl.pending = true;
    return WLCS_OK;
}

// Copy x and y into a pinned slot, then into the slot's device buffer, and
// encode them into xf (xf_len codes) and yg (yg_len codes), device arrays of
// the caller (either may be null); the slot is free again once the encode
// kernels are done.
int stage_encode(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, const uint8_t map[256],
                 uint16_t* xf, int64_t xf_len, uint16_t* yg, int64_t yg_len, hipStream_t stream, int sep = -1) {
    const size_t need = (size_t)(m + n);
    const uint8_t* raw = nullptr;  // device copy of x then y (none when both are empty: padding only)
    Slot* slot = nullptr;
    hipError_t e;
    if (need > 0) {
        const int st = acquire_slot(ctx, need, slot, true);
        if (st != WLCS_OK) return st;
        memcpy(slot->buf, x, (size_t)m);
        memcpy(slot->buf + m, y, (size_t)n);
        if ((e = hipMemcpyAsync(slot->dbuf, slot->buf, need, hipMemcpyHostToDevice, stream)) != hipSuccess)
            return fail(ctx, e);
        raw = slot->dbuf;
    }
    if (xf && (e = wlcs::launch_encode(raw, m, map, 1, xf, xf_len, stream, sep)) != hipSuccess) return fail(ctx, e);
    if (yg && (e = wlcs::launch_encode(raw + m, n, map, 0, yg, yg_len, stream, sep)) != hipSuccess)
        return fail(ctx, e);
    if (slot) {
        if ((e = hipEventRecord(slot->done, stream)) != hipSuccess) return fail(ctx, e);
        slot->pending = true;
    }
    return WLCS_OK;
}

// Code arrays of one plot call (stream-ordered allocations, released after
// the plot) holding x and y encoded.
int upload(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, const uint8_t map[256],
           int64_t xf_len, int64_t yg_len, hipStream_t stream, Prepared& p, int sep = -1) {
    if (m + n == 0) return WLCS_OK;
    hipError_t e;
    if (xf_len > 0 && (e = hipMallocAsync((void**)&p.xf, (size_t)xf_len * 2, stream)) != hipSuccess)
        return fail(ctx, e);
    if (yg_len > 0 && (e = hipMallocAsync((void**)&p.yg, (size_t)yg_len * 2, stream)) != hipSuccess)
        return fail(ctx, e);
    return stage_encode(ctx, x, m, y, n, map, p.xf, xf_len, p.yg, yg_len, stream, sep);
}

void release(Prepared& p, hipStream_t stream) {
    if (p.xf) (void)hipFreeAsync(p.xf, stream);
    if (p.yg) (void)hipFreeAsync(p.yg, stream);
    p = Prepared();
}

enum class Path { Seaweed, Dp, Blcs };

// Code-array lengths (16-bit elements) the kernels read for a plot: x is read
// up to 64 strips past the last block plus a window, y up to the end of the
// last tile pair (seaweed) or one 128-window chunk (DP) past the last window,
// plus a window.
void needed_lengths(Path path, int64_t rows, int64_t cols, int32_t w, const wlcs::PlotArgs& a, int64_t& xf_len,
                    int64_t& yg_len) {
    const int wc = wlcs::w_class(w);
    xf_len = (rows + 63) / 64 * 64 + wc + 64;
    if (path == Path::Seaweed) {
        const int64_t t2 = a.tile2 > 0 ? a.tile2 : a.tile;
        const int64_t nbig = a.tile2 > 0 ? a.nbig : 0;
        yg_len = 2 * nbig * a.tile + 2 * (a.npairs - nbig) * t2 + wc + 64;
    } else {
        yg_len = (cols + 127) / 128 * 128 + wc + 64;
    }
}

// Host-side checks shared by every plot entry point (no device access).
int check_outputs(int64_t rows, int64_t cols, uint8_t* out, int64_t ld, uint64_t* bitmap, int64_t ld_words,
                  int32_t threshold, uint16_t* indel, int64_t ld_indel) {
    if (rows > 0 && cols > 0) {
        if (!out && !bitmap && !indel) return WLCS_EINVAL;
        if (out && ld < cols) return WLCS_EINVAL;
        if (bitmap && (ld_words < (cols + 63) / 64 || threshold < 0 || threshold > 255)) return WLCS_EINVAL;
        if (indel && ld_indel < cols) return WLCS_EINVAL;
    }
    return WLCS_OK;
}

wlcs::PlotArgs make_args(int64_t rows, int64_t cols, int32_t w, uint8_t* out, int64_t ld, uint64_t* bitmap,
                         int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel) {
    wlcs::PlotArgs a{};
    a.rows = rows;
    a.cols = cols;
    a.w = w;
    a.threshold = threshold;
    a.wlcs = out;
    a.ld = ld;
    a.bitmap32 = (uint32_t*)bitmap;
    a.ld_words32 = ld_words * 2;
    a.indel = indel;
    a.ld_indel = ld_indel;
    return a;
}

hipError_t launch_path(Path path, const wlcs::PlotArgs& a, hipStream_t stream) {
    switch (path) {
        case Path::Seaweed: return wlcs::launch_seaweed(a, stream);
        case Path::Dp: return wlcs::launch_dp(a, stream);
        default: return wlcs::launch_blcs(a, stream);
    }
}

int plot_common(Path path, wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, int32_t w,
                const uint8_t* alphabet, int32_t sigma, uint8_t* out, int64_t ld, uint64_t* bitmap,
                int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel, uint32_t flags,
                void* stream_) {
    // every argument is checked on the host before the context is touched
    if (flags & ~WLCS_FULL_RANGE) return WLCS_EINVAL;
    uint8_t map[256];
    int st = validate(x, m, y, n, w, alphabet, sigma, map);
    if (st != WLCS_OK) return st;
    const bool full = (flags & WLCS_FULL_RANGE) != 0;
    const int64_t rows = n_windows(m, w, full), cols = n_windows(n, w, full);
    st = check_outputs(rows, cols, out, ld, bitmap, ld_words, threshold, indel, ld_indel);
    if (st != WLCS_OK) return st;
    if (!ctx) return WLCS_EINVAL;
    if (rows == 0 || cols == 0) return WLCS_OK;

    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    hipStream_t stream = (hipStream_t)stream_;

    wlcs::PlotArgs a = make_args(rows, cols, w, out, ld, bitmap, ld_words, threshold, indel, ld_indel);
    if (path == Path::Seaweed)
        choose_tiles(ctx, a, rows, cols, w);
    else
        uniform_tiles(a, cols, 64);
    int64_t xf_len, yg_len;
    needed_lengths(path, rows, cols, w, a, xf_len, yg_len);
    Prepared p;
    st = upload(ctx, x, m, y, n, map, xf_len, yg_len, stream, p);
    if (st != WLCS_OK) {
        release(p, stream);
        return st;
    }
    a.xf = p.xf;
    a.yg = p.yg;
    a.sigma = sigma;
    hipError_t e = launch_path(path, a, stream);
    release(p, stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

}  // namespace

// A device-resident, encoded pair of strings.
namespace {

constexpr int32_t kMaxTile = 32768;

// Record that work just enqueued on `stream` reads the pair's codes (see
// wlcs_pair::use_event).  Nothing to do on the creation stream, nor while the
// stream is being captured into a graph (the graph's owner keeps the pair
// alive for as long as it replays it).
hipError_t note_use(const wlcs_pair* p, hipStream_t stream) {
    if (stream == p->stream) return hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return e;
    if (cs != hipStreamCaptureStatusNone) return hipSuccess;
    int k = 0;
    while (k < p->nuses && p->use_stream[k] != stream) ++k;
    if (k == p->nuses) {
        if (p->nuses < wlcs_pair::kUses) {
            if ((e = hipEventCreateWithFlags(&p->use_event[k], hipEventDisableTiming)) != hipSuccess) return e;
            ++p->nuses;
        } else {  // retire the oldest entry: the creation stream waits for it now
            k = p->next_use;
            p->next_use = (p->next_use + 1) % wlcs_pair::kUses;
            if ((e = hipStreamWaitEvent(p->stream, p->use_event[k], 0)) != hipSuccess) return e;
        }
        p->use_stream[k] = stream;
    }
    return hipEventRecord(p->use_event[k], stream);
}

// Code-array capacities of a resident pair of m and n letters: room for any
// window (<= 256 rows of capacity) and any tile pair (<= 2 kMaxTile windows)
// past the last letter.
void pair_caps(int64_t m, int64_t n, int64_t& xf_cap, int64_t& yg_cap) {
    xf_cap = m + 64 + 256 + 64;
    yg_cap = n + 2 * (int64_t)kMaxTile + 128 + 256 + 64;
}

int pair_plot_common(Path path, wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, uint8_t* out, int64_t ld,
                     uint64_t* bitmap, int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel,
                     uint32_t flags, void* stream_) {
    if (flags & ~WLCS_FULL_RANGE) return WLCS_EINVAL;
    if (!pair) return WLCS_EINVAL;
    if (w < 1 || w > WLCS_MAX_W) return WLCS_ERANGE;
    const bool full = (flags & WLCS_FULL_RANGE) != 0;
    const int64_t rows = n_windows(pair->m, w, full), cols = n_windows(pair->n, w, full);
    int st = check_outputs(rows, cols, out, ld, bitmap, ld_words, threshold, indel, ld_indel);
    if (st != WLCS_OK) return st;
    if (!ctx || ctx->device != pair->device) return WLCS_EINVAL;
    if (rows == 0 || cols == 0) return WLCS_OK;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    wlcs::PlotArgs a = make_args(rows, cols, w, out, ld, bitmap, ld_words, threshold, indel, ld_indel);
    if (path == Path::Seaweed)
        choose_tiles(ctx, a, rows, cols, w);
    else
        uniform_tiles(a, cols, 64);
    int64_t xf_len, yg_len;
    needed_lengths(path, rows, cols, w, a, xf_len, yg_len);
    if (xf_len > pair->xf_cap || yg_len > pair->yg_cap) return WLCS_EINVAL;  // cannot happen for valid tiles
    a.xf = pair->xf;
    a.yg = pair->yg;
    a.sigma = pair->sigma;
    hipStream_t stream = (hipStream_t)stream_;
    hipError_t e = launch_path(path, a, stream);
    if (e == hipSuccess) e = note_use(pair, stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

// Strided and sparse plots on a resident pair (both paths).
int strided_common(Path path, wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, int32_t hx, int32_t hy, uint8_t* out,
                   int64_t ld, uint64_t* bitmap, int64_t ld_words, int32_t threshold, uint16_t* indel,
                   int64_t ld_indel, wlcs_dot* dots, int64_t dot_cap, uint64_t* dot_count, uint32_t flags,
                   void* stream_) {
    if (flags & ~WLCS_FULL_RANGE) return WLCS_EINVAL;
    if (!pair) return WLCS_EINVAL;
    if (w < 1 || w > WLCS_MAX_W || hx < 1 || hy < 1) return WLCS_ERANGE;
    const bool full = (flags & WLCS_FULL_RANGE) != 0;
    const int64_t rows_all = n_windows(pair->m, w, full), cols_all = n_windows(pair->n, w, full);
    const int64_t rows = (rows_all + hx - 1) / hx, cols = (cols_all + hy - 1) / hy;
    if (bitmap && hy > 1) return WLCS_EINVAL;  // the dot list serves thresholds on a y-step
    if (rows > 0 && cols > 0 && !out && !bitmap && !indel && !dot_count) return WLCS_EINVAL;
    if (rows > 0 && cols > 0 && (out || bitmap || indel)) {
        const int st = check_outputs(rows, cols, out, ld, bitmap, ld_words, threshold, indel, ld_indel);
        if (st != WLCS_OK) return st;
    }
    if (dot_count && (threshold < 0 || threshold > 255 || dot_cap < 0)) return WLCS_EINVAL;
    if (!dot_count && dots) return WLCS_EINVAL;  // a list needs its counter
    if (dots && rows_all > 0 && cols_all > 0 &&
        ((rows - 1) * (int64_t)hx > 0xFFFFFFFFll || (cols - 1) * (int64_t)hy > 0xFFFFFFFFll))
        return WLCS_ERANGE;  // window starts must fit the record's 32-bit fields
    if (!ctx || ctx->device != pair->device) return WLCS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    hipStream_t stream = (hipStream_t)stream_;
    if (dot_count) {  // the count is written even when the plot is empty
        const hipError_t e = wlcs::launch_zero_u64((unsigned long long*)dot_count, stream);
        if (e != hipSuccess) return fail(ctx, e);
    }
    if (rows == 0 || cols == 0) return WLCS_OK;
    wlcs::PlotArgs a = make_args(rows, path == Path::Seaweed ? cols_all : cols, w, out, ld, bitmap, ld_words,
                                 threshold, indel, ld_indel);
    a.xstride = hx;
    a.hy = hy;
    a.dots = (wlcs::DotRec*)dots;
    a.dot_cap = dots ? dot_cap : 0;
    a.dot_count = (unsigned long long*)dot_count;
    // strips past the last window read a copy of the last one, so the x codes
    // read stay below m + the window class; y as for an unstrided plot
    if (path == Path::Seaweed)
        choose_tiles(ctx, a, rows, a.cols, w);
    else
        uniform_tiles(a, a.cols, 64);
    int64_t xf_len, yg_len;
    needed_lengths(path, 1, path == Path::Seaweed ? a.cols : cols_all, w, a, xf_len, yg_len);
    if (pair->m + wlcs::w_class(w) > pair->xf_cap || yg_len > pair->yg_cap) return WLCS_EINVAL;
    a.xf = pair->xf;
    a.yg = pair->yg;
    a.sigma = pair->sigma;
    hipError_t e = launch_path(path, a, stream);
    if (e == hipSuccess) e = note_use(pair, stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

}  // namespace

struct wlcs_graph {
    int device = 0;
    wlcs::JobDesc* table = nullptr;
    unsigned long long* counter = nullptr;
    unsigned long long** counts = nullptr;  // the jobs' dot counters (zeroed by each replay)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const wlcs_pair*> pairs;  // read by every replay
};

namespace {

int32_t batch_tile(const wlcs_ctx* ctx, int64_t cols, int32_t w) {
    for (int r = ctx->nbatch_rules - 1; r >= 0; --r)
        if (w >= ctx->batch_rules[r].lo && w <= ctx->batch_rules[r].hi) return ctx->batch_rules[r].tile;
    // about equal combing work per unit for every window, and at least two
    // tiles per row so both halves of each register carry work
    int64_t t = (131072 / w + 63) / 64 * 64;
    const int64_t half = ((cols + 1) / 2 + 63) / 64 * 64;
    t = std::min<int64_t>(t, half);
    t = std::max<int64_t>(64, std::min<int64_t>(t, kMaxTile));
    return (int32_t)t;
}

// A batched job with fewer than min_units units (strip blocks x tile pairs)
// under its tile gets the longest shorter tile, in whole 64-window blocks and
// at least 64, that gives it min_units units (or 64 if none does).
void shrink_for_units(wlcs::PlotArgs& a, int64_t rows, int64_t cols, int64_t min_units) {
    const int64_t nblocks = (rows + 63) / 64;
    if (nblocks * (int64_t)a.npairs >= min_units || a.tile <= 64) return;
    const int64_t pairs = (min_units + nblocks - 1) / nblocks;  // pairs per block wanted
    int64_t t = (cols + 2 * pairs - 1) / (2 * pairs);           // windows per tile for that many
    t = std::max<int64_t>(64, t / 64 * 64);
    if (t < a.tile) uniform_tiles(a, cols, (int32_t)t);
}

// One table entry being planned: a job's tile pairs but the last, or its last pair.
struct PlanItem {
    wlcs::JobDesc d;
    double cost;  // of one unit
    bool last;    // the job's last tile pair
    int32_t seq;  // order of creation (ties keep it)
};

struct BatchPlan {
    // jobs with w <= kBatchMaxW, by kernel group, then by decreasing unit cost
    // within a group; a group's unit0 values count from its own first unit
    std::vector<wlcs::JobDesc> table;
    int32_t first[wlcs::kBatchGroups + 1] = {};  // table index of each group's first job
    int64_t units[wlcs::kBatchGroups] = {};      // units of each group
    bool sparse[wlcs::kBatchGroups] = {};        // some job of the group is strided or lists dots
    std::vector<wlcs::PlotArgs> singles;         // longer windows: single-plot launches
    std::vector<unsigned long long*> counts;     // every job's dot counter, zeroed first
    std::vector<PlanItem> items;                 // working list of plan_batch
    // empty again, keeping the vectors' storage for the next batch
    void clear() {
        table.clear();
        singles.clear();
        counts.clear();
        items.clear();
        for (int g = 0; g < wlcs::kBatchGroups; ++g) {
            first[g + 1] = 0;
            units[g] = 0;
            sparse[g] = false;
        }
        first[0] = 0;
    }
};

int plan_batch(wlcs_ctx* ctx, const wlcs_job* jobs, int32_t njobs, BatchPlan& plan) {
    if (!ctx || njobs < 0 || (njobs > 0 && !jobs)) return WLCS_EINVAL;
    using Item = PlanItem;
    std::vector<Item>& items = plan.items;
    for (int32_t k = 0; k < njobs; ++k) {
        const wlcs_job& j = jobs[k];
        if (j.flags & ~WLCS_FULL_RANGE) return WLCS_EINVAL;
        if (!j.pair || j.pair->device != ctx->device) return WLCS_EINVAL;
        if (j.w < 1 || j.w > WLCS_MAX_W || j.hx < 0 || j.hy < 0) return WLCS_ERANGE;
        const int64_t hx = j.hx > 1 ? j.hx : 1, hy = j.hy > 1 ? j.hy : 1;
        const bool full = (j.flags & WLCS_FULL_RANGE) != 0;
        const int64_t rows_all = n_windows(j.pair->m, j.w, full), cols = n_windows(j.pair->n, j.w, full);
        const int64_t rows = (rows_all + hx - 1) / hx, ocols = (cols + hy - 1) / hy;
        if (rows > 0 && ocols > 0 && !j.wlcs && !j.bitmap && !j.indel && !j.dot_count) return WLCS_EINVAL;
        if ((j.bitmap && hy > 1) || (j.dots && !j.dot_count)) return WLCS_EINVAL;
        if (j.dot_count && (j.threshold < 0 || j.threshold > 255 || j.dot_cap < 0)) return WLCS_EINVAL;
        if (j.wlcs || j.bitmap || j.indel) {
            const int st = check_outputs(rows, ocols, j.wlcs, j.ld, j.bitmap, j.ld_words, j.threshold, j.indel,
                                         j.ld_indel);
            if (st != WLCS_OK) return st;
        }
        if (j.dots && rows > 0 && ocols > 0 && ((rows - 1) * hx > 0xFFFFFFFFll || (ocols - 1) * hy > 0xFFFFFFFFll))
            return WLCS_ERANGE;
        if (j.dot_count) plan.counts.push_back((unsigned long long*)j.dot_count);
        if (rows == 0 || cols == 0) continue;
        wlcs::PlotArgs a =
            make_args(rows, cols, j.w, j.wlcs, j.ld, j.bitmap, j.ld_words, j.threshold, j.indel, j.ld_indel);
        a.xf = j.pair->xf;
        a.yg = j.pair->yg;
        a.xstride = hx;
        a.hy = hy;
        a.dots = (wlcs::DotRec*)j.dots;
        a.dot_cap = j.dots ? j.dot_cap : 0;
        a.dot_count = (unsigned long long*)j.dot_count;
        if (j.w > wlcs::kBatchMaxW) {
            choose_tiles(ctx, a, rows, cols, j.w);
            plan.singles.push_back(a);
            continue;
        }
        uniform_tiles(a, cols, batch_tile(ctx, cols, j.w));
        if (ctx->batch_min_units > 0) shrink_for_units(a, rows, cols, ctx->batch_min_units);
        int64_t xf_len, yg_len;
        needed_lengths(Path::Seaweed, rows, cols, j.w, a, xf_len, yg_len);
        if (xf_len > j.pair->xf_cap || yg_len > j.pair->yg_cap) return WLCS_EINVAL;
        Item it;
        it.d.xf = a.xf;
        it.d.yg32 = (const uint32_t*)a.yg;
        it.d.out = a.wlcs;
        it.d.bm32 = a.bitmap32;
        it.d.indel = a.indel;
        it.d.dots = a.dots;
        it.d.dot_count = a.dot_count;
        it.d.g = wlcs::geom_of(a);
        it.d.variant = wlcs::batch_variant(j.w);
        const int grp = wlcs::batch_group(it.d.variant);
        if (hy > 1 || a.dot_count) plan.sparse[grp] = true;
        const int64_t nblocks = (rows + 63) / 64;
        // the pairs before the last one (full tiles), then the last pair
        if (a.npairs > 1) {
            it.d.unit0 = nblocks * (a.npairs - 1);  // unit count for now
            it.d.pr0 = 0;
            it.last = false;
            it.cost = 2.0 * (double)(a.tile + j.w - 1) * (double)j.w;
            it.seq = (int32_t)items.size();
            items.push_back(it);
        }
        int64_t start;
        const int64_t tlast = wlcs::pair_tile(cols, a.tile, a.tile, 0, a.npairs - 1, &start);
        it.d.unit0 = nblocks;
        it.d.pr0 = a.npairs - 1;
        it.last = true;
        it.cost = 2.0 * (double)(tlast + j.w - 1) * (double)j.w;
        it.seq = (int32_t)items.size();
        items.push_back(it);
    }
    // (an unstable sort with the creation order as the last key: the same
    // order as a stable sort, without its temporary buffer)
    std::sort(items.begin(), items.end(), [](const Item& p, const Item& q) {
        const int gp = wlcs::batch_group(p.d.variant), gq = wlcs::batch_group(q.d.variant);
        if (gp != gq) return gp < gq;
        if (p.last != q.last) return q.last;
        if (p.cost != q.cost) return p.cost > q.cost;
        return p.seq < q.seq;
    });
    if (items.size() > 0x7FFFFFFF) return WLCS_ERANGE;  // table entries are counted in int32
    for (const Item& it : items) {
        const int grp = wlcs::batch_group(it.d.variant);
        wlcs::JobDesc d = it.d;
        const int64_t units = d.unit0;
        d.unit0 = plan.units[grp];
        plan.units[grp] += units;
        plan.table.push_back(d);
        plan.first[grp + 1] = (int32_t)plan.table.size();
    }
    for (int grp = 1; grp <= wlcs::kBatchGroups; ++grp)  // groups without jobs start where the last one ended
        plan.first[grp] = std::max(plan.first[grp], plan.first[grp - 1]);
    return WLCS_OK;
}

// Workgroups of a group's persistent grid: the waves per CU set by
// wlcs_ctx_set_batch_grid (else the group's resident capacity), two waves per
// workgroup in the 128-row group.
int batch_grid(const wlcs_ctx* ctx, int group, int64_t units) {
    const int64_t waves = ctx->batch_waves_per_cu > 0 ? ctx->batch_waves_per_cu : wlcs::batch_waves_per_cu(group);
    const int64_t per_cu = group == 2 ? std::max<int64_t>(1, waves / 2) : waves;
    return (int)std::min<int64_t>(units, (int64_t)ctx->cus * per_cu);
}

// Enqueue a planned batch whose job table already sits at table_dev and the
// list of its dot counters at counts_dev; counters holds the groups' work
// counters, 64 bytes apart.  The costliest group (128-row windows) runs first.
hipError_t enqueue_batch(const wlcs_ctx* ctx, const BatchPlan& plan, const wlcs::JobDesc* table_dev,
                         unsigned long long* counters, unsigned long long* const* counts_dev, hipStream_t stream) {
    hipError_t e = wlcs::launch_zero_each(counts_dev, (int32_t)plan.counts.size(), stream);
    for (int grp = wlcs::kBatchGroups - 1; grp >= 0 && e == hipSuccess; --grp) {
        const int32_t n = plan.first[grp + 1] - plan.first[grp];
        if (n > 0)
            e = wlcs::launch_batch(grp, table_dev + plan.first[grp], n, plan.units[grp], counters + 8 * grp,
                                   batch_grid(ctx, grp, plan.units[grp]), plan.sparse[grp], stream);
    }
    for (size_t k = 0; e == hipSuccess && k < plan.singles.size(); ++k) e = wlcs::launch_seaweed(plan.singles[k], stream);
    return e;
}

}  // namespace

extern "C" {

int wlcs_ctx_create(int device, wlcs_ctx** out) {
    if (!out) return WLCS_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return WLCS_EINVAL;
    wlcs_ctx* ctx = new (std::nothrow) wlcs_ctx();
    if (!ctx) return WLCS_ENOMEM;
    ctx->device = device;
    DeviceGuard guard(device);
    if (!guard.ok) {
        delete ctx;
        return WLCS_EHIP;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        ctx->cus = cus;
    // the allocation-free batch's scratch on this device (once per device)
    const hipError_t e = wlcs::scratch_address(device, &ctx->scratch);
    if (e != hipSuccess) {
        ctx->scratch = nullptr;
        ctx->scratch_err = (int)e;
    }
    *out = ctx;
    return WLCS_OK;
}

int wlcs_ctx_destroy(wlcs_ctx* ctx) {
    if (!ctx) return WLCS_OK;
    DeviceGuard guard(ctx->device);
    int st = WLCS_OK;
    for (int i = 0; i < ctx->nslots; ++i) {
        Slot& sl = ctx->slots[i];
        if (sl.pending && hipEventSynchronize(sl.done) != hipSuccess) st = WLCS_EHIP;
        if (sl.buf) (void)hipHostFree(sl.buf);
        if (sl.dbuf) (void)hipFree(sl.dbuf);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    delete ctx;
    return st;
}

int wlcs_ctx_last_hip_error(const wlcs_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

int wlcs_measure_valu_peak(wlcs_ctx* ctx, int32_t iters, double* ops_per_s) {
    if (!ctx || !ops_per_s || iters < 1 || iters > 1000000) return WLCS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    const int32_t blocks = 32 * ctx->cus;  // 128 waves per CU, 32 per SIMD
    uint32_t* out = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc((void**)&out, (size_t)blocks * 256 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = wlcs::launch_valu_peak(out, blocks, iters < 100 ? iters : 100, stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    if (e == hipSuccess) e = wlcs::launch_valu_peak(out, blocks, iters, stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e == hipSuccess && ms > 0.0f)
        *ops_per_s = (double)blocks * 256.0 * (double)iters * 64.0 * 2.0 / (ms * 1e-3);
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (stream) (void)hipStreamDestroy(stream);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return fail(ctx, e);
    return ms > 0.0f ? WLCS_OK : WLCS_EHIP;
}

int wlcs_measure_valu_issue(wlcs_ctx* ctx, int32_t kind, int32_t waves_per_simd, int32_t iters,
                            double* instr_per_s) {
    if (!ctx || !instr_per_s || kind < 0 || kind > 5 || waves_per_simd < 1 || waves_per_simd > 4 || iters < 1 ||
        iters > 1000000)
        return WLCS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    const int32_t blocks = ctx->cus;  // one workgroup of 256 k threads per CU: k waves on each SIMD
    const int32_t k = waves_per_simd;
    uint32_t* out = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc((void**)&out, (size_t)blocks * 256 * k * sizeof(uint32_t));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e == hipSuccess) e = wlcs::launch_valu_issue(out, kind, blocks, k, iters < 1000 ? iters : 1000, stream);
    if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
    if (e == hipSuccess) e = wlcs::launch_valu_issue(out, kind, blocks, k, iters, stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e == hipSuccess && ms > 0.0f) {
        const double per_round = kind == 4 ? 40.0 : (kind == 2 || kind == 3) ? 32.0 : 16.0;
        // waves x rounds x instructions, over the device's SIMDs (four per CU)
        *instr_per_s = (double)blocks * 4.0 * k * (double)iters * per_round / (4.0 * ctx->cus) / (ms * 1e-3);
    }
    for (hipEvent_t x : ev)
        if (x) (void)hipEventDestroy(x);
    if (stream) (void)hipStreamDestroy(stream);
    if (out) (void)hipFree(out);
    if (e != hipSuccess) return fail(ctx, e);
    return ms > 0.0f ? WLCS_OK : WLCS_EHIP;
}

const char* wlcs_status_str(int status) {
    switch (status) {
        case WLCS_OK: return "ok";
        case WLCS_EINVAL: return "invalid argument";
        case WLCS_ERANGE: return "window or length out of range";
        case WLCS_EALPHABET: return "bad alphabet or letter outside the alphabet";
        case WLCS_EHIP: return "HIP runtime error";
        case WLCS_ENOMEM: return "out of memory";
        case WLCS_EIO: return "file could not be written";
        case WLCS_ESCRATCH: return "batch too large for the fixed scratch of wlcs_batch_noalloc";
        default: return "unknown status";
    }
}

int wlcs_ctx_set_tile(wlcs_ctx* ctx, int32_t w_lo, int32_t w_hi, int32_t tile_windows) {
    if (!ctx || w_lo < 1 || w_hi < w_lo || w_hi > WLCS_MAX_W) return WLCS_EINVAL;
    if (tile_windows == 0) {  // drop rules covering this range
        int k = 0;
        for (int r = 0; r < ctx->nrules; ++r)
            if (!(ctx->rules[r].lo >= w_lo && ctx->rules[r].hi <= w_hi)) ctx->rules[k++] = ctx->rules[r];
        ctx->nrules = k;
        return WLCS_OK;
    }
    if (tile_windows < 64 || tile_windows > 32768 || tile_windows % 64) return WLCS_EINVAL;
    return add_rule(ctx->rules, ctx->nrules, TileRule{w_lo, w_hi, tile_windows, tile_windows, 0});
}

int wlcs_ctx_set_tiles(wlcs_ctx* ctx, int32_t w_lo, int32_t w_hi, int32_t long_tile, int32_t short_tile,
                       int32_t long_pairs) {
    if (!ctx || w_lo < 1 || w_hi < w_lo || w_hi > WLCS_MAX_W) return WLCS_EINVAL;
    if (long_tile == 0) return wlcs_ctx_set_tile(ctx, w_lo, w_hi, 0);
    auto bad = [](int32_t t) { return t < 64 || t > 32768 || t % 64 != 0; };
    if (bad(long_tile) || bad(short_tile) || long_pairs < 0) return WLCS_EINVAL;
    return add_rule(ctx->rules, ctx->nrules, TileRule{w_lo, w_hi, long_tile, short_tile, long_pairs});
}

int wlcs_plot(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, int32_t w,
              const uint8_t* alphabet, int32_t sigma, uint8_t* wlcs, int64_t ld, uint64_t* bitmap,
              int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel, uint32_t flags,
              void* stream) {
    return plot_common(Path::Seaweed, ctx, x, m, y, n, w, alphabet, sigma, wlcs, ld, bitmap, ld_words, threshold,
                       indel, ld_indel, flags, stream);
}

int wlcs_plot_blcs(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, int32_t w,
                   const uint8_t* alphabet, int32_t sigma, uint8_t* wlcs, int64_t ld, uint64_t* bitmap,
                   int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel, uint32_t flags,
                   void* stream) {
    return plot_common(Path::Blcs, ctx, x, m, y, n, w, alphabet, sigma, wlcs, ld, bitmap, ld_words, threshold,
                       indel, ld_indel, flags, stream);
}

int wlcs_plot_dp(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, int32_t w,
                 const uint8_t* alphabet, int32_t sigma, uint8_t* wlcs, int64_t ld, uint64_t* bitmap,
                 int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel, uint32_t flags,
                 void* stream) {
    return plot_common(Path::Dp, ctx, x, m, y, n, w, alphabet, sigma, wlcs, ld, bitmap, ld_words, threshold,
                       indel, ld_indel, flags, stream);
}

int wlcs_score_plot(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n, int32_t w, int32_t step,
                    const uint8_t* alphabet, int32_t sigma, int8_t* score, int64_t ld, uint64_t* bitmap,
                    int64_t ld_words, int32_t threshold, uint32_t flags, void* stream_) {
    if (flags & ~WLCS_FULL_RANGE) return WLCS_EINVAL;
    if (w < 1 || w > WLCS_MAX_SCORE_W || step < 1) return WLCS_ERANGE;
    if (sigma >= WLCS_MAX_SIGMA) return WLCS_EALPHABET;  // one code is kept for the separator
    uint8_t map[256];
    int st = validate(x, m, y, n, w, alphabet, sigma, map);
    if (st != WLCS_OK) return st;
    const bool full = (flags & WLCS_FULL_RANGE) != 0;
    const int64_t rows_all = n_windows(m, w, full), cols = n_windows(n, w, full);
    const int64_t rows = rows_all > 0 ? (rows_all + step - 1) / step : 0;
    if (rows > 0 && cols > 0) {
        if (!score && !bitmap) return WLCS_EINVAL;
        if (score && ld < cols) return WLCS_EINVAL;
        if (bitmap && (ld_words < (cols + 63) / 64 || threshold < -128 || threshold > 127)) return WLCS_EINVAL;
    }
    if (!ctx) return WLCS_EINVAL;
    if (rows == 0 || cols == 0) return WLCS_OK;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    hipStream_t stream = (hipStream_t)stream_;
    // the LCS plot of the blown-up strings x', y' (window 2w), at the strips of
    // x' that start x-windows 0, step, 2 step, ... and the even windows of y'
    const int32_t w2 = 2 * w;
    wlcs::PlotArgs a = make_args(rows, 2 * cols, w2, (uint8_t*)score, ld, bitmap, ld_words,
                                 std::min(std::max(threshold + w, 0), 256), nullptr, 0);
    a.ws = 2;
    a.xstride = 2 * (int64_t)step;
    a.bias = w;
    choose_tiles(ctx, a, rows, a.cols, w2, 2);
    int64_t xf_len, yg_len;
    needed_lengths(Path::Seaweed, rows, a.cols, w2, a, xf_len, yg_len);
    xf_len = (rows + 63) / 64 * 64 * a.xstride + wlcs::w_class(w2) + 64;
    Prepared p;
    st = upload(ctx, x, m, y, n, map, xf_len, yg_len, stream, p, sigma);
    if (st != WLCS_OK) {
        release(p, stream);
        return st;
    }
    a.xf = p.xf;
    a.yg = p.yg;
    hipError_t e = wlcs::launch_seaweed(a, stream);
    release(p, stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

int wlcs_pair_create(wlcs_ctx* ctx, const uint8_t* x, int64_t m, const uint8_t* y, int64_t n,
                     const uint8_t* alphabet, int32_t sigma, void* stream_, wlcs_pair** out) {
    if (!out) return WLCS_EINVAL;
    *out = nullptr;
    uint8_t map[256];
    int st = validate(x, m, y, n, 1, alphabet, sigma, map);
    if (st != WLCS_OK) return st;
    if (!ctx) return WLCS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    hipStream_t stream = (hipStream_t)stream_;
    wlcs_pair* pr = new (std::nothrow) wlcs_pair();
    if (!pr) return WLCS_ENOMEM;
    pr->device = ctx->device;
    pr->m = m;
    pr->n = n;
    pr->sigma = sigma;
    pair_caps(m, n, pr->xf_cap, pr->yg_cap);
    pr->stream = stream;
    hipError_t e = hipMallocAsync((void**)&pr->xf, (size_t)pr->xf_cap * 2, stream);
    if (e == hipSuccess) e = hipMallocAsync((void**)&pr->yg, (size_t)pr->yg_cap * 2, stream);
    if (e != hipSuccess) {
        wlcs_pair_destroy(pr);
        return fail(ctx, e);
    }
    st = stage_encode(ctx, x, m, y, n, map, pr->xf, pr->xf_cap, pr->yg, pr->yg_cap, stream);
    if (st != WLCS_OK) {
        (void)hipStreamSynchronize(stream);
        wlcs_pair_destroy(pr);
        return st;
    }
    *out = pr;
    return WLCS_OK;
}

int wlcs_pair_destroy(wlcs_pair* pair) {
    if (!pair) return WLCS_OK;
    DeviceGuard guard(pair->device);
    int st = WLCS_OK;
    // stream-ordered release on the creation stream (no device-wide wait),
    // after the last work on any other stream that read the codes
    for (int k = 0; k < pair->nuses; ++k)
        if (hipStreamWaitEvent(pair->stream, pair->use_event[k], 0) != hipSuccess) st = WLCS_EHIP;
    if (pair->xf && hipFreeAsync(pair->xf, pair->stream) != hipSuccess) st = WLCS_EHIP;
    if (pair->yg && hipFreeAsync(pair->yg, pair->stream) != hipSuccess) st = WLCS_EHIP;
    for (int k = 0; k < pair->nuses; ++k) (void)hipEventDestroy(pair->use_event[k]);
    delete pair;
    return st;
}

int wlcs_pair_plot(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, uint8_t* wlcs, int64_t ld, uint64_t* bitmap,
                   int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel, uint32_t flags,
                   void* stream) {
    return pair_plot_common(Path::Seaweed, ctx, pair, w, wlcs, ld, bitmap, ld_words, threshold, indel, ld_indel,
                            flags, stream);
}

int wlcs_pair_plot_strided(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, int32_t hx, int32_t hy, uint8_t* wlcs,
                           int64_t ld, uint64_t* bitmap, int64_t ld_words, int32_t threshold, uint16_t* indel,
                           int64_t ld_indel, wlcs_dot* dots, int64_t dot_cap, uint64_t* dot_count, uint32_t flags,
                           void* stream) {
    return strided_common(Path::Seaweed, ctx, pair, w, hx, hy, wlcs, ld, bitmap, ld_words, threshold, indel,
                          ld_indel, dots, dot_cap, dot_count, flags, stream);
}

int wlcs_pair_plot_dp_strided(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, int32_t hx, int32_t hy,
                              uint8_t* wlcs, int64_t ld, uint64_t* bitmap, int64_t ld_words, int32_t threshold,
                              uint16_t* indel, int64_t ld_indel, wlcs_dot* dots, int64_t dot_cap,
                              uint64_t* dot_count, uint32_t flags, void* stream) {
    return strided_common(Path::Dp, ctx, pair, w, hx, hy, wlcs, ld, bitmap, ld_words, threshold, indel, ld_indel,
                          dots, dot_cap, dot_count, flags, stream);
}

int wlcs_pair_dots_filtered(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, int32_t threshold,
                            int32_t probe_step, int64_t probe_cap, wlcs_dot* dots, int64_t dot_cap,
                            uint64_t* dot_count, uint32_t flags, void* stream_) {
    if (flags & ~WLCS_FULL_RANGE) return WLCS_EINVAL;
    if (!pair || !dot_count || (!dots && dot_cap > 0) || dot_cap < 0 || probe_cap < 0) return WLCS_EINVAL;
    if (w < 1 || w > WLCS_MAX_W || probe_step < 1) return WLCS_ERANGE;
    if (threshold < 0 || threshold > 255) return WLCS_EINVAL;
    const bool full = (flags & WLCS_FULL_RANGE) != 0;
    const int64_t rows = n_windows(pair->m, w, full), cols = n_windows(pair->n, w, full);
    if (rows > 0 && cols > 0 && ((rows - 1) > 0xFFFFFFFFll || (cols - 1) > 0xFFFFFFFFll))
        return WLCS_ERANGE;  // window starts must fit the record's 32-bit fields
    if (!ctx || ctx->device != pair->device) return WLCS_EINVAL;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    hipStream_t stream = (hipStream_t)stream_;
    hipError_t e = wlcs::launch_zero_u64((unsigned long long*)dot_count, stream);
    if (e != hipSuccess) return fail(ctx, e);
    if (rows == 0 || cols == 0) return WLCS_OK;
    const int64_t h = probe_step;
    // probe strips first, first + h, ..., starting at half the remainder of
    // (rows - 1) / h, so that the rows before the first probe and after the
    // last one are at most floor(h / 2) rows from it, like every other row
    const int64_t first = ((rows - 1) % h) / 2;
    const int64_t probe_rows = (rows - 1 - first) / h + 1;
    if (probe_cap == 0)  // about one entry in 32 of the probe strips, at least 64 Ki, at most 128 Mi
        probe_cap = std::min<int64_t>(std::max<int64_t>(65536, probe_rows * cols / 32), (int64_t)1 << 27);
    if (pair->m + wlcs::w_class(w) > pair->xf_cap) return WLCS_EINVAL;  // cannot happen for a valid pair
    // probe list, its counter and the fallback flag, for this call
    const size_t list_bytes = (size_t)probe_cap * sizeof(wlcs::DotRec);
    const size_t cnt_off = (list_bytes + 255) / 256 * 256;
    uint8_t* scr = nullptr;
    if ((e = hipMallocAsync((void**)&scr, cnt_off + 256, stream)) != hipSuccess) return fail(ctx, e);
    wlcs::DotRec* probe = (wlcs::DotRec*)scr;
    unsigned long long* probe_count = (unsigned long long*)(scr + cnt_off);
    uint32_t* fallback = (uint32_t*)(scr + cnt_off + 64);
    e = wlcs::launch_zero_u64(probe_count, stream);
    if (e == hipSuccess) e = wlcs::launch_zero_u64((unsigned long long*)fallback, stream);
    const int32_t tp = std::max(0, threshold - (int32_t)(h / 2));
    // the probe strips, listed at the lowered threshold; each launch's tiles
    // and the y codes it reads as for a strided plot of the pair
    auto probe_launch = [&](int64_t prow, int64_t x0, int64_t stride) -> hipError_t {
        wlcs::PlotArgs a = make_args(prow, cols, w, nullptr, 0, nullptr, 0, tp, nullptr, 0);
        a.xstride = stride;
        a.x0 = x0;
        a.dots = probe;
        a.dot_cap = probe_cap;
        a.dot_count = probe_count;
        choose_tiles(ctx, a, prow, cols, w);
        int64_t xf_len, yg_len;
        needed_lengths(Path::Seaweed, 1, cols, w, a, xf_len, yg_len);
        if (yg_len > pair->yg_cap) return hipErrorInvalidValue;
        a.xf = pair->xf + x0;
        a.yg = pair->yg;
        a.sigma = pair->sigma;
        return wlcs::launch_seaweed(a, stream);
    };
    if (e == hipSuccess) e = probe_launch(probe_rows, first, h);
    if (e == hipSuccess) {
        wlcs::FilterArgs f;
        f.xf = pair->xf;
        f.yg = pair->yg;
        f.probe = probe;
        f.probe_cap = probe_cap;
        f.probe_count = probe_count;
        f.rows = rows;
        f.first = first;
        f.w = w;
        f.sigma = pair->sigma;
        f.h = (int32_t)h;
        f.threshold = threshold;
        f.dots = (wlcs::DotRec*)dots;
        f.dot_cap = dots ? dot_cap : 0;
        f.dot_count = (unsigned long long*)dot_count;
        f.fallback = fallback;
        f.cus = ctx->cus;
        e = wlcs::launch_candidates(f, stream);
    }
    if (e == hipSuccess) {
        // every strip, listed at the threshold, if (and only if) the probe
        // list overflowed; otherwise every workgroup returns at once
        wlcs::PlotArgs a = make_args(rows, cols, w, nullptr, 0, nullptr, 0, threshold, nullptr, 0);
        a.dots = (wlcs::DotRec*)dots;
        a.dot_cap = dots ? dot_cap : 0;
        a.dot_count = (unsigned long long*)dot_count;
        a.gate = fallback;
        choose_tiles(ctx, a, rows, cols, w);
        int64_t xf_len, yg_len;
        needed_lengths(Path::Seaweed, 1, cols, w, a, xf_len, yg_len);
        if (yg_len > pair->yg_cap) e = hipErrorInvalidValue;
        a.xf = pair->xf;
        a.yg = pair->yg;
        a.sigma = pair->sigma;
        if (e == hipSuccess) e = wlcs::launch_seaweed(a, stream);
    }
    (void)hipFreeAsync(scr, stream);
    if (e == hipSuccess) e = note_use(pair, stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

int wlcs_pair_plot_blcs(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, uint8_t* wlcs, int64_t ld,
                        uint64_t* bitmap, int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel,
                        uint32_t flags, void* stream) {
    return pair_plot_common(Path::Blcs, ctx, pair, w, wlcs, ld, bitmap, ld_words, threshold, indel, ld_indel,
                            flags, stream);
}

int wlcs_pair_plot_dp(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, uint8_t* wlcs, int64_t ld,
                      uint64_t* bitmap, int64_t ld_words, int32_t threshold, uint16_t* indel, int64_t ld_indel,
                      uint32_t flags, void* stream) {
    return pair_plot_common(Path::Dp, ctx, pair, w, wlcs, ld, bitmap, ld_words, threshold, indel, ld_indel,
                            flags, stream);
}

int wlcs_batch(wlcs_ctx* ctx, const wlcs_job* jobs, int32_t njobs, void* stream_) {
    BatchPlan plan;
    int st = plan_batch(ctx, jobs, njobs, plan);
    if (st != WLCS_OK) return st;
    if (plan.table.empty() && plan.singles.empty() && plan.counts.empty()) return WLCS_OK;
    if (plan.counts.size() > 0x7FFFFFFF) return WLCS_ERANGE;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    hipStream_t stream = (hipStream_t)stream_;
    const size_t tbytes = plan.table.size() * sizeof(wlcs::JobDesc);
    const size_t cnt_off = (tbytes + 255) / 256 * 256;
    const size_t ptr_off = cnt_off + 256, pbytes = plan.counts.size() * sizeof(unsigned long long*);
    // job table, the 8-byte work counter at cnt_off, the dot counters' addresses at ptr_off
    std::vector<uint8_t> host(ptr_off + pbytes, 0);
    if (tbytes) memcpy(host.data(), plan.table.data(), tbytes);
    if (pbytes) memcpy(host.data() + ptr_off, plan.counts.data(), pbytes);
    uint8_t* dev = nullptr;
    hipError_t e = hipMallocAsync((void**)&dev, host.size(), stream);
    if (e != hipSuccess) return fail(ctx, e);
    st = stage_copy(ctx, host.data(), host.size(), dev, stream);
    if (st != WLCS_OK) {
        (void)hipFreeAsync(dev, stream);
        return st;
    }
    e = enqueue_batch(ctx, plan, (const wlcs::JobDesc*)dev, (unsigned long long*)(dev + cnt_off),
                      (unsigned long long* const*)(dev + ptr_off), stream);
    if (dev) (void)hipFreeAsync(dev, stream);
    for (int32_t k = 0; e == hipSuccess && k < njobs; ++k) e = note_use(jobs[k].pair, stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

static_assert(wlcs::kNoAllocScratchBytes == WLCS_NOALLOC_SCRATCH_BYTES, "scratch size of the C ABI");
static_assert(sizeof(wlcs::JobDesc) == 184, "table entry size stated in the C ABI");

int wlcs_batch_noalloc(wlcs_ctx* ctx, const wlcs_job* jobs, int32_t njobs, void* stream_) {
    // the plan's vectors are kept per thread: once they have held a batch
    // this large, planning takes no host memory either
    thread_local BatchPlan plan;
    plan.clear();
    int st = plan_batch(ctx, jobs, njobs, plan);
    if (st != WLCS_OK) return st;
    if (plan.table.empty() && plan.singles.empty() && plan.counts.empty()) return WLCS_OK;
    // the scratch holds the job table, the groups' work counters (zeroed by a
    // kernel before each group's launch) and the dot counters' addresses
    const size_t tbytes = plan.table.size() * sizeof(wlcs::JobDesc);
    const size_t cnt_off = (tbytes + 255) / 256 * 256;
    const size_t ptr_off = cnt_off + 256, pbytes = plan.counts.size() * sizeof(unsigned long long*);
    if (plan.table.size() > wlcs::kNoAllocScratchBytes || plan.counts.size() > wlcs::kNoAllocScratchBytes ||
        ptr_off + pbytes > wlcs::kNoAllocScratchBytes)
        return WLCS_ESCRATCH;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    if (!ctx->scratch) return fail(ctx, (hipError_t)ctx->scratch_err);
    hipStream_t stream = (hipStream_t)stream_;
    uint8_t* const scr = ctx->scratch;
    hipError_t e = wlcs::launch_upload(scr, (const uint8_t*)plan.table.data(), tbytes, stream);
    if (e == hipSuccess && pbytes) e = wlcs::launch_upload(scr + ptr_off, (const uint8_t*)plan.counts.data(), pbytes, stream);
    if (e == hipSuccess)
        e = enqueue_batch(ctx, plan, (const wlcs::JobDesc*)scr, (unsigned long long*)(scr + cnt_off),
                          (unsigned long long* const*)(scr + ptr_off), stream);
    if (e != hipSuccess) return fail(ctx, e);
    return WLCS_OK;
}

int wlcs_batch_graph(wlcs_ctx* ctx, const wlcs_job* jobs, int32_t njobs, wlcs_graph** out) {
    if (!out) return WLCS_EINVAL;
    *out = nullptr;
    BatchPlan plan;
    int st = plan_batch(ctx, jobs, njobs, plan);
    if (st != WLCS_OK) return st;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return fail(ctx, hipErrorInvalidDevice);
    wlcs_graph* g = new (std::nothrow) wlcs_graph();
    if (!g) return WLCS_ENOMEM;
    g->device = ctx->device;
    const size_t tbytes = plan.table.size() * sizeof(wlcs::JobDesc);
    hipStream_t cap = nullptr;
    const size_t pbytes = plan.counts.size() * sizeof(unsigned long long*);
    hipError_t e = plan.counts.size() > 0x7FFFFFFF ? hipErrorInvalidValue : hipSuccess;
    if (e == hipSuccess) e = hipMalloc((void**)&g->table, std::max<size_t>(tbytes, 64));
    if (e == hipSuccess) e = hipMalloc((void**)&g->counter, 256);
    if (e == hipSuccess) e = hipMalloc((void**)&g->counts, std::max<size_t>(pbytes, 64));
    if (e == hipSuccess && tbytes) e = hipMemcpy(g->table, plan.table.data(), tbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess && pbytes) e = hipMemcpy(g->counts, plan.counts.data(), pbytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t el = enqueue_batch(ctx, plan, g->table, g->counter, g->counts, cap);
        e = hipStreamEndCapture(cap, &g->graph);
        if (el != hipSuccess) e = el;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (cap) (void)hipStreamDestroy(cap);
    if (e == hipSuccess) {
        for (int32_t k = 0; k < njobs; ++k)
            if (std::find(g->pairs.begin(), g->pairs.end(), jobs[k].pair) == g->pairs.end())
                g->pairs.push_back(jobs[k].pair);
    }
    if (e != hipSuccess) {
        wlcs_graph_destroy(g);
        return fail(ctx, e);
    }
    *out = g;
    return WLCS_OK;
}

int wlcs_graph_launch(wlcs_graph* graph, void* stream) {
    if (!graph || !graph->exec) return WLCS_EINVAL;
    DeviceGuard guard(graph->device);
    if (!guard.ok) return WLCS_EHIP;
    if (hipGraphLaunch(graph->exec, (hipStream_t)stream) != hipSuccess) return WLCS_EHIP;
    for (const wlcs_pair* p : graph->pairs)
        if (note_use(p, (hipStream_t)stream) != hipSuccess) return WLCS_EHIP;
    return WLCS_OK;
}

int wlcs_graph_destroy(wlcs_graph* graph) {
    if (!graph) return WLCS_OK;
    DeviceGuard guard(graph->device);
    int st = WLCS_OK;
    if (graph->exec && hipGraphExecDestroy(graph->exec) != hipSuccess) st = WLCS_EHIP;
    if (graph->graph && hipGraphDestroy(graph->graph) != hipSuccess) st = WLCS_EHIP;
    if (graph->table && hipFree(graph->table) != hipSuccess) st = WLCS_EHIP;
    if (graph->counter && hipFree(graph->counter) != hipSuccess) st = WLCS_EHIP;
    if (graph->counts && hipFree(graph->counts) != hipSuccess) st = WLCS_EHIP;
    delete graph;
    return st;
}

int wlcs_ctx_set_batch_tile(wlcs_ctx* ctx, int32_t w_lo, int32_t w_hi, int32_t tile_windows) {
    if (!ctx || w_lo < 1 || w_hi < w_lo || w_hi > WLCS_MAX_W) return WLCS_EINVAL;
    if (tile_windows == 0) {
        int k = 0;
        for (int r = 0; r < ctx->nbatch_rules; ++r)
            if (!(ctx->batch_rules[r].lo >= w_lo && ctx->batch_rules[r].hi <= w_hi))
                ctx->batch_rules[k++] = ctx->batch_rules[r];
        ctx->nbatch_rules = k;
        return WLCS_OK;
    }
    if (tile_windows < 64 || tile_windows > kMaxTile || tile_windows % 64) return WLCS_EINVAL;
    return add_rule(ctx->batch_rules, ctx->nbatch_rules, TileRule{w_lo, w_hi, tile_windows});
}

int wlcs_ctx_set_batch_grid(wlcs_ctx* ctx, int32_t waves_per_cu) {
    if (!ctx || waves_per_cu < 0 || waves_per_cu > 16) return WLCS_EINVAL;
    ctx->batch_waves_per_cu = waves_per_cu;
    return WLCS_OK;
}

int wlcs_ctx_set_batch_min_units(wlcs_ctx* ctx, int64_t min_units) {
    if (!ctx || min_units < 0 || min_units > (1 << 20)) return WLCS_EINVAL;
    ctx->batch_min_units = min_units;
    return WLCS_OK;
}

}  // extern "C"
