// Internal state of a library context (include/wlcs.h), shared by the host
// runtime (api.cpp) and the tuner (tune.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlcs_rt {

// Staging slots per context (pinned and device buffers), made as needed: a
// slot whose last work is still queued (behind other work on a busy stream) is
// not waited for while fewer than this many exist.  A serving loop keeps about
// one per job in flight (three batches of up to 64 jobs).
constexpr int kMaxSlots = 256;

// A pinned host buffer and (for strings to encode) a device buffer of the
// same capacity; `done` marks the end of the last work that read them.
struct Slot {
    uint8_t* buf = nullptr;
    size_t cap = 0;
    uint8_t* dbuf = nullptr;
    size_t dcap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};

// y-windows per tile for windows w in [lo, hi]: the first nbig tile pairs of
// every strip block have tiles of `tile` windows, the later ones of tile2
// (tile2 == tile: one length)
struct TileRule {
    int32_t lo, hi, tile, tile2 = 0, nbig = 0;
};

// A tiling chosen for one plot shape (rows, cols, window, stored-window step)
struct TileChoice {
    int64_t rows = -1, cols = -1;
    int32_t w = 0, ws = 0;
    int32_t tile = 0, tile2 = 0, nbig = 0, npairs = 0;
};
constexpr int kTileCache = 16;
// Tilings measured fastest for one plot shape each (wlcs_tune_plot, or
// loaded from a tuning cache by wlcs_tune / wlcs_tune_plot)
constexpr int kTuned = 32;

}  // namespace wlcs_rt

// Resident letter codes of one pair (wlcs_pair_create).
struct wlcs_pair {
    int device = 0;
    hipStream_t stream = nullptr;  // creation stream: the codes are allocated and freed in its order
    int64_t m = 0, n = 0;
    int32_t sigma = 0;  // letters of the pair's alphabet
    uint16_t* xf = nullptr;  // capacity xf_cap
    uint16_t* yg = nullptr;  // capacity yg_cap
    int64_t xf_cap = 0, yg_cap = 0;
    // Other streams that have read the codes: an event recorded after the
    // last work enqueued there that reads them.  wlcs_pair_destroy makes the
    // creation stream wait for each before the stream-ordered free, so a
    // pair dropped while a plot on another stream is still queued is not
    // released under it.  With more streams than entries, the oldest entry is
    // retired by making the creation stream wait for its event at once.
    static constexpr int kUses = 8;
    mutable hipStream_t use_stream[kUses] = {};
    mutable hipEvent_t use_event[kUses] = {};
    mutable int nuses = 0, next_use = 0;
};

struct wlcs_ctx {
    int device = 0;
    int cus = 256;
    int last_hip = 0;
    wlcs_rt::Slot slots[wlcs_rt::kMaxSlots];
    int nslots = 0;  // slots made so far (each with its event)
    int next_slot = 0;
    wlcs_rt::TileRule rules[16];
    int nrules = 0;
    wlcs_rt::TileRule batch_rules[16];
    int nbatch_rules = 0;
    int batch_waves_per_cu = 0;  // 0: each batched kernel's resident capacity
    int64_t batch_min_units = 0;  // > 0: a batched job's tiles shrink until it has this many units
    wlcs_rt::TileChoice tile_cache[wlcs_rt::kTileCache];  // recent built-in tilings
    int tile_cache_next = 0;
    wlcs_rt::TileChoice tuned[wlcs_rt::kTuned];  // measured tilings by shape (general plots, ws = 1)
    int ntuned = 0, tuned_next = 0;
    // the device's fixed scratch of wlcs_batch_noalloc (looked up at creation;
    // null with the HIP error kept if the lookup failed)
    uint8_t* scratch = nullptr;
    int scratch_err = 0;
};

namespace wlcs_rt {

// Record (or replace) the measured tiling of one shape; tile == 0 removes it
// (the built-in choice was the fastest).
inline void set_tuned(wlcs_ctx* ctx, const TileChoice& c) {
    for (int k = 0; k < ctx->ntuned; ++k) {
        TileChoice& e = ctx->tuned[k];
        if (e.rows == c.rows && e.cols == c.cols && e.w == c.w && e.ws == c.ws) {
            if (c.tile > 0) {
                e = c;
            } else {  // drop it: move the last entry here
                e = ctx->tuned[ctx->ntuned - 1];
                --ctx->ntuned;
                if (ctx->tuned_next > ctx->ntuned) ctx->tuned_next = 0;
            }
            return;
        }
    }
    if (c.tile <= 0) return;
    if (ctx->ntuned < kTuned) {
        ctx->tuned[ctx->ntuned++] = c;
    } else {  // full: replace the oldest
        ctx->tuned[ctx->tuned_next] = c;
        ctx->tuned_next = (ctx->tuned_next + 1) % kTuned;
    }
}

inline const TileChoice* find_tuned(const wlcs_ctx* ctx, int64_t rows, int64_t cols, int32_t w, int32_t ws) {
    for (int k = 0; k < ctx->ntuned; ++k) {
        const TileChoice& e = ctx->tuned[k];
        if (e.rows == rows && e.cols == cols && e.w == w && e.ws == ws) return &e;
    }
    return nullptr;
}

}  // namespace wlcs_rt
