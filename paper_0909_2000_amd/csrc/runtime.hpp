// Internal state of a library context (include/wlcs.h), shared by the host
// runtime (api.cpp) and the tuner (tune.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wlcs_rt {

constexpr int kSlots = 4;  // pinned staging buffers per context

struct Slot {
    uint8_t* buf = nullptr;
    size_t cap = 0;
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

}  // namespace wlcs_rt

struct wlcs_ctx {
    int device = 0;
    int cus = 256;
    int last_hip = 0;
    wlcs_rt::Slot slots[wlcs_rt::kSlots];
    int next_slot = 0;
    wlcs_rt::TileRule rules[16];
    int nrules = 0;
    wlcs_rt::TileRule batch_rules[16];
    int nbatch_rules = 0;
    int batch_waves_per_cu = 0;  // 0: each batched kernel's resident capacity
    wlcs_rt::TileChoice tile_cache[wlcs_rt::kTileCache];  // recent built-in tilings
    int tile_cache_next = 0;
};
