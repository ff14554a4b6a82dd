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

// y-windows per tile for windows w in [lo, hi]
struct TileRule {
    int32_t lo, hi, tile;
};

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
    int batch_waves_per_cu = 0;  // 0: kBatchWavesPerCu
};
