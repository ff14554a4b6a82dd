// Tuner of the batched launch (wlcs_tune in include/wlcs.h).
//
// Two knobs decide how the persistent batched kernels cut their work: the
// y-windows per tile of each window class (a wave combs 64 x-windows against
// two tiles, so longer tiles spend less of their columns on the w - 1 warm-up
// columns that every tile restart costs, while shorter tiles give more units
// and balance the queue better), and the waves per compute unit of the
// persistent grids.  The tuner times real batched launches on the
// context's device for every candidate, keeps the fastest, applies the result
// to the context and stores it in a JSON cache keyed by device, which later
// calls load instead of timing again:
//
//   { "gfx950-256cu": { "batch_tiles": {"1-16": 512, "17-32": 512, ...},
//                       "batch_grid": 16,
//                       "batch_ms": {"default": 81.9, "tuned": 81.0},
//                       "plots": {"49936x49936x64": [3456, 768, 5], ...},
//                       "plots_ms": {...} }, ... }
//
// The workload is a seeded synthetic batch of uniform random DNA pairs of
// uneven lengths in every window class; the run time of the method does not
// depend on the letters, only on m, n and w.
//
// The same cache holds measured tilings of single plots ("plots", keyed by
// rows x cols x window): wlcs_tune_plot times a grid of two-length tilings of
// one shape on the caller's pair and keeps the fastest; the context then uses
// it for every plot of that shape instead of the tile model's choice.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdlib>
#include <string>
#include <utility>
#include <vector>

#include "../../include/wlcs.h"
#include "runtime.hpp"

namespace {

// ---- a small JSON value: enough for the cache file ------------------------

struct JVal {
    enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
    bool b = false;
    double num = 0.0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;

    JVal* get(const std::string& key) {
        if (kind != Obj) return nullptr;
        for (auto& kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
    void set(const std::string& key, JVal v) {
        kind = Obj;
        for (auto& kv : obj)
            if (kv.first == key) {
                kv.second = std::move(v);
                return;
            }
        obj.emplace_back(key, std::move(v));
    }
    static JVal number(double x) {
        JVal v;
        v.kind = Num;
        v.num = x;
        return v;
    }
    static JVal array() {
        JVal v;
        v.kind = Arr;
        return v;
    }
    static JVal object() {
        JVal v;
        v.kind = Obj;
        return v;
    }
};

struct Parser {
    const char* p;
    const char* end;
    bool ok = true;

    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(const char* s) {
        const size_t k = strlen(s);
        if ((size_t)(end - p) >= k && memcmp(p, s, k) == 0) {
            p += k;
            return true;
        }
        return false;
    }
    std::string string() {
        std::string out;
        if (p >= end || *p != '"') {
            ok = false;
            return out;
        }
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                if (++p >= end) break;
                switch (*p) {
                    case 'n': out += '\n'; break;
                    case 't': out += '\t'; break;
                    case 'r': out += '\r'; break;
                    case 'b': out += '\b'; break;
                    case 'f': out += '\f'; break;
                    case 'u': {  // keep ASCII, replace the rest
                        if (end - p < 5) {
                            ok = false;
                            return out;
                        }
                        const unsigned v = (unsigned)strtoul(std::string(p + 1, p + 5).c_str(), nullptr, 16);
                        out += v < 128 ? (char)v : '?';
                        p += 4;
                        break;
                    }
                    default: out += *p;
                }
                ++p;
            } else {
                out += *p++;
            }
        }
        if (p >= end) {
            ok = false;
            return out;
        }
        ++p;
        return out;
    }
    JVal value(int depth = 0) {
        JVal v;
        ws();
        if (p >= end || depth > 32) {
            ok = false;
            return v;
        }
        if (*p == '{') {
            ++p;
            v.kind = JVal::Obj;
            ws();
            if (p < end && *p == '}') {
                ++p;
                return v;
            }
            while (ok) {
                ws();
                std::string k = string();
                ws();
                if (p >= end || *p != ':') {
                    ok = false;
                    break;
                }
                ++p;
                JVal item = value(depth + 1);
                v.obj.emplace_back(std::move(k), std::move(item));
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == '}') {
                    ++p;
                    break;
                }
                ok = false;
            }
        } else if (*p == '[') {
            ++p;
            v.kind = JVal::Arr;
            ws();
            if (p < end && *p == ']') {
                ++p;
                return v;
            }
            while (ok) {
                v.arr.push_back(value(depth + 1));
                ws();
                if (p < end && *p == ',') {
                    ++p;
                    continue;
                }
                if (p < end && *p == ']') {
                    ++p;
                    break;
                }
                ok = false;
            }
        } else if (*p == '"') {
            v.kind = JVal::Str;
            v.str = string();
        } else if (lit("true")) {
            v.kind = JVal::Bool;
            v.b = true;
        } else if (lit("false")) {
            v.kind = JVal::Bool;
        } else if (lit("null")) {
            v.kind = JVal::Null;
        } else {
            char* q = nullptr;
            const std::string rest(p, (size_t)std::min<ptrdiff_t>(end - p, 64));
            v.num = strtod(rest.c_str(), &q);
            if (q == rest.c_str()) {
                ok = false;
                return v;
            }
            v.kind = JVal::Num;
            p += q - rest.c_str();
        }
        return v;
    }
};

void quote(const std::string& s, std::string& out) {
    out += '"';
    for (char c : s) {
        if (c == '"' || c == '\\') out += '\\';
        if (c == '\n') {
            out += "\\n";
            continue;
        }
        out += c;
    }
    out += '"';
}

void dump(const JVal& v, std::string& out, int indent) {
    const std::string pad(indent, ' ');
    switch (v.kind) {
        case JVal::Null: out += "null"; break;
        case JVal::Bool: out += v.b ? "true" : "false"; break;
        case JVal::Num: {
            char buf[64];
            if (v.num > -1e15 && v.num < 1e15 && v.num == (double)(int64_t)v.num)
                snprintf(buf, sizeof buf, "%lld", (long long)v.num);
            else
                snprintf(buf, sizeof buf, "%.17g", v.num);
            out += buf;
            break;
        }
        case JVal::Str: quote(v.str, out); break;
        case JVal::Arr: {
            out += "[";
            for (size_t i = 0; i < v.arr.size(); ++i) {
                out += i ? ", " : "";
                dump(v.arr[i], out, indent + 1);
            }
            out += "]";
            break;
        }
        case JVal::Obj: {
            if (v.obj.empty()) {
                out += "{}";
                break;
            }
            out += "{\n";
            for (size_t i = 0; i < v.obj.size(); ++i) {
                out += pad + " ";
                quote(v.obj[i].first, out);
                out += ": ";
                dump(v.obj[i].second, out, indent + 1);
                out += i + 1 < v.obj.size() ? ",\n" : "\n";
            }
            out += pad + "}";
            break;
        }
    }
}

bool read_file(const char* path, std::string& out) {
    FILE* f = fopen(path, "rb");
    if (!f) return false;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) out.append(buf, k);
    fclose(f);
    return true;
}

bool write_file(const char* path, const std::string& text) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return false;
    }
    return rename(tmp.c_str(), path) == 0;
}

// ---- the tuning itself -----------------------------------------------------

// candidates; 0 stands for the built-in choice, where the search starts
constexpr int32_t kTiles[] = {0, 256, 512, 1024, 2048, 4096};
constexpr int32_t kGrids[] = {0, 4, 6, 8, 16};
constexpr int32_t kClasses[4][2] = {{1, 16}, {17, 32}, {33, 64}, {65, 128}};
constexpr int kPairs = 128;  // 32 per window class
constexpr int64_t kMinLen = 1000, kMaxLen = 16000;
constexpr int kReps = 5;     // timed launches per candidate (the median counts)

// "gfx950-256cu": architecture and compute units, so a cache holds one entry
// per kind of device
bool device_key(int device, std::string& key) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return false;
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    key = arch + "-" + std::to_string(prop.multiProcessorCount) + "cu";
    return true;
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct Workload {
    std::vector<wlcs_pair*> pairs;
    std::vector<uint8_t*> outs;
    std::vector<wlcs_job> jobs;
    ~Workload() {
        for (auto* p : pairs) wlcs_pair_destroy(p);
        for (auto* o : outs) (void)hipFree(o);
    }
};

int build_workload(wlcs_ctx* ctx, hipStream_t stream, Workload& wl) {
    static const uint8_t dna[4] = {'A', 'C', 'G', 'T'};
    uint64_t seed = 0x5EA3EEDull;
    std::vector<uint8_t> x, y;
    for (int k = 0; k < kPairs; ++k) {
        const int32_t w = kClasses[k % 4][1];
        const int64_t m = kMinLen + (int64_t)(splitmix64(seed) % (uint64_t)(kMaxLen - kMinLen + 1));
        const int64_t n = kMinLen + (int64_t)(splitmix64(seed) % (uint64_t)(kMaxLen - kMinLen + 1));
        x.resize((size_t)m);
        y.resize((size_t)n);
        for (auto& c : x) c = dna[splitmix64(seed) & 3];
        for (auto& c : y) c = dna[splitmix64(seed) & 3];
        wlcs_pair* pair = nullptr;
        int st = wlcs_pair_create(ctx, x.data(), m, y.data(), n, dna, 4, stream, &pair);
        if (st != WLCS_OK) return st;
        wl.pairs.push_back(pair);
        const int64_t rows = m - w, cols = n - w;
        uint8_t* out = nullptr;
        hipError_t e = hipMalloc((void**)&out, (size_t)(rows * cols));
        if (e != hipSuccess) {
            ctx->last_hip = (int)e;
            return e == hipErrorOutOfMemory ? WLCS_ENOMEM : WLCS_EHIP;
        }
        wl.outs.push_back(out);
        wlcs_job j;
        memset(&j, 0, sizeof j);
        j.pair = pair;
        j.w = w;
        j.wlcs = out;
        j.ld = cols;
        wl.jobs.push_back(j);
    }
    return WLCS_OK;
}

// median of kReps timed launches of the jobs, after one untimed one
int time_batch(wlcs_ctx* ctx, const std::vector<wlcs_job>& jobs, hipStream_t stream, hipEvent_t a,
               hipEvent_t b, double& ms) {
    float t[kReps];
    int st = wlcs_batch(ctx, jobs.data(), (int32_t)jobs.size(), stream);
    if (st != WLCS_OK) return st;
    for (float& v : t) {
        hipError_t e = hipEventRecord(a, stream);
        if (e == hipSuccess) st = wlcs_batch(ctx, jobs.data(), (int32_t)jobs.size(), stream);
        if (e == hipSuccess && st == WLCS_OK) e = hipEventRecord(b, stream);
        if (e == hipSuccess && st == WLCS_OK) e = hipEventSynchronize(b);
        if (e == hipSuccess && st == WLCS_OK) e = hipEventElapsedTime(&v, a, b);
        if (st != WLCS_OK) return st;
        if (e != hipSuccess) {
            ctx->last_hip = (int)e;
            return WLCS_EHIP;
        }
    }
    std::sort(t, t + kReps);
    ms = t[kReps / 2];
    return WLCS_OK;
}

int run_tuning(wlcs_ctx* ctx, JVal& entry) {
    hipStream_t stream = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipStreamCreate(&stream);
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    int st = e == hipSuccess ? WLCS_OK : WLCS_EHIP;
    if (e != hipSuccess) ctx->last_hip = (int)e;
    {
        Workload wl;
        if (st == WLCS_OK) st = build_workload(ctx, stream, wl);
        // start from the built-in choices
        for (const auto& c : kClasses)
            if (st == WLCS_OK) st = wlcs_ctx_set_batch_tile(ctx, c[0], c[1], 0);
        if (st == WLCS_OK) st = wlcs_ctx_set_batch_grid(ctx, 0);
        double default_ms = 0.0;
        if (st == WLCS_OK) st = time_batch(ctx, wl.jobs, stream, a, b, default_ms);
        // coordinate descent on the time of the whole batch (a class's tile
        // is judged by what it does to all of it, its group's queue tail
        // included): each class's tile in turn, then the grid; a candidate
        // is kept only if it beats the best so far, so the result is never
        // slower than the built-in choices on this batch
        double tuned_ms = default_ms;
        JVal tiles = JVal::object();
        for (const auto& c : kClasses) {
            int32_t best = 0;
            for (int32_t t : kTiles) {
                if (st != WLCS_OK || t == 0) continue;  // 0 is the starting point
                double ms = 0.0;
                st = wlcs_ctx_set_batch_tile(ctx, c[0], c[1], t);
                if (st == WLCS_OK) st = time_batch(ctx, wl.jobs, stream, a, b, ms);
                if (st == WLCS_OK && ms < tuned_ms) {
                    tuned_ms = ms;
                    best = t;
                }
            }
            if (st == WLCS_OK) st = wlcs_ctx_set_batch_tile(ctx, c[0], c[1], best);
            tiles.set(std::to_string(c[0]) + "-" + std::to_string(c[1]), JVal::number(best));
        }
        int32_t grid = 0;
        for (int32_t g : kGrids) {
            if (st != WLCS_OK || g == 0) continue;
            double ms = 0.0;
            st = wlcs_ctx_set_batch_grid(ctx, g);
            if (st == WLCS_OK) st = time_batch(ctx, wl.jobs, stream, a, b, ms);
            if (st == WLCS_OK && ms < tuned_ms) {
                tuned_ms = ms;
                grid = g;
            }
        }
        if (st == WLCS_OK) st = wlcs_ctx_set_batch_grid(ctx, grid);
        if (st == WLCS_OK) {
            e = hipStreamSynchronize(stream);
            if (e != hipSuccess) {
                ctx->last_hip = (int)e;
                st = WLCS_EHIP;
            }
        }
        if (st == WLCS_OK) {
            JVal ms = JVal::object();
            ms.set("default", JVal::number(default_ms));
            ms.set("tuned", JVal::number(tuned_ms));
            entry = JVal::object();
            entry.set("batch_grid", JVal::number(grid));
            entry.set("batch_ms", std::move(ms));
            entry.set("batch_tiles", std::move(tiles));
        }
        if (stream) (void)hipStreamSynchronize(stream);
    }  // the workload's pairs and outputs are released here, after the stream drained
    if (stream) (void)hipStreamSynchronize(stream);  // the pairs' stream-ordered frees
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (stream) (void)hipStreamDestroy(stream);
    return st;
}

// The measured tilings of single plots in an entry ("plots": {"RxCxW":
// [tile, tile2, nbig]}, tile 0 for the built-in choice); false if malformed.
bool parse_plots(JVal& entry, std::vector<wlcs_rt::TileChoice>& out) {
    JVal* plots = entry.get("plots");
    if (!plots) return true;
    if (plots->kind != JVal::Obj) return false;
    for (auto& kv : plots->obj) {
        long long r = 0, c = 0;
        int w = 0;
        char tail = 0;
        if (sscanf(kv.first.c_str(), "%lldx%lldx%d%c", &r, &c, &w, &tail) != 3 || r < 1 || c < 1 || w < 1 ||
            w > WLCS_MAX_W)
            return false;
        const JVal& v = kv.second;
        if (v.kind != JVal::Arr || v.arr.size() != 3) return false;
        double t[3];
        for (int k = 0; k < 3; ++k) {
            if (v.arr[k].kind != JVal::Num) return false;
            t[k] = v.arr[k].num;
            if (t[k] < 0 || t[k] > 32768 || t[k] != (int32_t)t[k]) return false;
        }
        const bool builtin = t[0] == 0;
        if (!builtin && ((int32_t)t[0] < 64 || (int32_t)t[0] % 64 || (int32_t)t[1] < 64 || (int32_t)t[1] % 64 ||
                         t[1] > t[0]))
            return false;
        wlcs_rt::TileChoice ch;
        ch.rows = r;
        ch.cols = c;
        ch.w = w;
        ch.ws = 1;
        ch.tile = (int32_t)t[0];
        ch.tile2 = (int32_t)t[1];
        ch.nbig = (int32_t)t[2];
        out.push_back(ch);
    }
    return true;
}

// Apply a cache entry; WLCS_EINVAL if it does not have the expected shape
// (nothing is applied then).  batch: the entry must hold the batch knobs.
int apply_entry(wlcs_ctx* ctx, JVal& entry, bool batch = true) {
    std::vector<wlcs_rt::TileChoice> plots;
    if (!parse_plots(entry, plots)) return WLCS_EINVAL;
    if (batch) {
        JVal* tiles = entry.get("batch_tiles");
        JVal* grid = entry.get("batch_grid");
        if (!tiles || tiles->kind != JVal::Obj || (grid && grid->kind != JVal::Num)) return WLCS_EINVAL;
        std::vector<wlcs_rt::TileRule> rules;
        for (auto& kv : tiles->obj) {
            int lo = 0, hi = 0;
            if (sscanf(kv.first.c_str(), "%d-%d", &lo, &hi) != 2 || kv.second.kind != JVal::Num) return WLCS_EINVAL;
            const double t = kv.second.num;
            // 0: the built-in choice
            if (lo < 1 || hi < lo || hi > WLCS_MAX_W || t < 0 || t > 32768 || (t > 0 && t < 64) ||
                t != (int32_t)t || (int32_t)t % 64)
                return WLCS_EINVAL;
            rules.push_back({lo, hi, (int32_t)t});
        }
        const double g = grid ? grid->num : 0.0;
        if (g < 0 || g > 16 || g != (int32_t)g) return WLCS_EINVAL;
        for (const auto& r : rules) {
            const int st = wlcs_ctx_set_batch_tile(ctx, r.lo, r.hi, r.tile);
            if (st != WLCS_OK) return st;
        }
        const int st = wlcs_ctx_set_batch_grid(ctx, (int32_t)g);
        if (st != WLCS_OK) return st;
    }
    for (const auto& p : plots) wlcs_rt::set_tuned(ctx, p);
    return WLCS_OK;
}

std::string plot_key(int64_t rows, int64_t cols, int32_t w) {
    return std::to_string(rows) + "x" + std::to_string(cols) + "x" + std::to_string(w);
}

// ---- tiling search for one plot shape ---------------------------------------

struct PlotTiming {
    wlcs_ctx* ctx;
    const wlcs_pair* pair;
    int32_t w, hx;
    uint32_t flags;
    uint8_t* out;
    int64_t ld;
    hipStream_t stream;
    hipEvent_t a, b;
    wlcs_rt::TileRule saved[16];
    int nsaved;

    // median of reps timed plots after one untimed one, under tiling
    // (tile, tile2, nbig) (tile 0: the built-in choice)
    int time(int32_t tile, int32_t tile2, int32_t nbig, int reps, double& ms) {
        for (int r = 0; r < nsaved; ++r) ctx->rules[r] = saved[r];
        ctx->nrules = nsaved;
        if (tile > 0) {  // a rule for exactly this window, looked at first
            const int slot = nsaved < 16 ? nsaved : 15;
            ctx->rules[slot] = wlcs_rt::TileRule{w, w, tile, tile2, nbig};
            ctx->nrules = slot + 1;
        }
        std::vector<float> t((size_t)reps);
        int st = WLCS_OK;
        for (int k = -1; k < reps && st == WLCS_OK; ++k) {
            hipError_t e = k >= 0 ? hipEventRecord(a, stream) : hipSuccess;
            if (e == hipSuccess)
                st = wlcs_pair_plot_strided(ctx, pair, w, hx, 1, out, ld, nullptr, 0, 0, nullptr, 0, nullptr, 0,
                                            nullptr, flags, stream);
            if (st != WLCS_OK) break;
            if (k < 0) continue;
            if (e == hipSuccess) e = hipEventRecord(b, stream);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t[(size_t)k], a, b);
            if (e != hipSuccess) {
                ctx->last_hip = (int)e;
                st = WLCS_EHIP;
            }
        }
        for (int r = 0; r < nsaved; ++r) ctx->rules[r] = saved[r];
        ctx->nrules = nsaved;
        if (st != WLCS_OK) return st;
        std::sort(t.begin(), t.end());
        ms = t[(size_t)reps / 2];
        return WLCS_OK;
    }
};

struct Tried {
    int32_t tile, tile2, nbig;
    double ms;
};

// Coarse grid of two-length tilings (and one-length ones), then the
// neighbourhood of the fastest, then the three fastest and the built-in
// choice timed again with more launches; the fastest of those wins.
int search_tiling(PlotTiming& pt, int64_t cols, int32_t& tile, int32_t& tile2, int32_t& nbig, double& tuned_ms,
                  double& builtin_ms) {
    const int64_t cap = std::max<int64_t>(64, (cols + 63) / 64 * 64);
    std::vector<Tried> tried;
    int st = WLCS_OK;
    auto norm = [&](int32_t t, int32_t t2, int64_t nb) -> Tried {
        const int64_t nbm = cols / (2 * (int64_t)t);
        if (t2 >= t || nbm < 1) return Tried{t, t, 0, 0.0};  // one length
        return Tried{t, t2, (int32_t)std::max<int64_t>(1, std::min<int64_t>(nb, nbm)), 0.0};
    };
    auto attempt = [&](Tried c) {
        if (st != WLCS_OK || c.tile < 64 || c.tile > cap || c.tile % 64 || c.tile2 < 64 || c.tile2 % 64) return;
        for (const Tried& d : tried)
            if (d.tile == c.tile && d.tile2 == c.tile2 && d.nbig == c.nbig) return;
        st = pt.time(c.tile, c.tile2, c.nbig, 3, c.ms);
        if (st == WLCS_OK) tried.push_back(c);
    };
    static const int32_t kLong[] = {256, 512, 1024, 1536, 2048, 3072, 4096, 6144};
    static const int32_t kShort[] = {128, 256, 512, 1024};
    for (int32_t t : kLong) {
        if (t > cap) break;
        attempt(norm(t, t, 0));
        const int64_t nbm = cols / (2 * (int64_t)t);
        for (int32_t t2 : kShort) {
            if (t2 >= t || nbm < 1) continue;
            const int64_t nbs[4] = {nbm / 4, nbm / 2, 3 * nbm / 4, nbm};
            for (int64_t nb : nbs) attempt(norm(t, t2, nb));
        }
    }
    if (st != WLCS_OK) return st;
    if (tried.empty()) {  // no candidate fits the row: the built-in choice stays
        tile = tile2 = nbig = 0;
        st = pt.time(0, 0, 0, 5, builtin_ms);
        tuned_ms = builtin_ms;
        return st;
    }
    auto fastest = [&]() {
        return *std::min_element(tried.begin(), tried.end(), [](const Tried& p, const Tried& q) { return p.ms < q.ms; });
    };
    const Tried b1 = fastest();
    auto r64 = [](double v) { return (int32_t)std::max<int64_t>(64, (int64_t)(v / 64.0 + 0.5) * 64); };
    const double tf[5] = {0.75, 0.875, 1.0, 1.125, 1.25}, sf[3] = {0.75, 1.0, 1.5};
    for (double f : tf) {
        const int32_t t = r64(b1.tile * f);
        if (b1.tile2 == b1.tile) {
            attempt(norm(t, t, 0));
            continue;
        }
        for (double g : sf)
            for (int d = -2; d <= 2; ++d) attempt(norm(t, r64(b1.tile2 * g), (int64_t)b1.nbig + d));
    }
    if (st != WLCS_OK) return st;
    // the three fastest and the built-in choice, timed again
    std::sort(tried.begin(), tried.end(), [](const Tried& p, const Tried& q) { return p.ms < q.ms; });
    if (tried.size() > 3) tried.resize(3);
    st = pt.time(0, 0, 0, 9, builtin_ms);
    Tried best{0, 0, 0, builtin_ms};
    for (Tried& c : tried) {
        if (st == WLCS_OK) st = pt.time(c.tile, c.tile2, c.nbig, 9, c.ms);
        if (st == WLCS_OK && c.ms < best.ms) best = c;
    }
    if (st != WLCS_OK) return st;
    tile = best.tile;
    tile2 = best.tile2;
    nbig = best.nbig;
    tuned_ms = best.ms;
    return WLCS_OK;
}

// Read the cache file into cache (an empty object if path is NULL or the
// file does not exist); WLCS_EINVAL if it is not a JSON object.
int read_cache(const char* path, JVal& cache) {
    cache = JVal::object();
    std::string text;
    if (!path || !read_file(path, text)) return WLCS_OK;
    Parser ps{text.data(), text.data() + text.size()};
    JVal parsed = ps.value();
    ps.ws();
    if (!ps.ok || ps.p != ps.end || parsed.kind != JVal::Obj) return WLCS_EINVAL;  // reported, not overwritten
    cache = std::move(parsed);
    return WLCS_OK;
}

int write_cache(const char* path, const JVal& cache) {
    std::string out;
    dump(cache, out, 0);
    out += "\n";
    return write_file(path, out) ? WLCS_OK : WLCS_EIO;
}

}  // namespace

extern "C" {

int wlcs_tune(wlcs_ctx* ctx, const char* cache_path, uint32_t flags) {
    if (!ctx || (flags & ~WLCS_TUNE_FORCE)) return WLCS_EINVAL;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return WLCS_EHIP;
    std::string key;
    int st = device_key(ctx->device, key) ? WLCS_OK : WLCS_EHIP;
    JVal cache;
    if (st == WLCS_OK) st = read_cache(cache_path, cache);
    JVal* have = st == WLCS_OK ? cache.get(key) : nullptr;
    if (have && have->kind != JVal::Obj) st = WLCS_EINVAL;
    // batch knobs without their tiles: a malformed entry (an entry with only
    // measured plot tilings is completed below)
    if (have && !have->get("batch_tiles") && (have->get("batch_grid") || have->get("batch_ms"))) st = WLCS_EINVAL;
    if (st == WLCS_OK && have && have->get("batch_tiles") && !(flags & WLCS_TUNE_FORCE)) {
        st = apply_entry(ctx, *have);
    } else if (st == WLCS_OK) {
        // an entry without the batch knobs (only measured plot tilings) is
        // completed; its plot tilings are kept and applied
        std::vector<wlcs_rt::TileChoice> plots;
        if (have && !parse_plots(*have, plots)) st = WLCS_EINVAL;
        JVal entry;
        if (st == WLCS_OK) st = run_tuning(ctx, entry);
        for (const char* m : {"plots", "plots_ms"})
            if (st == WLCS_OK && have && have->get(m)) entry.set(m, *have->get(m));
        if (st == WLCS_OK) st = apply_entry(ctx, entry);
        if (st == WLCS_OK && cache_path) {
            cache.set(key, std::move(entry));
            st = write_cache(cache_path, cache);
        }
    }
    if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
    return st;
}

int wlcs_tune_plot(wlcs_ctx* ctx, const wlcs_pair* pair, int32_t w, int32_t hx, uint32_t flags,
                   const char* cache_path, uint32_t tune_flags) {
    if (!ctx || !pair || pair->device != ctx->device || (flags & ~WLCS_FULL_RANGE) ||
        (tune_flags & ~WLCS_TUNE_FORCE))
        return WLCS_EINVAL;
    if (w < 1 || w > WLCS_MAX_W || hx < 1) return WLCS_ERANGE;
    const bool full = (flags & WLCS_FULL_RANGE) != 0;
    const int64_t rows_all = std::max<int64_t>(0, pair->m - w + (full ? 1 : 0));
    const int64_t cols = std::max<int64_t>(0, pair->n - w + (full ? 1 : 0));
    const int64_t rows = (rows_all + hx - 1) / hx;
    if (rows == 0 || cols == 0) return WLCS_OK;  // an empty plot: nothing to tune
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != ctx->device && hipSetDevice(ctx->device) != hipSuccess) return WLCS_EHIP;
    std::string dkey;
    int st = device_key(ctx->device, dkey) ? WLCS_OK : WLCS_EHIP;
    const std::string pkey = plot_key(rows, cols, w);
    JVal cache;
    if (st == WLCS_OK) st = read_cache(cache_path, cache);
    JVal* have = st == WLCS_OK ? cache.get(dkey) : nullptr;
    if (have && have->kind != JVal::Obj) st = WLCS_EINVAL;
    JVal* plots = have ? have->get("plots") : nullptr;
    if (plots && plots->kind != JVal::Obj) st = WLCS_EINVAL;
    JVal* known = (st == WLCS_OK && plots) ? plots->get(pkey) : nullptr;
    if (known && !(tune_flags & WLCS_TUNE_FORCE)) {
        // apply the recorded tiling of this shape only
        JVal one = JVal::object();
        JVal p = JVal::object();
        p.set(pkey, *known);
        one.set("plots", std::move(p));
        st = apply_entry(ctx, one, false);
    } else if (st == WLCS_OK) {
        // the pair's codes may still be in flight on its creation stream
        hipError_t e = hipDeviceSynchronize();
        PlotTiming pt{};
        pt.ctx = ctx;
        pt.pair = pair;
        pt.w = w;
        pt.hx = hx;
        pt.flags = flags;
        pt.ld = cols;
        pt.nsaved = ctx->nrules;
        for (int r = 0; r < ctx->nrules; ++r) pt.saved[r] = ctx->rules[r];
        // a measured tiling of this shape must not steer the built-in timing
        wlcs_rt::TileChoice drop;
        drop.rows = rows;
        drop.cols = cols;
        drop.w = w;
        drop.ws = 1;
        drop.tile = 0;
        wlcs_rt::set_tuned(ctx, drop);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&pt.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreate(&pt.a);
        if (e == hipSuccess) e = hipEventCreate(&pt.b);
        if (e == hipSuccess) e = hipMalloc((void**)&pt.out, (size_t)(rows * cols));
        if (e != hipSuccess) {
            ctx->last_hip = (int)e;
            st = e == hipErrorOutOfMemory ? WLCS_ENOMEM : WLCS_EHIP;
        }
        int32_t tile = 0, tile2 = 0, nbig = 0;
        double tuned_ms = 0.0, builtin_ms = 0.0;
        if (st == WLCS_OK) st = search_tiling(pt, cols, tile, tile2, nbig, tuned_ms, builtin_ms);
        if (pt.stream) (void)hipStreamSynchronize(pt.stream);
        if (pt.out) (void)hipFree(pt.out);
        if (pt.a) (void)hipEventDestroy(pt.a);
        if (pt.b) (void)hipEventDestroy(pt.b);
        if (pt.stream) (void)hipStreamDestroy(pt.stream);
        if (st == WLCS_OK) {
            wlcs_rt::TileChoice ch;
            ch.rows = rows;
            ch.cols = cols;
            ch.w = w;
            ch.ws = 1;
            ch.tile = tile;
            ch.tile2 = tile2;
            ch.nbig = nbig;
            wlcs_rt::set_tuned(ctx, ch);
        }
        if (st == WLCS_OK && cache_path) {
            JVal rec = JVal::array();
            rec.arr.push_back(JVal::number(tile));
            rec.arr.push_back(JVal::number(tile2));
            rec.arr.push_back(JVal::number(nbig));
            if (!have) {
                cache.set(dkey, JVal::object());
                have = cache.get(dkey);
            }
            if (!have->get("plots")) have->set("plots", JVal::object());
            have->get("plots")->set(pkey, std::move(rec));
            JVal ms = JVal::object();
            ms.set("builtin", JVal::number(builtin_ms));
            ms.set("tuned", JVal::number(tuned_ms));
            if (!have->get("plots_ms")) have->set("plots_ms", JVal::object());
            have->get("plots_ms")->set(pkey, std::move(ms));
            st = write_cache(cache_path, cache);
        }
    }
    if (prev >= 0 && prev != ctx->device) (void)hipSetDevice(prev);
    return st;
}

int wlcs_ctx_get_plot_tiling(const wlcs_ctx* ctx, int64_t rows, int64_t cols, int32_t w, int32_t* tile,
                             int32_t* tile2, int32_t* nbig) {
    if (!ctx || !tile || !tile2 || !nbig || rows < 0 || cols < 0 || w < 1 || w > WLCS_MAX_W) return WLCS_EINVAL;
    const wlcs_rt::TileChoice* c = wlcs_rt::find_tuned(ctx, rows, cols, w, 1);
    *tile = c ? c->tile : 0;
    *tile2 = c ? c->tile2 : 0;
    *nbig = c ? c->nbig : 0;
    return WLCS_OK;
}

int wlcs_ctx_get_batch_tile(const wlcs_ctx* ctx, int32_t w, int32_t* tile_windows) {
    if (!ctx || !tile_windows || w < 1 || w > WLCS_MAX_W) return WLCS_EINVAL;
    *tile_windows = 0;
    for (int r = ctx->nbatch_rules - 1; r >= 0; --r)
        if (w >= ctx->batch_rules[r].lo && w <= ctx->batch_rules[r].hi) {
            *tile_windows = ctx->batch_rules[r].tile;
            break;
        }
    return WLCS_OK;
}

int wlcs_ctx_get_batch_grid(const wlcs_ctx* ctx, int32_t* waves_per_cu) {
    if (!ctx || !waves_per_cu) return WLCS_EINVAL;
    *waves_per_cu = ctx->batch_waves_per_cu;
    return WLCS_OK;
}

}  // extern "C"
