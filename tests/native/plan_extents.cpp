// CPU check of the batch planner and the kernels' unit decode (no GPU).
//
// Builds the library's host runtime (api.cpp) into this program and runs its
// planners -- plan_batch for wlcs_batch, and the tiling and length checks of
// the pair plots -- on random job mixes with fake device addresses.  For every
// unit a launch would run, it follows the kernels' decode on the host
// (batch: ticket -> find_job -> entry-local unit -> strip block and tile pair;
// single plots: blockIdx -> strip block and tile pair; then pair_tile and the
// per-unit extents of comb_unit) and checks, against the sizes the caller and
// the pair own:
//   * every x and y code a unit reads lies inside the pair's code arrays;
//   * every output written lies inside its buffer (rows < rows, column < ld,
//     bitmap word < ld_words, strided column < output columns);
//   * every plot entry and every bitmap word of every strip block is written
//     by exactly one unit (no block left unwritten, no two units racing);
//   * every entry-local unit maps to a tile pair of its job.
// A failure prints the job and unit and exits 1.
//
// Usage: plan_extents SEED ROUNDS
#include "../../paper_0909_2000_amd/csrc/api.cpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <tuple>

// The launch entry points are never reached here (nothing is enqueued).
namespace wlcs {
hipError_t launch_encode(const uint8_t*, int64_t, const uint8_t*, int, uint16_t*, int64_t, hipStream_t, int) {
    return hipErrorNotSupported;
}
hipError_t launch_seaweed(const PlotArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_zero_u64(unsigned long long*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_dp(const PlotArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_blcs(const PlotArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_epilogue(const PlotArgs&, const uint8_t*, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_batch(int, const JobDesc*, int32_t, int64_t, unsigned long long*, int32_t, bool, hipStream_t) {
    return hipErrorNotSupported;
}
hipError_t launch_zero_each(unsigned long long* const*, int32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_valu_peak(uint32_t*, int32_t, int32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_valu_issue(uint32_t*, int32_t, int32_t, int32_t, int32_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_candidates(const FilterArgs&, hipStream_t) { return hipErrorNotSupported; }
hipError_t scratch_address(int, uint8_t**) { return hipErrorNotSupported; }
hipError_t launch_upload(uint8_t*, const uint8_t*, size_t, hipStream_t) { return hipErrorNotSupported; }
}  // namespace wlcs

namespace {

[[noreturn]] void die(const char* what, int job, int64_t unit, long long a, long long b) {
    std::fprintf(stderr, "FAIL %s: job %d unit %lld (%lld vs %lld)\n", what, job, (long long)unit, a, b);
    std::exit(1);
}

// Fake device memory: every buffer its own range of addresses, far apart.
uint64_t g_next = 1ull << 40;
template <typename T>
T* fake(int64_t elems) {
    const uint64_t a = g_next;
    g_next += ((uint64_t)(elems > 0 ? elems : 1) * sizeof(T) + (1ull << 24)) & ~0xFFFFull;
    return (T*)a;
}

// One job as the caller sees it, with the sizes of everything it owns.
struct Spec {
    wlcs_pair pair;
    int32_t w = 0, hx = 1, hy = 1;
    bool full = false;
    int64_t rows = 0, cols = 0;    // windows compared (strided: output rows and columns)
    int64_t cols_all = 0;          // y-windows combed
    uint8_t* out = nullptr;
    int64_t ld = 0;
    uint64_t* bitmap = nullptr;
    int64_t ld_words = 0;
    uint16_t* indel = nullptr;
    int64_t ld_indel = 0;
    wlcs_dot* dots = nullptr;
    int64_t dot_cap = 0;
    uint64_t* dot_count = nullptr;
    int32_t threshold = 0;
    // written: per (strip block, output column) and per (strip block, bitmap u32 word)
    std::vector<uint8_t> cov, cov_bm;
};

Spec make_spec(std::mt19937_64& rng, bool big) {
    auto uni = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };
    Spec s;
    static const int32_t ws[] = {1, 2, 5, 15, 16, 17, 31, 32, 33, 40, 63, 64, 65, 100, 127, 128, 129, 200, 255};
    s.w = ws[uni(0, sizeof ws / sizeof ws[0] - 1)];
    const int64_t lmax = big ? 20000 : 3000;
    s.pair.m = uni(0, lmax);
    s.pair.n = uni(0, lmax);
    if (uni(0, 9) == 0) s.pair.m = s.w + uni(0, 2);  // a window or two
    s.pair.sigma = 4;
    pair_caps(s.pair.m, s.pair.n, s.pair.xf_cap, s.pair.yg_cap);
    s.pair.xf = fake<uint16_t>(s.pair.xf_cap);
    s.pair.yg = fake<uint16_t>(s.pair.yg_cap);
    s.full = uni(0, 3) == 0;
    const int kind = (int)uni(0, 5);  // 0-2 dense, 3 strided, 4 dot list, 5 strided dot list
    if (kind >= 3) {
        static const int32_t steps[] = {1, 2, 3, 5, 7};
        s.hx = steps[uni(0, 4)];
        s.hy = kind == 4 ? 1 : steps[uni(0, 4)];
    }
    const int64_t rows_all = n_windows(s.pair.m, s.w, s.full);
    s.cols_all = n_windows(s.pair.n, s.w, s.full);
    s.rows = (rows_all + s.hx - 1) / s.hx;
    s.cols = (s.cols_all + s.hy - 1) / s.hy;
    s.threshold = (int32_t)uni(0, s.w);
    const bool listing = kind >= 4;
    const bool plot = !listing || uni(0, 1);
    if (plot) {
        s.ld = s.cols + uni(0, 1) * uni(0, 70);
        s.out = fake<uint8_t>(std::max<int64_t>(s.rows * s.ld, 1));
    }
    if (s.hy == 1 && !listing && uni(0, 1)) {
        s.ld_words = (s.cols + 63) / 64 + uni(0, 1);
        s.bitmap = fake<uint64_t>(std::max<int64_t>(s.rows * s.ld_words, 1));
    }
    if (uni(0, 2) == 0 || (!plot && !listing)) {
        s.ld_indel = s.cols + uni(0, 3);
        s.indel = fake<uint16_t>(std::max<int64_t>(s.rows * s.ld_indel, 1));
    }
    if (listing) {
        s.dot_count = fake<uint64_t>(1);
        if (uni(0, 3)) {
            s.dot_cap = uni(0, 5000);
            s.dots = fake<wlcs_dot>(std::max<int64_t>(s.dot_cap, 1));
        }
    }
    return s;
}

bool in(const void* p, const void* base, int64_t bytes) {
    const uint64_t a = (uint64_t)p, b = (uint64_t)base;
    return a >= b && a < b + (uint64_t)bytes;
}

// The extents of unit (sb, pr) of a plot with geometry g, window w, class wc,
// read against the pair's code arrays and written against spec s; the output
// coverage is added to s.cov and s.cov_bm.  Follows comb_unit (WS = 1).
void check_unit(Spec& s, int job, int64_t unit, const wlcs::Geom& g, const uint16_t* xf, const uint32_t* yg32,
                int wc, bool exact, int64_t sb, int64_t pr, bool sp) {
    const int w = g.w;
    const int FL = wlcs::flush_windows(wc, 1);
    const int64_t nblocks = (g.rows + 63) / 64;
    if (sb < 0 || sb >= nblocks) die("strip block out of range", job, unit, sb, nblocks);
    if (pr < 0 || pr >= g.npairs) die("tile pair out of range", job, unit, pr, g.npairs);
    int64_t tA;
    const int64_t tlen = wlcs::pair_tile(g.cols, g.tile, g.tile2, g.nbig, pr, &tA);
    const int64_t tB = tA + tlen;
    if (tlen <= 0 || tlen % 64) die("tile length", job, unit, tlen, 64);
    const int64_t restA = g.cols - tA;
    if (restA <= 0) die("empty tile A", job, unit, tA, g.cols);
    const int64_t nA = (restA + 63) / 64 * 64;
    const int64_t nproc = nA < tlen ? nA : tlen;
    if (nproc % FL) die("windows per unit not whole flush blocks", job, unit, nproc, FL);
    const int64_t s0 = sb * 64;

    // x codes: the lane of the last strip of the block (past the last strip:
    // a copy of it) loads rows up to wc - 1 - pad of its window
    if (xf != s.pair.xf) die("x codes of another pair", job, unit, 0, 0);
    const int64_t sx = std::min<int64_t>(s0 + 63, g.rows - 1);
    // (the 256-row class: each wave of the chain loads the 64 rows from its
    // first one, in a strip padded to whole 8-row blocks)
    int last_row = wc - 1, pad = exact ? 0 : wlcs::pad_rows(w) - w;
    if (wc == 256) {
        pad = wlcs::wide_pad_rows(w) - w;
        last_row = 0;
        for (int q = 0; q < wlcs::kWideWaves; ++q) {
            int r0, nr;
            wlcs::wide_rows(w, q, &r0, &nr);
            last_row = std::max(last_row, r0 + wlcs::kWideRowsPerWave - 1);
        }
    }
    const int64_t xhi = sx * g.xstride + (last_row - pad);
    if (xhi >= s.pair.xf_cap) die("x read past the codes", job, unit, xhi, s.pair.xf_cap);
    // y codes: columns 0 .. nproc + w - 2 of each tile are combed, column
    // nproc + w - 1 is prefetched; each read is the u32 holding two columns
    if ((const uint16_t*)yg32 != s.pair.yg) die("y codes of another pair", job, unit, 0, 0);
    const int64_t lmax = nproc + w - 1;
    for (const int64_t t0 : {tA, tB}) {
        const int64_t yhi = 2 * ((t0 >> 1) + (lmax >> 1)) + 1;
        if (yhi >= s.pair.yg_cap) die("y read past the codes", job, unit, yhi, s.pair.yg_cap);
    }

    // stores, block by block, half by half
    const int64_t rows_here = std::min<int64_t>(64, g.rows - s0);
    const int64_t bm_words = ((g.ocols + 63) >> 6) * 2;
    for (int half = 0; half < 2; ++half) {
        const int64_t ts = half ? tB : tA;
        const int64_t te = std::min<int64_t>(ts + tlen, g.cols);
        for (int64_t jb = 0; jb < nproc; jb += FL) {
            const int64_t j0 = ts + jb;
            const int64_t nk = std::max<int64_t>(0, std::min<int64_t>(te - j0, FL));
            if (sp && nk > 0 && (g.hy > 1 || s.dot_count)) {
                const int64_t c_lo = (j0 + g.hy - 1) / g.hy;
                const int64_t nout = (j0 + nk + g.hy - 1) / g.hy - c_lo;
                if (nout > 64) die("strided outputs per block", job, unit, nout, 64);
                if (g.hy > 1) {
                    for (int64_t c = c_lo; c < c_lo + nout; ++c) {
                        if (c >= s.cols) die("strided column past the output", job, unit, c, s.cols);
                        if (s.out && c >= g.ld) die("strided column past ld", job, unit, c, g.ld);
                        if (s.indel && c >= g.ld_indel) die("strided indel past ld", job, unit, c, g.ld_indel);
                        ++s.cov[sb * s.cols + c];
                    }
                }
            }
            if (sp && g.hy > 1) continue;
            if (nk == 0 && (j0 >> 5) >= bm_words) continue;
            if (s.bitmap) {
                for (int sub = 0; sub < FL / 32; ++sub) {
                    const int64_t wi = (j0 >> 5) + sub;
                    if (wi < bm_words) {
                        if (wi >= g.ld_words32) die("bitmap word past ld_words", job, unit, wi, g.ld_words32);
                        ++s.cov_bm[sb * bm_words + wi];
                    }
                }
            }
            if (nk > 0) {
                if (j0 + nk > g.cols) die("plot columns past the plot", job, unit, j0 + nk, g.cols);
                if (s.out && j0 + nk > g.ld) die("plot columns past ld", job, unit, j0 + nk, g.ld);
                if (s.indel && j0 + nk > g.ld_indel) die("indel columns past ld", job, unit, j0 + nk, g.ld_indel);
                if (g.hy == 1)
                    for (int64_t j = j0; j < j0 + nk; ++j) ++s.cov[sb * s.cols + j];
            }
        }
    }
    if (rows_here <= 0) die("unit past the last strip", job, unit, s0, g.rows);
}

// Every output entry of every strip block written exactly once.
void check_coverage(const Spec& s, int job, bool dense_out) {
    const int64_t nblocks = (s.rows + 63) / 64;
    if (!dense_out) return;
    for (int64_t b = 0; b < nblocks; ++b)
        for (int64_t c = 0; c < s.cols; ++c)
            if (s.cov[b * s.cols + c] != 1) die("plot entry written !=1 times", job, b, c, s.cov[b * s.cols + c]);
    if (s.bitmap) {
        const int64_t bm_words = ((s.cols + 63) >> 6) * 2;
        for (int64_t b = 0; b < nblocks; ++b)
            for (int64_t wi = 0; wi < bm_words; ++wi)
                if (s.cov_bm[b * bm_words + wi] != 1)
                    die("bitmap word written !=1 times", job, b, wi, s.cov_bm[b * bm_words + wi]);
    }
}

void reset_coverage(Spec& s) {
    const int64_t nblocks = (s.rows + 63) / 64;
    s.cov.assign((size_t)std::max<int64_t>(nblocks * s.cols, 0), 0);
    s.cov_bm.assign((size_t)std::max<int64_t>(nblocks * ((s.cols + 63) >> 6) * 2, 0), 0);
}

// Units of a single-plot launch (launch_wc): unit = blockIdx, pair-major.
void check_single(Spec& s, int job, const wlcs::PlotArgs& a) {
    const wlcs::Geom g = wlcs::geom_of(a);
    const int wc = wlcs::w_class(a.w);
    const bool exact = a.w == wc && wc < 256;
    const bool sp = a.hy > 1 || a.dot_count;
    const int64_t nblocks = (a.rows + 63) / 64;
    const int64_t units = nblocks * a.npairs;
    if (units > 0x7FFFFFFFll) die("grid too large", job, units, units, 0x7FFFFFFFll);
    for (int64_t u = 0; u < units; ++u) {
        const int64_t pr = u / nblocks, sb = u - pr * nblocks;
        check_unit(s, job, u, g, a.xf, (const uint32_t*)a.yg, wc, exact, sb, pr, sp);
    }
}

// Fake context: the CU count of an MI355X and random tile rules.
void random_rules(std::mt19937_64& rng, wlcs_ctx& ctx) {
    auto uni = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };
    static const int32_t tiles[] = {64, 128, 256, 512, 576, 1024, 2048, 3456, 4096, 8192, 32768};
    ctx.nrules = 0;
    ctx.nbatch_rules = 0;
    const int nt = sizeof tiles / sizeof tiles[0];
    if (uni(0, 2) == 0) {
        const int32_t t = tiles[uni(0, nt - 1)], t2 = tiles[uni(0, nt - 1)];
        add_rule(ctx.rules, ctx.nrules, TileRule{1, 255, std::max(t, t2), std::min(t, t2), (int32_t)uni(0, 20)});
    }
    if (uni(0, 1) == 0) {
        for (int k = 0; k < 4; ++k) {
            const int32_t lo = k == 0 ? 1 : 16 << (k - 1), hi = 16 << k;
            if (uni(0, 1)) add_rule(ctx.batch_rules, ctx.nbatch_rules, TileRule{lo + (k > 0), hi, tiles[uni(0, 8)]});
        }
    }
    // batched jobs with too few units on shorter tiles (wlcs_ctx_set_batch_min_units)
    static const int64_t min_units[] = {0, 0, 1, 64, 1024, 4096, 1 << 20};
    ctx.batch_min_units = min_units[uni(0, 6)];
}

wlcs_job to_job(const Spec& s) {
    wlcs_job j;
    memset(&j, 0, sizeof j);
    j.pair = const_cast<wlcs_pair*>(&s.pair);
    j.w = s.w;
    j.flags = s.full ? WLCS_FULL_RANGE : 0;
    j.wlcs = s.out;
    j.ld = s.ld;
    j.bitmap = s.bitmap;
    j.ld_words = s.ld_words;
    j.threshold = s.threshold;
    j.indel = s.indel;
    j.ld_indel = s.ld_indel;
    j.hx = s.hx;
    j.hy = s.hy;
    j.dots = s.dots;
    j.dot_cap = s.dot_cap;
    j.dot_count = s.dot_count;
    return j;
}

void batch_round(std::mt19937_64& rng, wlcs_ctx& ctx, int njobs, bool big) {
    std::vector<Spec> specs;
    specs.reserve((size_t)njobs);
    for (int k = 0; k < njobs; ++k) specs.push_back(make_spec(rng, big && k % 8 == 0));
    std::vector<wlcs_job> jobs;
    for (auto& s : specs) {
        reset_coverage(s);
        jobs.push_back(to_job(s));
    }
    BatchPlan plan;
    const int st = plan_batch(&ctx, jobs.data(), (int32_t)jobs.size(), plan);
    if (st != WLCS_OK) die("plan_batch rejected valid jobs", st, 0, 0, 0);
    // which spec each table entry belongs to (by its outputs and codes)
    std::map<std::tuple<const void*, const void*, const void*, const void*, const void*>, int> owner;
    for (int k = 0; k < njobs; ++k)
        owner[{specs[k].pair.xf, specs[k].out, specs[k].bitmap, specs[k].indel, specs[k].dot_count}] = k;
    auto spec_of = [&](const wlcs::JobDesc& d) {
        auto it = owner.find({d.xf, d.out, d.bm32, d.indel, d.dot_count});
        if (it == owner.end()) die("table entry of no job", -1, 0, 0, 0);
        return it->second;
    };
    for (int grp = 0; grp < wlcs::kBatchGroups; ++grp) {
        const int32_t f0 = plan.first[grp], f1 = plan.first[grp + 1];
        const wlcs::JobDesc* jobs_g = plan.table.data() + f0;
        const int32_t n = f1 - f0;
        if (n == 0) {
            if (plan.units[grp] != 0) die("units without entries", -1, grp, plan.units[grp], 0);
            continue;
        }
        if (jobs_g[0].unit0 != 0) die("first entry not at unit 0", -1, grp, jobs_g[0].unit0, 0);
        for (int32_t e = 0; e < n; ++e) {
            if (wlcs::batch_group(jobs_g[e].variant) != grp) die("entry in the wrong group", -1, e, grp, 0);
            if (e > 0 && jobs_g[e].unit0 <= jobs_g[e - 1].unit0) die("unit0 not increasing", -1, e, 0, 0);
        }
        // the kernel's decode of every ticket below the group's unit count
        for (int64_t u = 0; u < plan.units[grp]; ++u) {
            int lo = 0, hi = n - 1;  // find_job
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs_g[mid].unit0 <= u) lo = mid;
                else hi = mid - 1;
            }
            const wlcs::JobDesc& jd = jobs_g[lo];
            const int64_t local = u - jd.unit0;
            const int64_t nblocks = (jd.g.rows + 63) / 64;
            const int64_t q = local / nblocks, sb = local - q * nblocks;
            const int64_t pr = jd.pr0 + q;
            const int k = spec_of(jd);
            const int wc = wlcs::w_class(jd.g.w);
            const bool exact = jd.variant == wlcs::kBatch16 || jd.variant == wlcs::kBatch32 ||
                               jd.variant == wlcs::kBatch64 || jd.variant == wlcs::kBatch128;
            if (exact != (jd.g.w == wc)) die("variant and window disagree", k, u, jd.variant, jd.g.w);
            if (jd.g.w != specs[k].w) die("window of another job", k, u, jd.g.w, specs[k].w);
            const bool sp = plan.sparse[grp];
            if ((jd.g.hy > 1 || jd.dot_count) && !sp) die("sparse job in a dense launch", k, u, 0, 0);
            check_unit(specs[k], k, u, jd.g, jd.xf, jd.yg32, wc, exact, sb, pr, sp);
        }
    }
    for (const wlcs::PlotArgs& a : plan.singles) {
        int k = -1;
        for (int q = 0; q < njobs; ++q)
            if (specs[q].pair.xf == a.xf && specs[q].out == a.wlcs && specs[q].dot_count == (uint64_t*)a.dot_count &&
                specs[q].indel == a.indel && specs[q].bitmap == (uint64_t*)a.bitmap32)
                k = q;
        if (k < 0) die("single plot of no job", -1, 0, 0, 0);
        if (a.w <= wlcs::kBatchMaxW) die("batchable window sent to a single plot", k, 0, a.w, 0);
        check_single(specs[k], k, a);
    }
    // counters: every job that lists dots, once
    size_t listing = 0;
    for (const auto& s : specs) listing += s.dot_count != nullptr;
    if (plan.counts.size() != listing) die("dot counters", -1, 0, (long long)plan.counts.size(), (long long)listing);
    for (int k = 0; k < njobs; ++k) {
        const Spec& s = specs[k];
        if (s.rows == 0 || s.cols == 0) continue;
        check_coverage(s, k, s.hy > 1 ? (s.out || s.indel) : true);
    }
}

// Single pair plots (pair_plot_common and strided_common on the seaweed
// path): the tiling, the code-length check, then every unit.
void single_round(std::mt19937_64& rng, wlcs_ctx& ctx) {
    Spec s = make_spec(rng, std::uniform_int_distribution<int>(0, 3)(rng) == 0);
    if (s.rows == 0 || s.cols == 0) return;
    reset_coverage(s);
    const bool strided = s.hx > 1 || s.hy > 1 || s.dot_count;
    wlcs::PlotArgs a = make_args(s.rows, strided ? s.cols_all : s.cols, s.w, s.out, s.ld, s.bitmap, s.ld_words,
                                 s.threshold, s.indel, s.ld_indel);
    a.xstride = s.hx;
    a.hy = s.hy;
    a.dots = (wlcs::DotRec*)s.dots;
    a.dot_cap = s.dots ? s.dot_cap : 0;
    a.dot_count = (unsigned long long*)s.dot_count;
    choose_tiles(&ctx, a, a.rows, a.cols, s.w);
    int64_t xf_len, yg_len;
    if (strided) {
        needed_lengths(Path::Seaweed, 1, a.cols, s.w, a, xf_len, yg_len);
        if (s.pair.m + wlcs::w_class(s.w) > s.pair.xf_cap || yg_len > s.pair.yg_cap)
            die("strided plot refused", 0, 0, yg_len, s.pair.yg_cap);
    } else {
        needed_lengths(Path::Seaweed, a.rows, a.cols, s.w, a, xf_len, yg_len);
        if (xf_len > s.pair.xf_cap || yg_len > s.pair.yg_cap) die("pair plot refused", 0, 0, yg_len, s.pair.yg_cap);
    }
    a.xf = s.pair.xf;
    a.yg = s.pair.yg;
    check_single(s, 0, a);
    check_coverage(s, 0, s.hy > 1 ? (s.out || s.indel) : true);
}

}  // namespace

int main(int argc, char** argv) {
    const uint64_t seed = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
    const int rounds = argc > 2 ? std::atoi(argv[2]) : 20;
    std::mt19937_64 rng(seed);
    // the 256-row class: the waves of a strip's chain hold consecutive runs of
    // whole 16-row blocks that cover the padded strip, at most 64 rows each
    // and at most the class's 256 rows of codes read, the last wave (which
    // also counts and stores) holding the fewest
    for (int w = 129; w <= 255; ++w) {
        const int np = wlcs::kWideWaves, wpad = wlcs::wide_pad_rows(w);
        if (wpad < w || wpad > 256 || wpad > 64 * np) die("wide chain length", 0, w, np, wpad);
        int next = 0, last_nr = 0, min_nr = 1 << 30;
        for (int q = 0; q < np; ++q) {
            int r0, nr;
            wlcs::wide_rows(w, q, &r0, &nr);
            if (r0 != next || nr < wlcs::kWideMinRows || nr > wlcs::kWideRowsPerWave || nr % wlcs::kWideRowBlock ||
                r0 + wlcs::kWideRowsPerWave - 1 > 255)
                die("wide rows", 0, w, r0, nr);
            next = r0 + nr;
            last_nr = nr;
            min_nr = std::min(min_nr, nr);
        }
        if (next != wpad || last_nr != min_nr) die("wide rows cover", 0, w, next, wpad);
    }
    // every window is combed in exactly its padded rows: each wave's row loop
    // (as comb_rows runs it, with the kernels' own stop tests) covers its
    // rows of the strip and no more, for every window length and class
    for (int w = 1; w <= 255; ++w) {
        const int wc = wlcs::w_class(w);
        if (wc < 256) {
            const bool exact = w == wc;
            const int wpad = exact ? wc : wlcs::pad_rows(w);
            // one wave holds the strip, or two halves (the 128-row class)
            const int nparts = wc == 128 ? 2 : 1, nr = wc / nparts;
            int combed = 0;
            for (int q = 0; q < nparts; ++q) {
                const int r0 = q * nr;
                for (int k = 0; k < nr; ++k) {
                    if (!exact && wlcs::stops_at_row(wc, r0 + k, wpad)) break;
                    if (r0 + k != combed) die("rows combed out of order", 0, w, r0 + k, combed);
                    ++combed;
                }
            }
            if (combed != wpad || wpad < w || wpad - w >= wlcs::kPadRowBlock) die("padded rows", 0, w, combed, wpad);
        } else {
            int next = 0;
            for (int q = 0; q < wlcs::kWideWaves; ++q) {
                int r0, nr;
                wlcs::wide_rows(w, q, &r0, &nr);
                int k = 0;
                while (k < wlcs::kWideRowsPerWave && !wlcs::wide_stops_at_row(k, nr)) ++k;
                if (r0 != next || k != nr) die("wide wave rows combed", 0, w, k, nr);
                next += k;
            }
            if (next != wlcs::wide_pad_rows(w)) die("wide padded rows", 0, w, next, wlcs::wide_pad_rows(w));
        }
    }
    wlcs_ctx* ctx = new wlcs_ctx();
    ctx->cus = 256;
    long long units = 0;
    for (int r = 0; r < rounds; ++r) {
        random_rules(rng, *ctx);
        batch_round(rng, *ctx, 1 + (int)(rng() % 48), r % 4 == 0);
        for (int k = 0; k < 8; ++k) single_round(rng, *ctx);
        ++units;
    }
    // the sizes of the benchmark's plots and batch, with the built-in tilings
    ctx->nrules = ctx->nbatch_rules = 0;
    ctx->batch_min_units = 0;
    for (const auto& shp : {std::make_tuple(50000, 50000, 64), std::make_tuple(30000, 30000, 128),
                            std::make_tuple(1000, 1000, 16), std::make_tuple(20000, 20000, 255)}) {
        Spec s;
        s.w = std::get<2>(shp);
        s.pair.m = std::get<0>(shp);
        s.pair.n = std::get<1>(shp);
        pair_caps(s.pair.m, s.pair.n, s.pair.xf_cap, s.pair.yg_cap);
        s.pair.xf = fake<uint16_t>(s.pair.xf_cap);
        s.pair.yg = fake<uint16_t>(s.pair.yg_cap);
        s.rows = s.pair.m - s.w;
        s.cols = s.cols_all = s.pair.n - s.w;
        s.ld = (s.cols + 63) / 64 * 64;
        s.out = fake<uint8_t>(s.rows * s.ld);
        s.ld_words = (s.cols + 63) / 64;
        s.bitmap = fake<uint64_t>(s.rows * s.ld_words);
        s.threshold = 48;
        reset_coverage(s);
        wlcs::PlotArgs a = make_args(s.rows, s.cols, s.w, s.out, s.ld, s.bitmap, s.ld_words, 48, nullptr, 0);
        choose_tiles(ctx, a, a.rows, a.cols, s.w);
        a.xf = s.pair.xf;
        a.yg = s.pair.yg;
        check_single(s, 0, a);
        check_coverage(s, 0, true);
    }
    delete ctx;
    std::printf("ok: seed %llu, %d rounds\n", (unsigned long long)seed, rounds);
    return 0;
}
