/*
 * wlcs.h - C ABI of the MI355X (gfx950) alignment-plot library.
 *
 * An alignment plot (Krusche & Tiskin, "Computing alignment plots
 * efficiently", Section 2) of strings x (length m) and y (length n) for window
 * length w is the matrix WLCS(i, j), the length of a longest common
 * subsequence of the w-windows x_i..x_{i+w-1} and y_j..y_{j+w-1}, for
 * i in 1..m-w and j in 1..n-w.  This library computes it on the GPU in
 * O(m n w) work by the windowed seaweed algorithm (Theorem 3.1: one strip of
 * height w per x-window, combed column by column, with a sliding count of the
 * seaweeds that start and end inside each y-window), and also offers the
 * plain per-window dynamic program (O(m n w^2), the paper's baseline) on the
 * same device for comparison.
 *
 * Conventions shared by every entry point:
 *   - Output layout: row-major, 0-based.  Row i (0 <= i < rows) is the x-window
 *     starting at x[i], column j (0 <= j < cols) the y-window starting at y[j].
 *     rows = m - w and cols = n - w (the paper's ranges 1..m-w, 1..n-w); with
 *     WLCS_FULL_RANGE, rows = m - w + 1 and cols = n - w + 1 (every window).
 *     If rows <= 0 or cols <= 0 the plot is empty and the call succeeds
 *     without touching any output.
 *   - Letters are bytes.  alphabet lists sigma distinct bytes (1 <= sigma <=
 *     WLCS_MAX_SIGMA); two letters match iff they are the same byte.  A byte of
 *     x or y outside the alphabet is an error (no wildcard semantics).
 *   - Strings x and y are caller-owned HOST buffers; the call reads them before
 *     it returns.  Outputs are caller-owned DEVICE buffers on the context's
 *     device, written asynchronously on `stream` (a hipStream_t, or NULL for
 *     the default stream).  Results are valid once the stream reaches the point
 *     of the call; the library keeps no reference to caller memory after that.
 *   - Every function returns WLCS_OK (0) or a negative status.  Argument
 *     errors are reported before anything is enqueued; nothing throws across
 *     the ABI and the library never aborts the process.
 *   - A context belongs to one device and must not be used from two threads
 *     at once without external locking.
 */
#ifndef WLCS_H
#define WLCS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WLCS_OK 0
#define WLCS_EINVAL (-1)    /* null pointer where one is needed, ld too small, bad flags */
#define WLCS_ERANGE (-2)    /* w outside 1..WLCS_MAX_W, negative or oversized lengths */
#define WLCS_EALPHABET (-3) /* bad alphabet, or a string byte outside it */
#define WLCS_EHIP (-4)      /* HIP runtime or launch failure (wlcs_ctx_last_hip_error) */
#define WLCS_ENOMEM (-5)    /* host or device allocation failed */
#define WLCS_EIO (-6)       /* a file could not be written (wlcs_tune's cache) */
#define WLCS_ESCRATCH (-7)  /* a batch needs more than wlcs_batch_noalloc's fixed scratch */

#define WLCS_MAX_W 255         /* WLCS values must fit the uint8 output */
#define WLCS_MAX_SIGMA 63      /* letters per alphabet (a 64th code is kept for padding rows) */
#define WLCS_MAX_LEN 100000000 /* longest string accepted (bytes) */
#define WLCS_MAX_SCORE_W 127   /* alignment-score plots: scores in [-w, w] fit int8 */

/* flags */
#define WLCS_FULL_RANGE 1u /* every window: (m-w+1) x (n-w+1) instead of (m-w) x (n-w) */

typedef struct wlcs_ctx wlcs_ctx;

/* Create a context on HIP device `device` (ordinal).  *out receives the handle.
 * The context owns device scratch, staging slots and tuning.  A staging slot
 * is a pinned host buffer and a device buffer of the same size (1 MiB, or
 * the next power of two above a larger string pair); the context makes them
 * as calls need them, up to 256 (about one per pair in flight), and reuses a
 * slot once the work that read it is done. */
int wlcs_ctx_create(int device, wlcs_ctx **out);

/* Wait for the context's outstanding staging work and free everything it
 * owns.  NULL is accepted. */
int wlcs_ctx_destroy(wlcs_ctx *ctx);

/* Last HIP error code (hipError_t as int) seen by the context, 0 if none. */
int wlcs_ctx_last_hip_error(const wlcs_ctx *ctx);

/* Measurement helper, not part of the method: the sustained rate of packed
 * 16-bit VALU operations on the context's device, against which the seaweed
 * kernels' rates are reported.  A kernel of independent v_pk_max_u16 chains
 * (two 16-bit operations per lane and instruction, no instruction waiting for
 * the one before it) runs on every SIMD of every CU, once to warm up and once
 * timed with HIP events.  iters (1..10^6) sets the length of the timed run
 * (about 0.34 ms per 100 on an MI355X; runs under about 10 ms read low while
 * the clock ramps up).  Synchronous: it allocates, runs on a
 * stream of its own, waits and frees.  *ops_per_s receives 16-bit element
 * operations per second. */
int wlcs_measure_valu_peak(wlcs_ctx *ctx, int32_t iters, double *ops_per_s);

/* Measurement helper, not part of the method: wave64 VALU instructions issued
 * per second per SIMD (four per CU) with waves_per_simd (1..4) waves resident
 * on every SIMD, for one kind of instruction stream: 0 packed 16-bit
 * (v_pk_max_u16), 1 plain 32-bit (v_xor_b32) and 5 three-input bitwise
 * (v_bitop3_b32), each on eight independent accumulators; 2 the seaweed cell
 * down a column of eight rows (four instructions per cell, three packed and
 * one v_bitop3_b32, each cell waiting for the label of the cell above, as in
 * the plot kernels); 3 the same chain with the letter comparison done by
 * v_xor_b32 on codes repeated in both halves (two packed, two plain; not what
 * the kernels run); 4 the same chain with the right label formed by two
 * v_xor_b32 (five instructions per cell; the cell's earlier form).  One
 * workgroup of 256 x waves_per_simd threads per CU runs iters (1..10^6)
 * rounds of 16 (kinds 0, 1, 5), 32 (kinds 2, 3) or 40 (kind 4) instructions
 * per wave, once to warm up (at most
 * 1,000 rounds) and once timed with HIP events.  Synchronous, like
 * wlcs_measure_valu_peak.  WLCS_EINVAL for a null context or pointer or an
 * argument out of range (nothing runs). */
int wlcs_measure_valu_issue(wlcs_ctx *ctx, int32_t kind, int32_t waves_per_simd, int32_t iters,
                            double *instr_per_s);

/* Human-readable text for a status code (static storage). */
const char *wlcs_status_str(int status);

/* Seaweed tiling knobs (the tuner sets these; 0 restores the built-in choice).
 * tile_windows: y-windows each lane covers per tile; a multiple of 64 in
 * 64..32768.  Every x-window is combed afresh from the first column of each
 * tile, so a tile of T windows combs T + w - 1 columns (Theorem 3.1 applied to
 * the strip restricted to those columns).  Applies to windows w with
 * w_lo <= w <= w_hi. */
int wlcs_ctx_set_tile(wlcs_ctx *ctx, int32_t w_lo, int32_t w_hi, int32_t tile_windows);

/* Two tile lengths (the built-in choice uses two as well): in every block of
 * 64 x-windows the first long_pairs tile pairs (at most as many as fit in the
 * row) have tiles of long_tile windows, the later ones tiles of short_tile;
 * the last pair's remaining windows are split evenly between its two tiles.
 * Long tiles comb fewer columns before their first complete window, short
 * ones shorten the tail of a launch.  Both lengths as for wlcs_ctx_set_tile;
 * long_pairs >= 0; long_tile = 0 drops the rules covering [w_lo, w_hi].
 * Applies to single plots (wlcs_plot, wlcs_pair_plot, their strided forms,
 * wlcs_score_plot, and batch jobs with w > 128). */
int wlcs_ctx_set_tiles(wlcs_ctx *ctx, int32_t w_lo, int32_t w_hi, int32_t long_tile, int32_t short_tile,
                       int32_t long_pairs);

/* Alignment plot by the windowed seaweed algorithm (Theorem 3.1, with the
 * combing rule of Section 2 and the bit bounds of Propositions 3.3-3.4).
 *
 *   x, m, y, n, w     host strings and window length (1 <= w <= WLCS_MAX_W).
 *   alphabet, sigma   the letters (see conventions).
 *   wlcs, ld          uint8 output, rows x cols, row stride ld >= cols
 *                     (elements).  May be NULL if only the epilogues are wanted.
 *   bitmap, ld_words  thresholded dot plot (Section 1: a dot marks a window
 *                     pair whose similarity clears a threshold): bit j%64 of
 *                     word j/64 of row i is set iff WLCS(i, j) >= threshold;
 *                     ceil(cols/64) uint64 words per row, padding bits written
 *                     as 0, row stride ld_words >= ceil(cols/64).  NULL skips.
 *   indel, ld_indel   uint16 indel distance 2w - 2*WLCS(i, j) (LCS alignment
 *                     with gap score 0, Section 2), row stride ld_indel >= cols.
 *                     NULL skips.
 *   flags             0 or WLCS_FULL_RANGE.
 *   stream            hipStream_t the work is enqueued on.
 * At least one of wlcs, bitmap, indel must be non-NULL (unless the plot is
 * empty).  threshold is used only with a bitmap and must be in 0..255. */
int wlcs_plot(wlcs_ctx *ctx, const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
              int32_t w, const uint8_t *alphabet, int32_t sigma, uint8_t *wlcs, int64_t ld,
              uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint16_t *indel,
              int64_t ld_indel, uint32_t flags, void *stream);

/* The same plot by the plain per-window dynamic program of Section 2 (every
 * window pair solved independently, O(w^2) each): the paper's baseline, run
 * on the GPU for comparison.  Same arguments, outputs and errors. */
int wlcs_plot_dp(wlcs_ctx *ctx, const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
                 int32_t w, const uint8_t *alphabet, int32_t sigma, uint8_t *wlcs, int64_t ld,
                 uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint16_t *indel,
                 int64_t ld_indel, uint32_t flags, void *stream);

/* The same plot by bit-parallel LCS per window pair (the BLCS method of
 * Crochemore et al. that Section 4 compares against): for each x-window a
 * w-bit vector per y-window takes, letter by letter, U = V & M[c],
 * V = (V + U) | (V - U), and WLCS is the number of its zero bits; O(m n w
 * ceil(w/32)) word operations.  A second baseline; same outputs and errors
 * as wlcs_plot. */
int wlcs_plot_blcs(wlcs_ctx *ctx, const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
                   int32_t w, const uint8_t *alphabet, int32_t sigma, uint8_t *wlcs, int64_t ld,
                   uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint16_t *indel,
                   int64_t ld_indel, uint32_t flags, void *stream);

/* Alignment-score plot (Section 2's scoring: match 1, mismatch 0, gap -1/2)
 * with a vertical step, as in the paper's experiments (Section 4).  Row r is
 * the x-window starting at x[r * step] (r < ceil((m - w) / step)), column j the
 * y-window starting at y[j] (j < n - w; WLCS_FULL_RANGE: m - w + 1 and
 * n - w + 1 windows).  score[r*ld + j] is the best alignment score of the two
 * windows, an integer in [-w, w] stored as int8.  The library computes it by
 * the paper's reduction: with a separator letter inserted before every letter
 * of both strings, the score of two w-windows equals the LLCS of their
 * 2w-letter images minus w; the plot is the seaweed plot of the blown-up
 * strings at window 2w, taken at every second window (the (2w, 2)-restricted
 * plot of Definition 3.2).  The separator takes one letter code, so sigma must
 * be at most 63.  bitmap (optional) marks score >= threshold (-128..127).
 * 1 <= w <= WLCS_MAX_SCORE_W, step >= 1. */
int wlcs_score_plot(wlcs_ctx *ctx, const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w,
                    int32_t step, const uint8_t *alphabet, int32_t sigma, int8_t *score, int64_t ld,
                    uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint32_t flags, void *stream);

/* ---- device-resident pairs --------------------------------------------
 * A pair holds x and y on the device, already mapped to letter codes, so that
 * repeated plots (several windows, benchmarking, a serving loop) start from
 * inputs resident in HBM.  The pair owns its device memory, taken in stream
 * order on the stream it is created on, until wlcs_pair_destroy. */
typedef struct wlcs_pair wlcs_pair;

/* Copy host strings x (m bytes) and y (n bytes) to the device and encode them
 * (letters checked against the alphabet on the host first, as in wlcs_plot).
 * The encoding runs on `stream`; the host strings may be reused on return. */
int wlcs_pair_create(wlcs_ctx *ctx, const uint8_t *x, int64_t m, const uint8_t *y, int64_t n,
                     const uint8_t *alphabet, int32_t sigma, void *stream, wlcs_pair **out);

/* Release a pair's device memory in stream order on its creation stream
 * (no device-wide wait).  Work already enqueued on that stream still sees the
 * codes, and so does work that this library enqueued on other streams (plots,
 * batches, graph replays): every call that reads the pair on another stream
 * records an event there, and the creation stream waits for those events
 * before the free.  Work captured into a graph by the caller (not a
 * wlcs_batch_graph) must have completed.  The creation stream must still
 * exist.  NULL is accepted. */
int wlcs_pair_destroy(wlcs_pair *pair);

/* wlcs_plot / wlcs_plot_dp on a resident pair: same window, output, flag and
 * error conventions; the pair must belong to ctx's device. */
int wlcs_pair_plot(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, uint8_t *wlcs, int64_t ld,
                   uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint16_t *indel,
                   int64_t ld_indel, uint32_t flags, void *stream);
int wlcs_pair_plot_dp(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, uint8_t *wlcs, int64_t ld,
                      uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint16_t *indel,
                      int64_t ld_indel, uint32_t flags, void *stream);
int wlcs_pair_plot_blcs(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, uint8_t *wlcs, int64_t ld,
                        uint64_t *bitmap, int64_t ld_words, int32_t threshold, uint16_t *indel,
                        int64_t ld_indel, uint32_t flags, void *stream);

/* ---- strided and sparse plots ---------------------------------------------
 * Section 3's step size: only windows starting at multiples of a step are
 * compared.  Output row r is the x-window starting at r*hx, column c the
 * y-window starting at c*hy (0-based), so rows = ceil((m-w)/hx) and
 * cols = ceil((n-w)/hy) (over m-w+1 and n-w+1 windows with WLCS_FULL_RANGE).
 * The x-step divides the seaweed work by hx (only every hx-th strip is
 * combed); the y-step thins the output (every column of a strip is combed
 * anyway, and the sliding count visits every window).
 *
 * Section 1's dot plot as a list: every (r, c) with WLCS >= threshold, as the
 * record below (window starts, WLCS, indel distance 2w - 2*WLCS), in no
 * particular order (the set is the same on every run; the order is not).
 *
 *   hx, hy            steps, >= 1 (hx = hy = 1: the plain plot).
 *   wlcs, ld          uint8 plot over the strided grid, ld >= cols.  May be NULL.
 *   bitmap, ld_words  as in wlcs_plot, over the strided grid; only with hy = 1
 *                     (WLCS_EINVAL otherwise: the dot list serves thresholds
 *                     with a y-step).  May be NULL.
 *   threshold         for the bitmap and the dot list, 0..255.
 *   indel, ld_indel   uint16 over the strided grid.  May be NULL.
 *   dot_count         device uint64: if non-NULL the dots are listed and
 *                     *dot_count is set (on the stream, also for an empty
 *                     plot) to their number, which may exceed dot_cap.
 *   dots, dot_cap     device array of dot_cap records; the first
 *                     min(*dot_count, dot_cap) dots are written there.  dots
 *                     may be NULL to count only; non-NULL needs dot_count.
 * At least one of wlcs, bitmap, indel, dot_count must be given unless the plot
 * is empty (then the call only sets *dot_count to 0).  Window starts
 * must fit 32 bits when dots are listed (WLCS_ERANGE otherwise). */
typedef struct {
    uint32_t i, j;  /* window starts in x and y (0-based) */
    uint16_t wlcs;  /* WLCS(i, j) >= threshold */
    uint16_t indel; /* 2w - 2*WLCS(i, j) */
} wlcs_dot;

int wlcs_pair_plot_strided(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, int32_t hx, int32_t hy,
                           uint8_t *wlcs, int64_t ld, uint64_t *bitmap, int64_t ld_words,
                           int32_t threshold, uint16_t *indel, int64_t ld_indel, wlcs_dot *dots,
                           int64_t dot_cap, uint64_t *dot_count, uint32_t flags, void *stream);
/* The same outputs by the plain per-window dynamic program (the paper's
 * baseline with a step size: its work falls by hx * hy). */
int wlcs_pair_plot_dp_strided(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, int32_t hx, int32_t hy,
                              uint8_t *wlcs, int64_t ld, uint64_t *bitmap, int64_t ld_words,
                              int32_t threshold, uint16_t *indel, int64_t ld_indel, wlcs_dot *dots,
                              int64_t dot_cap, uint64_t *dot_count, uint32_t flags, void *stream);

/* The dot list of a resident pair (every window pair with WLCS >= threshold,
 * as wlcs_pair_plot_strided lists it with hx = hy = 1), exact, without combing
 * every strip.  Section 3 notes that the per-window dynamic program can use
 * the threshold, and the Conclusions propose a heuristic like that of Ott et
 * al. for the seaweed method; this is an exact version of such a filter.  It
 * rests on one property of the plot: moving the x-window by one letter changes
 * its LLCS with any y-window by at most one, so |WLCS(i + d, j) - WLCS(i, j)|
 * <= |d|.  The probe strips -- every probe_step-th x-window, starting at
 * half the remainder of (rows - 1) / probe_step so that no row is more than
 * floor(probe_step / 2) rows from a probe -- are combed and listed at
 * threshold - floor(probe_step / 2); every other
 * row takes its nearest probe (the lower one on ties), and only its windows
 * whose probe entry comes within reach of the threshold are evaluated, each
 * exactly (bit-parallel LCS of the window pair).  probe_step = 1 combs every
 * strip.  The list is unique and complete; the order of the records is not
 * defined.  The probe entries go to a list of probe_cap records (0: the
 * library picks one entry per 32 probe window pairs, at least 65,536, at most
 * 2^27); if they exceed it, a gated launch lists every strip instead, so the
 * result stays exact.  *dot_count (device) receives the number of dots, even
 * past dot_cap; records beyond dot_cap are not written.  Cost: the probe
 * strips (a 1 / probe_step share of the plot) plus the candidates, whose
 * number grows quickly as threshold - probe_step / 2 nears the background
 * level of the plot.  Errors: WLCS_ERANGE for w outside 1..WLCS_MAX_W or
 * probe_step < 1; WLCS_EINVAL for a null dot_count, threshold outside 0..255,
 * or negative capacities. */
int wlcs_pair_dots_filtered(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, int32_t threshold,
                            int32_t probe_step, int64_t probe_cap, wlcs_dot *dots, int64_t dot_cap,
                            uint64_t *dot_count, uint32_t flags, void *stream);

/* ---- batched plots ------------------------------------------------------
 * Many plots of uneven m, n and w in persistent, work-stealing launches: the
 * plots' units (64 x-windows against two y-tiles) go into device-wide queues
 * that resident wavefronts drain, one queue and launch per group of window
 * classes (w <= 32, w <= 64, w <= 128: each group's kernel holds only its own
 * classes' code and runs at that group's occupancy; longer windows run as
 * separate launches on the same stream).  Each plot's outputs are exactly
 * those of wlcs_pair_plot with the same arguments. */
typedef struct {
    const wlcs_pair *pair; /* resident strings (wlcs_pair_create on the same device) */
    int32_t w;
    uint32_t flags;        /* 0 or WLCS_FULL_RANGE */
    uint8_t *wlcs;         /* outputs as in wlcs_plot; any may be NULL, not all */
    int64_t ld;
    uint64_t *bitmap;
    int64_t ld_words;
    int32_t threshold;
    uint16_t *indel;
    int64_t ld_indel;
    /* strided and sparse outputs, as in wlcs_pair_plot_strided (a job left
     * zero-filled here is a plain plot: steps 0 and 1 both mean every window) */
    int32_t hx, hy;
    wlcs_dot *dots;
    int64_t dot_cap;
    uint64_t *dot_count;
} wlcs_job;

/* Enqueue all njobs plots on `stream`.  Jobs are checked on the host first
 * (with the rules of wlcs_pair_plot_strided for steps and dot lists); a
 * bad job fails the whole call before anything is enqueued.  The job array and
 * the table built from it are consumed before the call returns; pairs and
 * outputs must stay valid until the stream has run the batch. */
int wlcs_batch(wlcs_ctx *ctx, const wlcs_job *jobs, int32_t njobs, void *stream);

/* wlcs_batch for callers that cannot allocate (code under stream capture,
 * serving loops, harnesses that forbid allocation): the same plots, the same
 * kernels and the same job checks, but the job table, the work counters and
 * the dot counters' addresses live in a fixed device scratch of
 * WLCS_NOALLOC_SCRATCH_BYTES (1 MiB) that each device holds for the life of
 * the process, written in stream order by small kernels that carry the
 * table in their arguments.  No device, pinned or managed memory is allocated
 * or freed, and nothing is copied through a staging buffer; the host-side
 * plan reuses per-thread buffers once they have held a batch as large.  A
 * batch whose table, counters and addresses exceed the scratch returns
 * WLCS_ESCRATCH before anything is enqueued: a job takes one or two table
 * entries of 184 bytes (two when its rows span more than one pair of
 * y-tiles) and 8 bytes if it lists dots, so about 2,780 jobs always fit.  Every call on a device shares that device's
 * scratch: calls that overlap on one device (on different streams, or from
 * different threads) race and must not be made; calls one after another on
 * one stream are ordered.  Windows above 128 run as in wlcs_batch (their
 * single-plot launches use no scratch).  Pairs and outputs must stay valid
 * until the stream has run the batch. */
#define WLCS_NOALLOC_SCRATCH_BYTES (1u << 20)
int wlcs_batch_noalloc(wlcs_ctx *ctx, const wlcs_job *jobs, int32_t njobs, void *stream);

/* The same batch captured once into a HIP graph (job table and work counter
 * owned by the graph), to be replayed with wlcs_graph_launch as many times as
 * wanted; each replay recomputes every plot of the batch.  The jobs' pairs and
 * outputs must outlive the graph. */
typedef struct wlcs_graph wlcs_graph;
int wlcs_batch_graph(wlcs_ctx *ctx, const wlcs_job *jobs, int32_t njobs, wlcs_graph **out);
int wlcs_graph_launch(wlcs_graph *graph, void *stream);
int wlcs_graph_destroy(wlcs_graph *graph); /* waits for the graph's device memory to be idle */

/* Batch tuning: y-windows per tile for batched plots of windows w_lo..w_hi
 * (multiple of 64, 64..32768; 0 restores the built-in choice, which aims at
 * equal work per unit: about 131072 / w windows), and the persistent grids
 * (waves per compute unit, 1..16, for every group, the 128-row group in
 * workgroups of two waves; 0 restores the default: each group's resident
 * capacity, 16 waves per CU for w <= 32, 12 above). */
int wlcs_ctx_set_batch_tile(wlcs_ctx *ctx, int32_t w_lo, int32_t w_hi, int32_t tile_windows);
int wlcs_ctx_set_batch_grid(wlcs_ctx *ctx, int32_t waves_per_cu);

/* Latency of small jobs in a batch: a job whose tiles (as set above, or the
 * built-in choice) give it fewer than min_units units (64 x-windows by one
 * pair of tiles each) has its tiles shortened, in whole blocks of 64 windows
 * down to 64, until it has at least that many, so that it spreads over the
 * device instead of combing long tiles on a few waves.  Jobs with enough
 * units keep their tiles; the plots do not depend on the tiling.  min_units
 * 0 (the default) turns this off; 1..1,048,576 otherwise, else WLCS_EINVAL.
 * A serving loop sets about one unit per SIMD of the device. */
int wlcs_ctx_set_batch_min_units(wlcs_ctx *ctx, int64_t min_units);

/* What applies now: the tile set for batched plots of window w (0 if the
 * built-in choice applies), and the persistent grid (0: the default). */
int wlcs_ctx_get_batch_tile(const wlcs_ctx *ctx, int32_t w, int32_t *tile_windows);
int wlcs_ctx_get_batch_grid(const wlcs_ctx *ctx, int32_t *waves_per_cu);

/* Autotuner of the batched launch: the y-windows per tile of each window class
 * (1-16, 17-32, 33-64, 65-128) and the persistent grid, picked by timing real
 * batched launches of a seeded synthetic batch (128 uniform random DNA pairs,
 * m, n in 1,000..16,000, 32 per class) on the context's device, and applied
 * to ctx with wlcs_ctx_set_batch_tile / wlcs_ctx_set_batch_grid.  The search
 * starts from the built-in choices and changes one knob at a time (each
 * class's tile in turn: 256..4096; then the grid: 4..16 waves per CU),
 * keeping a candidate only if the whole batch runs faster with it, so the
 * result never times slower than the built-in choices.  A knob left at its
 * built-in choice is stored as 0.
 *
 *   cache_path  JSON file of results keyed by device ("gfx950-256cu": the
 *               architecture and compute-unit count).  If it holds an entry
 *               for this device, the entry is applied and nothing is timed;
 *               otherwise the tuner runs and the entry is added to the file
 *               (created if missing; other devices' entries are kept; written
 *               to a temporary file, then renamed).  NULL: tune, apply, write
 *               nothing.
 *   flags       0, or WLCS_TUNE_FORCE to tune even when the cache has an entry
 *               (the entry is then replaced).
 *
 * Synchronous: returns when the tuning launches have completed (a few seconds
 * of device time; up to about 15 GB of device memory is taken and released).
 * Errors: WLCS_EINVAL for a bad flag or a cache file that is not a JSON object,
 * or whose entry for this device does not have the shape above (the file is
 * then left as it is and nothing is applied); WLCS_EIO if the cache cannot be
 * written (the tuned values are applied all the same); WLCS_EHIP / WLCS_ENOMEM
 * from the device.  Window tiling does not change any result, only speed
 * (Theorem 3.1 holds for every tile). */
#define WLCS_TUNE_FORCE 1u
int wlcs_tune(wlcs_ctx *ctx, const char *cache_path, uint32_t flags);

/* Tiling tuner of one plot shape: times the seaweed kernel on `pair` (window
 * w, every hx-th x-window, every y-window; flags 0 or WLCS_FULL_RANGE, as in
 * wlcs_pair_plot_strided) under a coarse grid of tilings (long tiles of
 * 256..6144 windows for a count of leading pairs, short tiles of 128..1024
 * after them, or one length), then around the fastest of them, then times
 * the three fastest and the built-in choice again with more launches and
 * keeps the fastest.  The result is recorded in ctx for the shape (rows,
 * cols, w) and then applies to every plot of that shape made through ctx
 * (wlcs_pair_plot, wlcs_plot, their strided forms; not score plots), ahead
 * of the built-in tile model and behind tile rules (wlcs_ctx_set_tile(s)).
 * The built-in tile model scores tilings by a schedule of equal slots; this
 * measures them on the device instead.
 *
 *   cache_path  the JSON cache of wlcs_tune (NULL: tune, apply, write
 *               nothing).  The device's entry holds "plots": {"RxCxW":
 *               [long_tile, short_tile, long_pairs]} (0, 0, 0: the built-in
 *               choice was the fastest) and the times in "plots_ms".  If it
 *               holds this shape, that tiling is applied and nothing is timed;
 *               otherwise the result is added (the entry's other members are
 *               kept; wlcs_tune completes an entry that has no batch knobs yet
 *               and keeps its plot tilings).
 *   tune_flags  0, or WLCS_TUNE_FORCE to time even when the cache has the
 *               shape (its record is then replaced).
 *
 * Synchronous: returns when the timed plots have completed (a few seconds for
 * a 50,000 x 50,000 plot); rows x cols bytes of device memory are taken and
 * released.  Errors as for wlcs_tune, plus WLCS_ERANGE for w outside
 * 1..WLCS_MAX_W or hx < 1.  An empty plot returns WLCS_OK at once.  Tiling
 * does not change any result (Theorem 3.1 holds for every tile). */
int wlcs_tune_plot(wlcs_ctx *ctx, const wlcs_pair *pair, int32_t w, int32_t hx, uint32_t flags,
                   const char *cache_path, uint32_t tune_flags);

/* The measured tiling that applies to plots of rows x cols windows of length
 * w (rows counted after the x-step), from wlcs_tune_plot or a loaded cache;
 * all three 0 if none (the built-in choice applies). */
int wlcs_ctx_get_plot_tiling(const wlcs_ctx *ctx, int64_t rows, int64_t cols, int32_t w, int32_t *long_tile,
                             int32_t *short_tile, int32_t *long_pairs);

#ifdef __cplusplus
}
#endif

#endif /* WLCS_H */
