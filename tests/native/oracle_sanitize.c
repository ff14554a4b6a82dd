/*
 * CPU check of the oracle under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Links oracle/wlcs_oracle.c into this program and calls every entry point on
 * seeded random strings (DNA, binary and 20-letter alphabets; windows 1..255;
 * empty, single-window and full-range plots; every thread count up to 9),
 * checking that the entry points agree with each other (O-batch with the plain
 * plot, selected rows and single entries with the plot, the strided plot with
 * the plot's sub-grid) and that bad arguments are refused.  Any out-of-bounds
 * access or undefined behaviour aborts the program; a disagreement prints the
 * case and exits 1.
 *
 * Usage: oracle_sanitize SEED ROUNDS
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_llcs(const uint8_t *a, int64_t la, const uint8_t *b, int64_t lb);
int oracle_wlcs(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, int32_t full_range,
                uint8_t *out, int64_t ld, int32_t nthreads);
int oracle_wlcs_strided(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, int64_t hx,
                        int64_t hy, int32_t full_range, uint8_t *out, int64_t ld, int32_t nthreads);
int oracle_wlcs_rows(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, int32_t full_range,
                     const int64_t *row_ids, int64_t nrows, uint8_t *out, int64_t ld, int32_t nthreads);
int oracle_wlcs_at(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, const int64_t *ii,
                   const int64_t *jj, int64_t count, uint8_t *out);
int oracle_wlcs_batch(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, int32_t full_range,
                      const int64_t *row_ids, int64_t nrows, uint8_t *out, int64_t ld, int32_t nthreads);
int oracle_score2(const uint8_t *a, int64_t la, const uint8_t *b, int64_t lb, int32_t *out);
int oracle_score_plot(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, int32_t step,
                      int32_t full_range, int8_t *out, int64_t ld, int32_t nthreads);

static uint64_t rng_state;
static uint64_t next_u64(void)
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int64_t uni(int64_t lo, int64_t hi) { return lo + (int64_t)(next_u64() % (uint64_t)(hi - lo + 1)); }

static void fail(const char *what, int round, int w, int64_t m, int64_t n)
{
    fprintf(stderr, "FAIL %s: round %d w=%d m=%lld n=%lld\n", what, round, w, (long long)m, (long long)n);
    exit(1);
}

static uint8_t *rand_string(int64_t len, const char *alpha)
{
    const int64_t s = (int64_t)strlen(alpha);
    uint8_t *p = (uint8_t *)malloc((size_t)(len > 0 ? len : 1));
    for (int64_t i = 0; i < len; ++i) p[i] = (uint8_t)alpha[uni(0, s - 1)];
    return p;
}

int main(int argc, char **argv)
{
    rng_state = argc > 1 ? strtoull(argv[1], NULL, 10) : 1;
    const int rounds = argc > 2 ? atoi(argv[2]) : 40;
    static const char *alphas[] = {"ACGT", "AB", "ACDEFGHIKLMNPQRSTVWY"};
    static const int ws[] = {1, 2, 3, 5, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 100, 128, 129, 200, 255};
    for (int round = 0; round < rounds; ++round) {
        const int w = ws[uni(0, (int64_t)(sizeof ws / sizeof ws[0]) - 1)];
        const char *alpha = alphas[uni(0, 2)];
        const int64_t m = w + uni(-1, 40), n = w + uni(-1, 150);
        const int full = (int)uni(0, 1);
        const int nt = (int)uni(1, 9);
        const int64_t mm = m > 0 ? m : 0, nn = n > 0 ? n : 0;
        uint8_t *x = rand_string(mm, alpha), *y = rand_string(nn, alpha);
        const int64_t rows = mm - w + full > 0 ? mm - w + full : 0;
        const int64_t cols = nn - w + full > 0 ? nn - w + full : 0;
        const int64_t ld = cols + uni(0, 5);
        uint8_t *plot = (uint8_t *)calloc((size_t)(rows * ld + 1), 1);
        uint8_t *plot_b = (uint8_t *)calloc((size_t)(rows * ld + 1), 1);
        if (oracle_wlcs(x, mm, y, nn, w, full, plot, ld, nt) != 0) fail("oracle_wlcs", round, w, mm, nn);
        if (oracle_wlcs_batch(x, mm, y, nn, w, full, NULL, 0, plot_b, ld, nt) != 0)
            fail("oracle_wlcs_batch", round, w, mm, nn);
        for (int64_t r = 0; r < rows; ++r)
            if (memcmp(plot + r * ld, plot_b + r * ld, (size_t)cols)) fail("batch != plot", round, w, mm, nn);
        for (int64_t r = 0; r < rows; ++r)
            for (int64_t c = 0; c < cols; ++c)
                if (plot[r * ld + c] > w) fail("entry above w", round, w, mm, nn);
        if (rows > 0 && cols > 0) {
            /* selected rows, plain and O-batch */
            const int64_t k = uni(1, rows < 6 ? rows : 6);
            int64_t *ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
            for (int64_t q = 0; q < k; ++q) ids[q] = uni(0, rows - 1);
            uint8_t *sel = (uint8_t *)malloc((size_t)(k * cols));
            if (oracle_wlcs_rows(x, mm, y, nn, w, full, ids, k, sel, cols, nt) != 0)
                fail("oracle_wlcs_rows", round, w, mm, nn);
            for (int64_t q = 0; q < k; ++q)
                if (memcmp(sel + q * cols, plot + ids[q] * ld, (size_t)cols)) fail("rows != plot", round, w, mm, nn);
            if (oracle_wlcs_batch(x, mm, y, nn, w, full, ids, k, sel, cols, nt) != 0)
                fail("oracle_wlcs_batch rows", round, w, mm, nn);
            for (int64_t q = 0; q < k; ++q)
                if (memcmp(sel + q * cols, plot + ids[q] * ld, (size_t)cols))
                    fail("batch rows != plot", round, w, mm, nn);
            /* single entries */
            int64_t ii[8], jj[8];
            uint8_t at[8];
            for (int q = 0; q < 8; ++q) {
                ii[q] = uni(0, rows - 1);
                jj[q] = uni(0, cols - 1);
            }
            if (oracle_wlcs_at(x, mm, y, nn, w, ii, jj, 8, at) != 0) fail("oracle_wlcs_at", round, w, mm, nn);
            for (int q = 0; q < 8; ++q)
                if (at[q] != plot[ii[q] * ld + jj[q]]) fail("at != plot", round, w, mm, nn);
            /* strided: the sub-grid of the plot */
            const int64_t hx = uni(1, 5), hy = uni(1, 5);
            const int64_t orows = (rows + hx - 1) / hx, ocols = (cols + hy - 1) / hy;
            uint8_t *st = (uint8_t *)malloc((size_t)(orows * ocols));
            if (oracle_wlcs_strided(x, mm, y, nn, w, hx, hy, full, st, ocols, nt) != 0)
                fail("oracle_wlcs_strided", round, w, mm, nn);
            for (int64_t r = 0; r < orows; ++r)
                for (int64_t c = 0; c < ocols; ++c)
                    if (st[r * ocols + c] != plot[r * hx * ld + c * hy]) fail("strided != plot", round, w, mm, nn);
            /* a window pair by the textbook table */
            if (w <= 200 && oracle_llcs(x + ii[0], w, y + jj[0], w) != plot[ii[0] * ld + jj[0]])
                fail("llcs != plot", round, w, mm, nn);
            free(ids);
            free(sel);
            free(st);
        }
        /* alignment scores (w <= 127): a plot entry equals the pair's score */
        if (w <= 127 && rows > 0 && cols > 0) {
            const int32_t step = (int32_t)uni(1, 4);
            const int64_t srows = (rows + step - 1) / step;
            int8_t *sp = (int8_t *)malloc((size_t)(srows * cols));
            if (oracle_score_plot(x, mm, y, nn, w, step, full, sp, cols, nt) != 0)
                fail("oracle_score_plot", round, w, mm, nn);
            const int64_t r = uni(0, srows - 1), c = uni(0, cols - 1);
            int32_t s2 = 0;
            if (oracle_score2(x + r * step, w, y + c, w, &s2) != 0) fail("oracle_score2", round, w, mm, nn);
            if (sp[r * cols + c] != s2 / 2) fail("score plot != score", round, w, mm, nn);
            free(sp);
        }
        /* refusals */
        uint8_t tiny[4];
        int64_t bad = rows + 1;
        if (oracle_wlcs(x, mm, y, nn, 0, full, plot, ld, nt) == 0) fail("w = 0 accepted", round, w, mm, nn);
        if (oracle_wlcs(x, mm, y, nn, 256, full, plot, ld, nt) == 0) fail("w = 256 accepted", round, w, mm, nn);
        if (rows > 0 && cols > 1 && oracle_wlcs(x, mm, y, nn, w, full, plot, cols - 1, nt) == 0)
            fail("short ld accepted", round, w, mm, nn);
        if (rows > 0 && cols > 0 && oracle_wlcs_rows(x, mm, y, nn, w, full, &bad, 1, tiny, cols, nt) == 0)
            fail("row past the plot accepted", round, w, mm, nn);
        if (oracle_wlcs_strided(x, mm, y, nn, w, 0, 1, full, plot, ld, nt) == 0)
            fail("step 0 accepted", round, w, mm, nn);
        free(x);
        free(y);
        free(plot);
        free(plot_b);
    }
    printf("ok: %d rounds\n", rounds);
    return 0;
}
