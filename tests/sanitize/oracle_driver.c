/* Host sanitizer driver for the CPU oracle: every entry point on small and
 * edge-case inputs (empty arrays, empty segments, out-of-range heads, rows
 * with zeros), with a few results checked against closed forms.  Built with
 * -fsanitize=address,undefined; any report or a wrong value fails the run. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                            \
        }                                                        \
    } while (0)

int main(void) {
    enum { N = 1000 };
    static uint32_t u32[N];
    static uint64_t u64[N];
    static uint16_t u16[N];
    static float f32[N];
    static double f64[N];
    for (int i = 0; i < N; ++i) {
        u32[i] = (uint32_t)i;
        u64[i] = (uint64_t)i * 3u;
        u16[i] = (uint16_t)(0x3C00 + (i % 7)); /* float16 values near 1 */
        f32[i] = (float)i;
        f64[i] = 0.5 * i;
    }
    uint32_t o32;
    uint64_t o64;
    uint16_t o16;
    for (int op = 0; op < 7; ++op) {
        CHECK(orc_fold_u32(u32, N, op, 1, &o32) == 0);
        CHECK(orc_fold_u32(u32, 0, op, 0, &o32) == 0);
        CHECK(orc_fold_u64(u64, N, op, 0, &o64) == 0);
    }
    CHECK(orc_fold_u32(u32, N, 0, 1, &o32) == 0 && o32 == 499500u);
    for (int op = 4; op < 7; ++op) CHECK(orc_fold_u16(u16, N, op, &o16) == 0);
    int64_t at;
    CHECK(orc_argext_int(u32, N, 32, 1, 1, &o64, &at) == 0 && at == N - 1);
    CHECK(orc_argext_int(u64, 0, 64, 0, 0, &o64, &at) == 0 && at == -1);

    double s, a;
    CHECK(orc_exact_sum(f32, N, 2, &s, &a) == 0 && s == 499500.0);
    CHECK(orc_exact_sum(f64, N, 3, &s, &a) == 0 && s == 249750.0);
    CHECK(orc_exact_sum(u16, N, 4, &s, &a) == 0);
    CHECK(orc_exact_sum(u16, N, 5, &s, &a) == 0);
    CHECK(orc_exact_sum(f32, 0, 2, &s, &a) == 0 && s == 0.0);
    double p;
    CHECK(orc_prod(f64 + 1, 10, 3, &p) == 0 && p == 3628800.0 / 1024.0);
    CHECK(orc_prod(u16, N, 4, &p) == 0);
    double m;
    CHECK(orc_minmax(f32, N, 2, 1, &m, &at) == 0 && m == 999.0 && at == N - 1);
    CHECK(orc_minmax(f32, 0, 2, 0, &m, &at) == 0 && isinf(m) && at == -1);
    CHECK(orc_load_float(u16, 3, 4) > 0.0);

    /* segmented: empty segments, a zero-length start, one long segment */
    const int64_t off[] = {0, 0, 5, 5, 5, 500, 999, 1000};
    const int64_t nseg = 7;
    double segd[7];
    uint64_t segb[7];
    for (int op = 0; op < 4; ++op) CHECK(orc_segmented(f32, off, nseg, 2, op, segd) == 0);
    CHECK(orc_segmented(f32, off, nseg, 2, 0, segd) == 0 && segd[1] == 10.0 && segd[0] == 0.0);
    for (int op = 0; op < 7; ++op) CHECK(orc_segmented(u32, off, nseg, 0, op, segb) == 0);
    CHECK(orc_segmented(u16, off, nseg, 5, 6, segb) == 0);

    /* scans: plain, exclusive, heads in and out of range */
    static double scd[N];
    static uint64_t scb[N];
    const int64_t heads[] = {-3, 0, 10, 10, 500, 999, 1000, 5000};
    CHECK(orc_scan(f32, N, 2, 0, 0, NULL, 0, scd) == 0 && scd[N - 1] == 499500.0);
    CHECK(orc_scan(f32, N, 2, 1, 1, heads, 8, scd) == 0);
    for (int op = 0; op < 7; ++op) CHECK(orc_scan(u32, N, 1, op, op & 1, heads, 8, scb) == 0);
    CHECK(orc_scan(u16, N, 4, 6, 0, heads, 8, scb) == 0);
    CHECK(orc_scan(f32, 0, 2, 0, 0, NULL, 0, scd) == 0);

    /* row-wise forward and gradients, with zeros in the product rows */
    enum { R = 4, C = 37 };
    static float x[R * C];
    for (int i = 0; i < R * C; ++i) x[i] = 1.0f + 0.01f * (float)(i % 5);
    x[C + 3] = 0.0f;                    /* row 1: one zero */
    x[2 * C + 1] = x[2 * C + 30] = 0.0f; /* row 2: two zeros */
    double y[R], g[R] = {1.0, -2.0, 0.5, 3.0};
    int64_t idx[R], zeros[R];
    static double grad[R * C];
    for (int op = 0; op < 4; ++op) {
        CHECK(orc_row_forward(x, R, C, op, y, idx, zeros) == 0);
        CHECK(orc_row_grad(x, R, C, op, g, grad) == 0);
    }
    CHECK(orc_row_forward(x, R, C, 1, y, idx, zeros) == 0 && zeros[1] == 1 && zeros[2] == 2);
    CHECK(orc_row_forward(x, R, 0, 0, y, idx, zeros) == 0 && y[0] == 0.0);

    /* the timing fold, single- and multi-threaded */
    double fsum;
    CHECK(orc_fold_sum_f32(f32, N, 1, &fsum) == 0 && fsum == 499500.0);
    CHECK(orc_fold_sum_f32(f32, N, 6, &fsum) == 0 && fsum == 499500.0);
    CHECK(orc_fold_sum_f32(f32, 3, 8, &fsum) == 0 && fsum == 3.0);
    CHECK(orc_fold_sum_f32(f32, N, 0, &fsum) != 0);

    /* bad arguments are rejected, not read */
    CHECK(orc_fold_u32(u32, N, 9, 0, &o32) != 0);
    CHECK(orc_exact_sum(f32, N, 0, &s, &a) != 0);
    puts("oracle driver ok");
    return 0;
}
