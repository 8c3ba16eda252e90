/* Host sanitizer driver for the C ABI's host code: argument validation, the
 * launch-table parser and lookup, configuration forcing, saved-state sizes
 * and error reporting.  The kernel launchers are stubbed out (no GPU is
 * needed or touched); built with -fsanitize=address,undefined on the host
 * side only.  argv[1]: the installed launch table; argv[2]: a scratch path. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "rd.h"

#define CHECK(c)                                                 \
    do {                                                         \
        if (!(c)) {                                              \
            fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, rd_last_error()); \
            return 1;                                            \
        }                                                        \
    } while (0)

int main(int argc, char** argv) {
    if (argc < 3) return 2;
    void* fake = (void*)(uintptr_t)0x10000; /* never dereferenced: validation fails first */
    rd_dtype out;
    for (int dt = 0; dt < 8; ++dt)
        for (int op = 0; op < 7; ++op) CHECK(rd_out_dtype((rd_dtype)dt, (rd_op)op, &out) == RD_OK);
    CHECK(rd_out_dtype((rd_dtype)9, RD_SUM, &out) == RD_ERR_INVALID_ARG);
    CHECK(rd_dtype_size(RD_BF16) == 2 && rd_dtype_size((rd_dtype)42) == 0);

    CHECK(rd_reduce(fake, -1, RD_F32, RD_SUM, fake, NULL, NULL) == RD_ERR_INVALID_ARG);
    CHECK(strstr(rd_last_error(), "n = -1") != NULL);
    CHECK(rd_reduce(NULL, 4, RD_F32, RD_SUM, fake, NULL, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_reduce((void*)(uintptr_t)0x10001, 4, RD_F32, RD_SUM, fake, NULL, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_reduce_noalloc(fake, -5, RD_I32, RD_XOR, fake, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_reduce_noalloc(fake, 5, RD_I32, (rd_op)12, fake, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_reduce_compensated(fake, 4, RD_I32, (double*)fake, NULL, NULL) == RD_ERR_UNSUPPORTED);
    CHECK(rd_segmented_reduce(fake, (const int64_t*)fake, -1, RD_F32, RD_SUM, fake, NULL, NULL) ==
          RD_ERR_INVALID_ARG);
    CHECK(rd_segmented_reduce(fake, (const int64_t*)fake, 0, RD_F32, RD_SUM, fake, NULL, NULL) == RD_OK);
    CHECK(rd_argreduce(fake, 4, RD_F32, RD_SUM, fake, (int64_t*)fake, NULL, NULL) == RD_ERR_UNSUPPORTED);
    CHECK(rd_scan(fake, -2, RD_F32, RD_SUM, 0, fake, NULL, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_scan(fake, 0, RD_F32, RD_SUM, 0, fake, NULL, NULL) == RD_OK);
    CHECK(rd_segmented_scan(fake, 4, (const int64_t*)fake, -1, RD_F32, RD_SUM, 0, fake, NULL, NULL) ==
          RD_ERR_INVALID_ARG);
    CHECK(rd_reduce_paper_design(fake, 4, RD_F64, 0, 1, fake, NULL, NULL) == RD_ERR_UNSUPPORTED);
    CHECK(rd_reduce_paper_design(fake, 4, RD_F32, 1, 9, fake, NULL, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_rowreduce_fwd(fake, 2, 2, RD_F64, RD_SUM, fake, fake, NULL) == RD_ERR_UNSUPPORTED);
    CHECK(rd_rowreduce_fwd(fake, -1, 2, RD_F32, RD_SUM, fake, fake, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_rowreduce_bwd(fake, fake, fake, 2, 2, RD_F32, RD_XOR, fake, NULL) == RD_ERR_UNSUPPORTED);
    CHECK(rd_rowreduce_bwd(fake, fake, fake, 0, 5, RD_F32, RD_SUM, fake, NULL) == RD_OK);
    (void)rd_saved_bytes(RD_PROD, 8, 16385);
    CHECK(rd_workspace_destroy(NULL) == RD_OK);
    CHECK(rd_workspace_reset(NULL, NULL) == RD_ERR_INVALID_ARG);
    CHECK(rd_workspace_status(NULL, NULL) == RD_ERR_INVALID_ARG);

    /* configuration: get, force, clear, reject */
    rd_config c;
    CHECK(rd_config_get(RD_KIND_PLAIN, RD_F32, RD_SUM, (int64_t)1 << 28, &c) == RD_OK);
    rd_config forced = {512, 4, 2, 1, 1};
    CHECK(rd_config_force(RD_KIND_PLAIN, &forced) == RD_OK);
    CHECK(rd_config_get(RD_KIND_PLAIN, RD_I32, RD_XOR, 31, &c) == RD_OK && c.block == 512 && c.unroll == 4);
    CHECK(rd_config_force(RD_KIND_PLAIN, NULL) == RD_OK);
    rd_config bad = {100, 3, 0, 2, 7};
    CHECK(rd_config_force(RD_KIND_SCAN, &bad) == RD_ERR_INVALID_ARG);
    CHECK(rd_config_force((rd_kind)99, &forced) == RD_ERR_INVALID_ARG);
    CHECK(rd_config_get((rd_kind)-1, RD_F32, RD_SUM, 4, &c) == RD_ERR_INVALID_ARG);

    /* the launch-table parser: the installed table, a malformed one, defaults */
    CHECK(rd_tune_load(argv[1]) == RD_OK);
    for (int k = 0; k <= RD_KIND_SEGMENTED_SCAN; ++k)
        for (int dt = 0; dt < 8; ++dt)
            for (int op = 0; op < 7; ++op)
                for (int l = 0; l < 63; l += 7)
                    CHECK(rd_config_get((rd_kind)k, (rd_dtype)dt, (rd_op)op, (int64_t)1 << l, &c) == RD_OK);
    FILE* f = fopen(argv[2], "w");
    if (!f) return 2;
    fputs("# comment only\n\n0 4 0 0 62 256 2 2 1 0   # trailing comment\n0 4 0 0 62 256 3\n", f);
    fclose(f);
    CHECK(rd_tune_load(argv[2]) == RD_ERR_INVALID_ARG);
    CHECK(strstr(rd_last_error(), "malformed") != NULL);
    f = fopen(argv[2], "w");
    if (!f) return 2;
    fputs("0 4 0 0 62 256 2 2 1 0\n", f);
    for (int i = 0; i < 600; ++i) fputc('x', f); /* a line longer than the parser's buffer */
    fputc('\n', f);
    fclose(f);
    (void)rd_tune_load(argv[2]); /* either verdict is fine; it must not overrun */
    CHECK(rd_tune_load("/nonexistent/table.txt") == RD_ERR_INVALID_ARG);
    CHECK(rd_tune_load(NULL) == RD_OK);
    puts("abi driver ok");
    return 0;
}
