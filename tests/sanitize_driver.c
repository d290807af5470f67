/*
 * Host-side paths of the C ABI under AddressSanitizer and UndefinedBehavior-
 * Sanitizer (built by tests/test_sanitize_cpu.py with host-only objects, so
 * no kernel runs): status strings, layout queries of every dtype and layout,
 * wisdom files with malformed and over-long lines, and the argument checks
 * of every entry point.  Prints "ok" and exits 0 when every call returned
 * the expected status; a sanitizer report aborts the run.
 *
 *   sanitize_driver <scratch directory>
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "bspline.h"

static int failures = 0;

#define EXPECT(call, status)                                                          \
    do {                                                                              \
        bspl_status s_ = (call);                                                      \
        if (s_ != (status)) {                                                         \
            fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__,  \
                    #call, (int)s_, (int)(status), spline_last_error());              \
            ++failures;                                                               \
        }                                                                             \
    } while (0)

static void layouts(void) {
    bspl_table_info info;
    const bspl_dtype dts[3] = {BSPL_F32, BSPL_F16, BSPL_BF16};
    const int64_t ns[6] = {1, 33, 256, 600, 2048, 4097};
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 6; ++k)
            for (unsigned fl = 0; fl <= BSPL_LAYOUT_BLOCKED; fl += BSPL_LAYOUT_BLOCKED) {
                EXPECT(spline_layout_query(5, 6, 7, ns[k], dts[d], fl, &info), BSPL_OK);
                if (info.n_padded < ns[k] || info.row_bytes % 128 != 0 ||
                    info.table_bytes != (int64_t)8 * 9 * 10 * info.n_padded * info.elem_bytes) {
                    fprintf(stderr, "layout of N=%lld dtype %d flags %u is inconsistent\n",
                            (long long)ns[k], (int)dts[d], fl);
                    ++failures;
                }
            }
    EXPECT(spline_layout_query(0, 4, 4, 8, BSPL_F32, 0, &info), BSPL_EINVAL);
    EXPECT(spline_layout_query(4, 4, 4, -1, BSPL_F32, 0, &info), BSPL_EINVAL);
    EXPECT(spline_layout_query(4, 4, 4, 8, (bspl_dtype)7, 0, &info), BSPL_EINVAL);
    EXPECT(spline_layout_query(4, 4, 4, 8, BSPL_F32, 0, NULL), BSPL_EINVAL);
    EXPECT(spline_layout_query(4096, 4096, 4096, 4096, BSPL_F32, 0, &info), BSPL_EUNSUPPORTED);
    EXPECT(spline_layout_query(1 << 28, 1 << 28, 1 << 28, 1 << 30, BSPL_F32, 0, &info),
           BSPL_EUNSUPPORTED);
}

static void wisdom(const char* dir) {
    char in[4096], out[4096], bad[4096];
    snprintf(in, sizeof in, "%s/wisdom_in.txt", dir);
    snprintf(out, sizeof out, "%s/wisdom_out.txt", dir);
    snprintf(bad, sizeof bad, "%s/no/such/dir/w.txt", dir);
    FILE* f = fopen(in, "w");
    if (!f) {
        ++failures;
        return;
    }
    fprintf(f, "# comment\n");
    fprintf(f, "single|gfx950|f32|vgh|N64|16x16x16|p1024 2 2 1 0 1 1 12.5\n");
    fprintf(f, "single-blocked|gfx950|f16|v|N600|5x6x7|p8 4 1 1 0 0 1\n");
    fprintf(f, "garbage\n\n   \nkey 1 2\n");
    for (int i = 0; i < 2000; ++i) fputc('x', f); /* a token longer than any buffer */
    fprintf(f, " 1 1 1 0 0 1\n");
    for (int i = 0; i < 700; ++i) fputs("y ", f); /* a line longer than the line buffer */
    fputc('\n', f);
    fclose(f);
    EXPECT(spline_wisdom_load(in), BSPL_OK);
    EXPECT(spline_wisdom_save(out), BSPL_OK);
    EXPECT(spline_wisdom_load(out), BSPL_OK);
    EXPECT(spline_wisdom_load(bad), BSPL_EIO);
    EXPECT(spline_wisdom_save(bad), BSPL_EIO);
    EXPECT(spline_wisdom_load(NULL), BSPL_EINVAL);
    EXPECT(spline_wisdom_save(NULL), BSPL_EINVAL);
}

static void arguments(void) {
    float coefs[8] = {0};
    double box_bad[3] = {1.0, 0.0, 1.0};
    double lat_singular[9] = {1, 0, 0, 2, 0, 0, 0, 0, 1};
    double lat_nan[9] = {1, 0, 0, 0, 1, 0, 0, 0, 0.0 / 0.0};
    bspl_table* t = (bspl_table*)1;
    EXPECT(spline_table_create(NULL, 2, 2, 2, 1, coefs, BSPL_F32, NULL, 0, NULL), BSPL_EINVAL);
    EXPECT(spline_table_create(&t, 2, 2, 2, 1, NULL, BSPL_F32, NULL, 0, NULL), BSPL_EINVAL);
    if (t != NULL) ++failures; /* cleared on failure */
    EXPECT(spline_table_create(&t, 2, 2, 2, 1, coefs, BSPL_F32, NULL, 0x100u, NULL), BSPL_EINVAL);
    EXPECT(spline_table_create(&t, 2, 2, 2, 1, coefs, BSPL_F32, NULL,
                               BSPL_COEFS_PADDED | BSPL_COEFS_GRID_VALUES, NULL), BSPL_EINVAL);
    EXPECT(spline_table_create(&t, 2, 2, 2, 1, coefs, BSPL_F32, box_bad, 0, NULL), BSPL_EINVAL);
    EXPECT(spline_table_create(&t, 0, 2, 2, 1, coefs, BSPL_F32, NULL, 0, NULL), BSPL_EINVAL);
    EXPECT(spline_table_create(&t, 2, 2, 2, 1, coefs, (bspl_dtype)5, NULL, 0, NULL), BSPL_EINVAL);
    EXPECT(spline_table_create_lattice(&t, 2, 2, 2, 1, coefs, BSPL_F32, NULL, 0, NULL),
           BSPL_EINVAL);
    EXPECT(spline_table_create_lattice(&t, 2, 2, 2, 1, coefs, BSPL_F32, lat_singular, 0, NULL),
           BSPL_EINVAL);
    EXPECT(spline_table_create_lattice(&t, 2, 2, 2, 1, coefs, BSPL_F32, lat_nan, 0, NULL),
           BSPL_EINVAL);
    EXPECT(spline_fit_interpolating(0, 2, 2, 1, coefs, coefs, NULL), BSPL_EINVAL);
    EXPECT(spline_fit_interpolating(2, 2, 2, 1, NULL, coefs, NULL), BSPL_EINVAL);
    EXPECT(spline_fit_interpolating(1 << 30, 1 << 30, 1 << 30, 1 << 20, coefs, coefs, NULL),
           BSPL_EUNSUPPORTED);

    EXPECT(spline_table_destroy(NULL), BSPL_OK);
    EXPECT(spline_table_info(NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_eval_v(NULL, 1, NULL, NULL, 1, NULL), BSPL_EINVAL);
    EXPECT(spline_eval_vgl(NULL, 1, NULL, NULL, NULL, NULL, 1, NULL), BSPL_EINVAL);
    EXPECT(spline_eval_vgh(NULL, 1, NULL, NULL, NULL, NULL, 1, NULL), BSPL_EINVAL);
    EXPECT(spline_eval(NULL, BSPL_VGH, 1, NULL, NULL, NULL, NULL, 1, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_eval_ratio(NULL, BSPL_VGH, 1, NULL, NULL, 1, NULL, NULL, NULL), BSPL_EINVAL);
    bspl_tile tile;
    EXPECT(spline_tile_select(NULL, BSPL_V, 1, &tile), BSPL_EINVAL);
    EXPECT(spline_autotune(NULL, BSPL_V, 1, NULL, NULL, NULL), BSPL_EINVAL);

    bspl_plan* plan = NULL;
    const bspl_table* tabs[1] = {NULL};
    int64_t npos[1] = {1}, ldo[1] = {1};
    EXPECT(spline_batch_plan_create(NULL, 1, tabs, npos, BSPL_V, NULL, NULL, NULL, NULL, ldo,
                                    NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_plan_create(&plan, 0, tabs, npos, BSPL_V, NULL, NULL, NULL, NULL, ldo,
                                    NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_plan_create(&plan, 17, tabs, npos, BSPL_V, NULL, NULL, NULL, NULL, ldo,
                                    NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_plan_create(&plan, 1, tabs, npos, BSPL_V, NULL, NULL, NULL, NULL, ldo,
                                    NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_plan_destroy(NULL), BSPL_OK);
    EXPECT(spline_batch_execute(NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_launch(NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_rebind(NULL, 0, NULL, NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_batch_plan_tile(NULL, &tile), BSPL_EINVAL);

    bspl_table_info lay;
    int64_t units = 0, wgs = 0;
    int32_t thr = 0;
    bspl_tile t1 = {1, 1, 1, 0, 0, 1}, t8 = {1, 1, 8, 0, 0, 1}, ts = {1, 1, 1, 0, 0, 4};
    EXPECT(spline_layout_query(4, 4, 4, 700, BSPL_F32, 0, &lay), BSPL_OK);
    EXPECT(spline_launch_query(&lay, BSPL_VGH, (int64_t)1 << 31, NULL, &units, &wgs, &thr),
           BSPL_EUNSUPPORTED);
    EXPECT(spline_launch_query(&lay, BSPL_VGH, ((int64_t)1 << 31) - 1, &t1, &units, &wgs, &thr),
           BSPL_EUNSUPPORTED);
    EXPECT(spline_launch_query(&lay, BSPL_VGH, (((int64_t)1 << 31) - 1) / 11, &t8, &units, &wgs,
                               &thr), BSPL_OK);
    if (wgs * thr > 4294967295LL) ++failures;
    EXPECT(spline_launch_query(&lay, BSPL_VGH, 2000000, &ts, NULL, NULL, NULL), BSPL_EUNSUPPORTED);
    EXPECT(spline_launch_query(&lay, BSPL_VGH, 100, NULL, NULL, NULL, NULL), BSPL_OK);
    EXPECT(spline_launch_query(&lay, (bspl_kind)-5, 100, NULL, NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_launch_query(&lay, BSPL_V, -1, NULL, NULL, NULL, NULL), BSPL_EINVAL);
    EXPECT(spline_launch_query(NULL, BSPL_V, 1, NULL, NULL, NULL, NULL), BSPL_EINVAL);
    lay.dtype = 77;
    EXPECT(spline_launch_query(&lay, BSPL_V, 1, NULL, NULL, NULL, NULL), BSPL_EINVAL);

    unsigned layout = 99;
    EXPECT(spline_layout_select(8, 8, 8, 2048, BSPL_F32, BSPL_VGH, 64, NULL, NULL, NULL),
           BSPL_EINVAL);
    EXPECT(spline_layout_select(8, 8, 8, 2048, BSPL_F32, (bspl_kind)9, 64, NULL, &layout, NULL),
           BSPL_EINVAL);
    EXPECT(spline_layout_select(8, 8, 8, 2048, BSPL_F32, BSPL_VGH, 0, NULL, &layout, NULL),
           BSPL_EINVAL);
    EXPECT(spline_layout_select(8, 8, 8, 256, BSPL_F32, BSPL_VGH, 64, NULL, &layout, NULL),
           BSPL_OK);
    if (layout != 0) ++failures;
}

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s scratch_dir\n", argv[0]);
        return 2;
    }
    for (int s = -1; s <= 6; ++s)
        if (!spline_status_string((bspl_status)s) || !spline_last_error()) ++failures;
    layouts();
    wisdom(argv[1]);
    arguments();
    if (failures) {
        fprintf(stderr, "%d unexpected results\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
