/*
 * Plain C use of the library, with no Python and no PyTorch: build a table
 * from host coefficients, evaluate VGH at host positions copied to the
 * device, and write the outputs back to a file.  Then the same evaluation
 * on a spline-blocked copy of the table, and a batch plan over both tables
 * replayed as a graph and issued as plain launches, each compared byte for
 * byte with the first result.
 *
 *   c_abi_demo nx ny nz n npos coef.bin pos.bin out.bin
 *
 * coef.bin: float32 [nx][ny][nz][n]; pos.bin: float64 [3][npos];
 * out.bin:  float32 v [npos][n], then g [npos][3][n], then h [npos][6][n].
 * Exit status 0 on success, 4 if a comparison fails; every library failure
 * is printed with spline_last_error().
 */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "bspline.h"

static void* read_file(const char* path, size_t bytes)
{
    FILE* f = fopen(path, "rb");
    if (!f) return NULL;
    void* p = malloc(bytes);
    if (p && fread(p, 1, bytes, f) != bytes) {
        free(p);
        p = NULL;
    }
    fclose(f);
    return p;
}

#define CHECK_HIP(call)                                                    \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) {                                            \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));     \
            return 2;                                                      \
        }                                                                  \
    } while (0)

#define CHECK_BSPL(call)                                                   \
    do {                                                                   \
        bspl_status s_ = (call);                                           \
        if (s_ != BSPL_OK) {                                               \
            fprintf(stderr, "%s: %s (%s)\n", #call, spline_status_string(s_), \
                    spline_last_error());                                  \
            return 3;                                                      \
        }                                                                  \
    } while (0)

int main(int argc, char** argv)
{
    if (argc != 9) {
        fprintf(stderr, "usage: %s nx ny nz n npos coef.bin pos.bin out.bin\n", argv[0]);
        return 1;
    }
    const int nx = atoi(argv[1]), ny = atoi(argv[2]), nz = atoi(argv[3]);
    const int64_t n = atoll(argv[4]), npos = atoll(argv[5]);
    if (nx <= 0 || ny <= 0 || nz <= 0 || n <= 0 || npos <= 0) return 1;
    const size_t ncoef = (size_t)nx * ny * nz * n;
    float* coef = (float*)read_file(argv[6], ncoef * sizeof(float));
    double* pos = (double*)read_file(argv[7], 3 * (size_t)npos * sizeof(double));
    if (!coef || !pos) {
        fprintf(stderr, "cannot read the input files\n");
        return 1;
    }

    bspl_table* table = NULL;
    CHECK_BSPL(spline_table_create(&table, nx, ny, nz, n, coef, BSPL_F32, NULL, 0, NULL));
    bspl_table_info info;
    CHECK_BSPL(spline_table_info(table, &info));
    printf("table %d x %d x %d, N = %lld, %lld bytes on the device\n", info.nx, info.ny,
           info.nz, (long long)info.n_splines, (long long)info.table_bytes);

    const size_t out_elems = (size_t)npos * 10 * n;  /* v + 3 g + 6 h */
    double* d_pos = NULL;
    float* d_out = NULL;
    CHECK_HIP(hipMalloc((void**)&d_pos, 3 * (size_t)npos * sizeof(double)));
    CHECK_HIP(hipMalloc((void**)&d_out, out_elems * sizeof(float)));
    CHECK_HIP(hipMemcpy(d_pos, pos, 3 * (size_t)npos * sizeof(double), hipMemcpyHostToDevice));
    float* d_v = d_out;
    float* d_g = d_v + (size_t)npos * n;
    float* d_h = d_g + (size_t)npos * 3 * n;
    CHECK_BSPL(spline_eval_vgh(table, npos, d_pos, d_v, d_g, d_h, n, NULL));
    CHECK_HIP(hipDeviceSynchronize());

    float* out = (float*)malloc(out_elems * sizeof(float));
    float* again = (float*)malloc(out_elems * sizeof(float));
    if (!out || !again) return 1;
    CHECK_HIP(hipMemcpy(out, d_out, out_elems * sizeof(float), hipMemcpyDeviceToHost));

    /* the spline-blocked layout gives the same bytes */
    bspl_table* blocked = NULL;
    CHECK_BSPL(spline_table_create(&blocked, nx, ny, nz, n, coef, BSPL_F32, NULL,
                                   BSPL_LAYOUT_BLOCKED, NULL));
    bspl_tile tile; /* the decomposition the first evaluation used */
    CHECK_BSPL(spline_tile_select(table, BSPL_VGH, npos, &tile));
    CHECK_HIP(hipMemset(d_out, 0, out_elems * sizeof(float)));
    CHECK_BSPL(spline_eval(blocked, BSPL_VGH, npos, d_pos, d_v, d_g, d_h, n, &tile, NULL));
    CHECK_HIP(hipMemcpy(again, d_out, out_elems * sizeof(float), hipMemcpyDeviceToHost));
    if (memcmp(out, again, out_elems * sizeof(float)) != 0) {
        fprintf(stderr, "the spline-blocked table gave different outputs\n");
        return 4;
    }
    printf("spline-blocked table: identical outputs\n");

    /* one plan over both tables: the second table writes a second buffer */
    float* d_out2 = NULL;
    CHECK_HIP(hipMalloc((void**)&d_out2, out_elems * sizeof(float)));
    const bspl_table* tabs[2] = {table, blocked};
    const int64_t np2[2] = {npos, npos}, ld2[2] = {n, n};
    const double* pos2[2] = {d_pos, d_pos};
    float* v2[2] = {d_v, d_out2};
    float* g2[2] = {d_g, d_out2 + (size_t)npos * n};
    float* h2[2] = {d_h, d_out2 + (size_t)npos * 4 * n};
    bspl_plan* plan = NULL;
    CHECK_BSPL(spline_batch_plan_create(&plan, 2, tabs, np2, BSPL_VGH, pos2, v2, g2, h2, ld2,
                                        tile.split > 1 ? NULL : &tile, NULL, NULL));
    for (int mode = 0; mode < 2; ++mode) {
        CHECK_HIP(hipMemset(d_out, 0, out_elems * sizeof(float)));
        CHECK_HIP(hipMemset(d_out2, 0, out_elems * sizeof(float)));
        if (mode == 0)
            CHECK_BSPL(spline_batch_execute(plan, NULL));
        else
            CHECK_BSPL(spline_batch_launch(plan, NULL));
        CHECK_HIP(hipDeviceSynchronize());
        for (int b = 0; b < 2; ++b) {
            CHECK_HIP(hipMemcpy(again, b == 0 ? d_out : d_out2, out_elems * sizeof(float),
                                hipMemcpyDeviceToHost));
            if (memcmp(out, again, out_elems * sizeof(float)) != 0) {
                fprintf(stderr, "plan %s, table %d: outputs differ\n",
                        mode == 0 ? "graph replay" : "direct launch", b);
                return 4;
            }
        }
    }
    printf("batch plan over both tables (graph replay and direct launch): identical outputs\n");
    CHECK_BSPL(spline_batch_plan_destroy(plan));
    CHECK_BSPL(spline_table_destroy(blocked));
    CHECK_HIP(hipFree(d_out2));
    free(again);
    FILE* f = fopen(argv[8], "wb");
    if (!f || fwrite(out, sizeof(float), out_elems, f) != out_elems) {
        fprintf(stderr, "cannot write %s\n", argv[8]);
        return 1;
    }
    fclose(f);

    CHECK_BSPL(spline_table_destroy(table));
    CHECK_HIP(hipFree(d_pos));
    CHECK_HIP(hipFree(d_out));
    free(out);
    free(coef);
    free(pos);
    printf("ok: %lld positions evaluated\n", (long long)npos);
    return 0;
}
