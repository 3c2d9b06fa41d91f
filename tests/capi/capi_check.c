/*
 * A C program that uses the SGM library only through include/sgm.h and the
 * HIP runtime API: device buffers from hipMalloc, its own stream, no Python.
 * It checks the disparities against the CPU oracle (test infrastructure,
 * linked into this test program only) and the documented error paths.
 * Exit status 0 and "capi_check OK" on success.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sgm.h"

int oracle_sgm(const uint8_t *left, const uint8_t *right, int W, int H, int D, int P1, int P2,
               int n_paths, int cw, int ch, unsigned flags, int lr_thr, uint16_t *out,
               uint64_t *census_l, uint64_t *census_r, uint32_t *S_out, uint16_t *dl_raw,
               uint16_t *dr_raw);

#define CHECK(cond, msg)                                                  \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "capi_check FAILED: %s (%s)\n", msg, sgm_last_error()); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

/* a blurred-noise pair shifted by `s` pixels, from a 32-bit LCG */
static void make_pair(uint8_t *l, uint8_t *r, int W, int H, int s, uint32_t seed)
{
    int Wb = W + s + 2, Hb = H + 2;
    uint8_t *noise = (uint8_t *)malloc((size_t)Wb * Hb);
    for (int i = 0; i < Wb * Hb; i++) {
        seed = seed * 1664525u + 1013904223u;
        noise[i] = (uint8_t)(seed >> 24);
    }
    for (int y = 0; y < H; y++)
        for (int x = 0; x < W + s; x++) {
            int acc = 0;
            for (int j = 0; j < 3; j++)
                for (int i = 0; i < 3; i++) acc += noise[(y + j) * Wb + x + i];
            uint8_t v = (uint8_t)((acc + 4) / 9);
            if (x < W) l[y * W + x] = v;
            if (x >= s) r[y * W + x - s] = v;
        }
    free(noise);
}

static int run_case(int W, int H, int D, int paths, unsigned flags, hipStream_t st)
{
    size_t npx = (size_t)W * H;
    uint8_t *hl = (uint8_t *)malloc(npx), *hr = (uint8_t *)malloc(npx);
    uint16_t *got = (uint16_t *)malloc(npx * 2), *want = (uint16_t *)malloc(npx * 2);
    make_pair(hl, hr, W, H, D / 3, 1610u + (uint32_t)W);

    uint8_t *dl = NULL, *dr = NULL;
    uint16_t *dout = NULL;
    CHECK(hipMalloc((void **)&dl, npx) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&dr, npx) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&dout, npx * 2) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(dl, hl, npx, hipMemcpyHostToDevice) == hipSuccess, "copy");
    CHECK(hipMemcpy(dr, hr, npx, hipMemcpyHostToDevice) == hipSuccess, "copy");

    sgm_ctx *c = sgm_create(W, H, D, 7, 86, paths, 9, 7);
    CHECK(c != NULL, "sgm_create");
    CHECK(sgm_set_options(c, flags, 1) == SGM_OK, "sgm_set_options");
    CHECK(sgm_compute(c, dl, dr, dout, (sgm_stream_t)st) == SGM_OK, "sgm_compute");
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    CHECK(hipMemcpy(got, dout, npx * 2, hipMemcpyDeviceToHost) == hipSuccess, "copy back");
    sgm_destroy(c);

    unsigned oflags = ((flags & SGM_MEDIAN3) ? 1u : 0u) | ((flags & SGM_LRCHECK) ? 2u : 0u);
    CHECK(oracle_sgm(hl, hr, W, H, D, 7, 86, paths, 9, 7, oflags, 1, want, NULL, NULL, NULL, NULL, NULL) == 0,
          "oracle");
    size_t bad = 0;
    for (size_t i = 0; i < npx; i++) bad += got[i] != want[i];
    printf("case %dx%d D=%d paths=%d flags=%u: %zu of %zu pixels differ\n", W, H, D, paths, flags, bad, npx);
    (void)hipFree(dl);
    (void)hipFree(dr);
    (void)hipFree(dout);
    free(hl); free(hr); free(got); free(want);
    return bad != 0;
}

int main(void)
{
    int n = 0;
    CHECK(hipGetDeviceCount(&n) == hipSuccess && n > 0, "no HIP device");
    hipStream_t st;
    CHECK(hipStreamCreate(&st) == hipSuccess, "hipStreamCreate");

    /* documented error paths: nothing is enqueued, a message is left */
    CHECK(sgm_create(0, 10, 8, 7, 86, 4, 9, 7) == NULL && strlen(sgm_last_error()) > 0, "invalid create");
    CHECK(sgm_validate(64, 48, 300, 7, 86, 4, 9, 7, 0) == SGM_EINVAL, "validate D");
    sgm_ctx *c = sgm_create(32, 16, 8, 7, 86, 4, 9, 7);
    CHECK(c != NULL, "create");
    CHECK(sgm_compute(c, NULL, NULL, NULL, (sgm_stream_t)st) == SGM_EINVAL, "null buffers");
    CHECK(sgm_set_options(c, 1u << 30, 1) == SGM_EINVAL, "unknown flag");
    sgm_destroy(c);
    sgm_destroy(NULL);

    int fails = 0;
    fails += run_case(160, 90, 48, 4, 0, st);
    fails += run_case(200, 120, 64, 8, SGM_MEDIAN3 | SGM_LRCHECK, st);
    fails += run_case(97, 31, 20, 2, SGM_LRCHECK, st);
    CHECK(hipStreamDestroy(st) == hipSuccess, "hipStreamDestroy");
    if (fails) {
        fprintf(stderr, "capi_check FAILED: %d case(s) differ from the oracle\n", fails);
        return 1;
    }
    printf("capi_check OK\n");
    return 0;
}
