/*
 * A C program that uses the SGM library only through include/sgm.h and the
 * HIP runtime API: device buffers from hipMalloc, its own stream, no Python.
 * Every library call is written against the boundary's declarations as the
 * interface lists them - the sgm_item initializers are positional, in the
 * order {w, h, max_disp, n_paths, flags, left, right, out}, and the server is
 * created with (budget, max_slots, P1, P2, census_w, census_h) - so a layout
 * or arity change breaks this program.  Results are checked against the CPU
 * oracle (test infrastructure, linked into this test program only), and the
 * documented error paths are exercised.
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
int oracle_census_full(const uint8_t *img, int W, int H, int cw, int ch, uint64_t *out);
int oracle_cost_volume(const uint64_t *cbase, const uint64_t *cmatch, int W, int H, int D, int cmax,
                       uint8_t *mc);
int oracle_aggregate(const uint8_t *mc, int W, int H, int D, int P1, int P2, int rx, int ry,
                     int32_t *lr_out, uint32_t *sum);
int oracle_direction(int n_paths, int index, int *rx, int *ry);

#define CHECK(cond, msg)                                                                    \
    do {                                                                                    \
        if (!(cond)) {                                                                      \
            fprintf(stderr, "capi_check FAILED: %s (%s)\n", msg, sgm_last_error());         \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

/* oracle flag bits (oracle/sgm_oracle.c) */
#define ORC_MEDIAN 1u
#define ORC_LRCHECK 2u
#define ORC_LRFULL 8u

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

static unsigned oracle_flags(unsigned flags)
{
    return ((flags & SGM_MEDIAN3) ? ORC_MEDIAN : 0u) | ((flags & SGM_LRCHECK) ? ORC_LRCHECK : 0u) |
           ((flags & SGM_LR_FULL) ? ORC_LRFULL : 0u);
}

/* One pair on the device: images in, output buffer, host copies. */
typedef struct {
    int W, H, D, paths;
    unsigned flags;
    uint8_t *hl, *hr;
    uint16_t *want;
    uint8_t *dl, *dr;
    uint16_t *dout;
} pair_t;

static int pair_setup(pair_t *p, int W, int H, int D, int paths, unsigned flags, uint32_t seed)
{
    size_t npx = (size_t)W * H;
    p->W = W; p->H = H; p->D = D; p->paths = paths; p->flags = flags;
    p->hl = (uint8_t *)malloc(npx);
    p->hr = (uint8_t *)malloc(npx);
    p->want = (uint16_t *)malloc(npx * 2);
    make_pair(p->hl, p->hr, W, H, D / 3, seed);
    CHECK(hipMalloc((void **)&p->dl, npx) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&p->dr, npx) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&p->dout, npx * 2) == hipSuccess, "hipMalloc");
    CHECK(hipMemcpy(p->dl, p->hl, npx, hipMemcpyHostToDevice) == hipSuccess, "copy");
    CHECK(hipMemcpy(p->dr, p->hr, npx, hipMemcpyHostToDevice) == hipSuccess, "copy");
    CHECK(oracle_sgm(p->hl, p->hr, W, H, D, 7, 86, paths, 9, 7, oracle_flags(flags), 1, p->want, NULL, NULL, NULL,
                     NULL, NULL) == 0,
          "oracle");
    return 0;
}

static void pair_free(pair_t *p)
{
    (void)hipFree(p->dl);
    (void)hipFree(p->dr);
    (void)hipFree(p->dout);
    free(p->hl); free(p->hr); free(p->want);
}

/* differing pixels between the device output and the oracle */
static long pair_diff(const pair_t *p, const char *what)
{
    size_t npx = (size_t)p->W * p->H;
    uint16_t *got = (uint16_t *)malloc(npx * 2);
    if (hipMemcpy(got, p->dout, npx * 2, hipMemcpyDeviceToHost) != hipSuccess) {
        free(got);
        return -1;
    }
    long bad = 0;
    for (size_t i = 0; i < npx; i++) bad += got[i] != p->want[i];
    printf("%s %dx%d D=%d paths=%d flags=%u: %ld of %zu pixels differ\n", what, p->W, p->H, p->D, p->paths,
           p->flags, bad, npx);
    free(got);
    return bad;
}

static int run_single(int W, int H, int D, int paths, unsigned flags, hipStream_t st)
{
    pair_t p;
    if (pair_setup(&p, W, H, D, paths, flags, 1610u + (uint32_t)W)) return 1;
    sgm_ctx *c = sgm_create(W, H, D, 7, 86, paths, 9, 7);
    CHECK(c != NULL, "sgm_create");
    CHECK(sgm_set_options(c, flags, 1) == SGM_OK, "sgm_set_options");
    CHECK(sgm_compute(c, p.dl, p.dr, p.dout, (sgm_stream_t)st) == SGM_OK, "sgm_compute");
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    sgm_destroy(c);
    long bad = pair_diff(&p, "sgm_compute");
    pair_free(&p);
    return bad != 0;
}

/* The census tap and both phase-sum taps against the oracle's stages. */
static int run_taps(hipStream_t st)
{
    const int W = 61, H = 23, D = 24, P = 4;
    pair_t p;
    if (pair_setup(&p, W, H, D, P, 0, 77u)) return 1;
    size_t npx = (size_t)W * H, ncell = npx * D;
    uint64_t *cl = (uint64_t *)malloc(npx * 8), *cr = (uint64_t *)malloc(npx * 8), *cg = (uint64_t *)malloc(npx * 8);
    uint8_t *mc = (uint8_t *)malloc(ncell);
    uint32_t *s0 = (uint32_t *)calloc(ncell, 4), *s1 = (uint32_t *)calloc(ncell, 4);
    uint16_t *got = (uint16_t *)malloc(ncell * 2);
    oracle_census_full(p.hl, W, H, 9, 7, cl);
    oracle_census_full(p.hr, W, H, 9, 7, cr);
    oracle_cost_volume(cl, cr, W, H, D, 62, mc);
    for (int r = 0; r < P; r++) {
        int rx, ry;
        oracle_direction(P, r, &rx, &ry);
        /* the last direction of the set (right-to-left) joins only phase 1 */
        if (r != 1) oracle_aggregate(mc, W, H, D, 7, 86, rx, ry, NULL, s0);
        oracle_aggregate(mc, W, H, D, 7, 86, rx, ry, NULL, s1);
    }
    sgm_ctx *c = sgm_create(W, H, D, 7, 86, P, 9, 7);
    CHECK(c != NULL, "sgm_create");
    uint64_t *dcen = NULL;
    uint16_t *dsum = NULL;
    CHECK(hipMalloc((void **)&dcen, npx * 8) == hipSuccess, "hipMalloc");
    CHECK(hipMalloc((void **)&dsum, ncell * 2) == hipSuccess, "hipMalloc");
    CHECK(sgm_debug_census(c, p.dl, dcen, (sgm_stream_t)st) == SGM_OK, "sgm_debug_census");
    CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
    CHECK(hipMemcpy(cg, dcen, npx * 8, hipMemcpyDeviceToHost) == hipSuccess, "copy back");
    long bad = 0;
    for (size_t i = 0; i < npx; i++) bad += cg[i] != cl[i];
    for (int phase = 0; phase < 2; phase++) {
        const uint32_t *want = phase ? s1 : s0;
        CHECK(sgm_debug_phase_sums(c, p.dl, p.dr, phase, dsum, (sgm_stream_t)st) == SGM_OK, "sgm_debug_phase_sums");
        CHECK(hipStreamSynchronize(st) == hipSuccess, "sync");
        CHECK(hipMemcpy(got, dsum, ncell * 2, hipMemcpyDeviceToHost) == hipSuccess, "copy back");
        for (size_t i = 0; i < ncell; i++) bad += got[i] != want[i];
    }
    CHECK(sgm_debug_phase_sums(c, p.dl, p.dr, 2, dsum, (sgm_stream_t)st) == SGM_EINVAL, "phase 2 rejected");
    printf("taps %dx%d D=%d: census + 2 phase sums, %ld values differ\n", W, H, D, bad);
    sgm_destroy(c);
    (void)hipFree(dcen);
    (void)hipFree(dsum);
    free(cl); free(cr); free(cg); free(mc); free(s0); free(s1); free(got);
    pair_free(&p);
    return bad != 0;
}

/* sgm_compute_batch over three pairs of different shapes. */
static int run_batch(hipStream_t st)
{
    pair_t p[3];
    if (pair_setup(&p[0], 96, 40, 32, 4, SGM_MEDIAN3 | SGM_LRCHECK, 11u)) return 1;
    if (pair_setup(&p[1], 57, 33, 70, 8, 0, 12u)) return 1;
    if (pair_setup(&p[2], 120, 17, 16, 2, SGM_LRCHECK, 13u)) return 1;
    sgm_item items[3];
    for (int k = 0; k < 3; k++) {
        sgm_item it = {p[k].W, p[k].H, p[k].D, p[k].paths, p[k].flags, p[k].dl, p[k].dr, p[k].dout};
        items[k] = it;
    }
    CHECK(sgm_compute_batch(items, 3, 7, 86, 9, 7, (sgm_stream_t)st) == SGM_OK, "sgm_compute_batch");
    long bad = 0;
    for (int k = 0; k < 3; k++) {
        long b = pair_diff(&p[k], "sgm_compute_batch");
        bad += b < 0 ? 1 : b;
        pair_free(&p[k]);
    }
    return bad != 0;
}

/* A batch runner replaying a captured graph, twice, the second time into
 * freshly cleared outputs. */
static int run_batch_graph(hipStream_t st)
{
    pair_t p[2];
    if (pair_setup(&p[0], 70, 44, 40, 4, SGM_MEDIAN3 | SGM_LRCHECK, 31u)) return 1;
    if (pair_setup(&p[1], 45, 60, 64, 8, SGM_LRCHECK | SGM_LR_FULL, 32u)) return 1;
    sgm_item items[2];
    for (int k = 0; k < 2; k++) {
        sgm_item it = {p[k].W, p[k].H, p[k].D, p[k].paths, p[k].flags, p[k].dl, p[k].dr, p[k].dout};
        items[k] = it;
    }
    sgm_batch *b = sgm_batch_create(7, 86, 9, 7);
    CHECK(b != NULL, "sgm_batch_create");
    CHECK(sgm_batch_set_graph(b, 2) == SGM_EINVAL, "graph flag out of range");
    CHECK(sgm_batch_set_graph(b, 1) == SGM_OK, "sgm_batch_set_graph");
    long bad = 0;
    for (int rep = 0; rep < 2; rep++) {
        for (int k = 0; k < 2; k++)
            CHECK(hipMemsetAsync(p[k].dout, 0xAB, (size_t)p[k].W * p[k].H * 2, st) == hipSuccess, "clear");
        CHECK(sgm_batch_compute(b, items, 2, (sgm_stream_t)st) == SGM_OK, "sgm_batch_compute (graph)");
        for (int k = 0; k < 2; k++) {
            long d = pair_diff(&p[k], "sgm_batch_compute (graph)");
            bad += d < 0 ? 1 : d;
        }
    }
    sgm_batch_destroy(b);
    for (int k = 0; k < 2; k++) pair_free(&p[k]);
    return bad != 0;
}

/* A server with two slots: two requests, waited for by polling. */
static int run_server(void)
{
    pair_t p[2];
    if (pair_setup(&p[0], 80, 48, 48, 8, SGM_MEDIAN3 | SGM_LRCHECK, 21u)) return 1;
    if (pair_setup(&p[1], 33, 70, 20, 4, SGM_MEDIAN3, 22u)) return 1;
    sgm_server *s = sgm_server_create((size_t)256 << 20, 2, 7, 86, 9, 7);
    CHECK(s != NULL, "sgm_server_create");
    uint64_t ticket[2];
    for (int k = 0; k < 2; k++) {
        sgm_item req = {p[k].W, p[k].H, p[k].D, p[k].paths, p[k].flags, p[k].dl, p[k].dr, p[k].dout};
        CHECK(sgm_server_submit(s, &req, &ticket[k]) == SGM_OK, "sgm_server_submit");
    }
    long bad = 0;
    for (int k = 0; k < 2; k++) {
        int status = SGM_REQ_QUEUED;
        double lat = 0.0;
        for (long spins = 0; status != SGM_REQ_DONE; spins++) {
            CHECK(spins < 2000000000L, "request never finished");
            CHECK(sgm_server_poll(s, ticket[k], &status, &lat) == SGM_OK, "sgm_server_poll");
            CHECK(status != SGM_REQ_FAILED && status != SGM_REQ_CANCELED, "request failed");
        }
        CHECK(lat > 0.0, "latency");
        long b = pair_diff(&p[k], "sgm_server");
        bad += b < 0 ? 1 : b;
    }
    sgm_server_destroy(s);
    for (int k = 0; k < 2; k++) pair_free(&p[k]);
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
    CHECK(sgm_footprint_bytes(640, 480, 128, 4, 0) > (size_t)640 * 480 * 128 * 5, "footprint");
    CHECK(sgm_footprint_bytes(640, 480, 300, 4, 0) == 0, "footprint of an invalid shape");
    sgm_ctx *c = sgm_create(32, 16, 8, 7, 86, 4, 9, 7);
    CHECK(c != NULL, "create");
    CHECK(sgm_compute(c, NULL, NULL, NULL, (sgm_stream_t)st) == SGM_EINVAL, "null buffers");
    CHECK(sgm_set_options(c, 1u << 30, 1) == SGM_EINVAL, "unknown flag");
    sgm_destroy(c);
    sgm_destroy(NULL);
    CHECK(sgm_server_create(1 << 20, 0, 7, 86, 9, 7) == NULL, "server with no slot");
    sgm_server_destroy(NULL);
    /* a forced allocation failure: no context, a message, then recovery */
    sgm_debug_fail_alloc(0, 1);
    CHECK(sgm_create(32, 16, 8, 7, 86, 4, 9, 7) == NULL && strlen(sgm_last_error()) > 0, "forced failure");
    sgm_debug_fail_alloc(0, 0);
    c = sgm_create(32, 16, 8, 7, 86, 4, 9, 7);
    CHECK(c != NULL, "create after the forced failure");
    sgm_destroy(c);

    int fails = 0;
    fails += run_single(160, 90, 48, 4, 0, st);
    fails += run_single(200, 120, 64, 8, SGM_MEDIAN3 | SGM_LRCHECK, st);
    fails += run_single(97, 31, 20, 2, SGM_LRCHECK, st);
    fails += run_taps(st);
    fails += run_batch(st);
    fails += run_batch_graph(st);
    fails += run_server();
    CHECK(hipStreamDestroy(st) == hipSuccess, "hipStreamDestroy");
    if (fails) {
        fprintf(stderr, "capi_check FAILED: %d case(s) differ from the oracle\n", fails);
        return 1;
    }
    printf("capi_check OK\n");
    return 0;
}
