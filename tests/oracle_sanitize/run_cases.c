/* Runs the C oracle's whole pipeline on cases read from stdin and writes each
 * output map to stdout.  Built with AddressSanitizer and UndefinedBehavior-
 * Sanitizer by tests/test_oracle_sanitized.py (CPU only), which compares the
 * outputs with the regular build's.
 *
 * Input, per case: ten little-endian int32 (W, H, D, P1, P2, n_paths, cw, ch,
 * flags, lr_thr), then the left and right images (u8 [H][W] each).
 * Output, per case: the int32 return code, then u16 [H][W] (only if 0). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_sgm(const uint8_t *left, const uint8_t *right, int W, int H, int D, int P1, int P2,
               int n_paths, int cw, int ch, unsigned flags, int lr_thr, uint16_t *out,
               uint64_t *census_l, uint64_t *census_r, uint32_t *S_out, uint16_t *dl_raw,
               uint16_t *dr_raw);

int main(void)
{
    int32_t hdr[10];
    while (fread(hdr, sizeof hdr, 1, stdin) == 1) {
        const int W = hdr[0], H = hdr[1];
        if (W < 1 || H < 1 || W > 4096 || H > 4096) return 2;
        const size_t npx = (size_t)W * H;
        uint8_t *l = malloc(npx), *r = malloc(npx);
        uint16_t *out = malloc(npx * 2);
        if (!l || !r || !out) return 3;
        if (fread(l, 1, npx, stdin) != npx || fread(r, 1, npx, stdin) != npx) return 4;
        /* the optional outputs are requested, so their code paths run too */
        uint64_t *cl = malloc(npx * 8), *cr = malloc(npx * 8);
        uint32_t *S = malloc(npx * (size_t)hdr[2] * 4);
        uint16_t *dl = malloc(npx * 2), *dr = malloc(npx * 2);
        if (!cl || !cr || !S || !dl || !dr) return 3;
        int32_t rc = oracle_sgm(l, r, W, H, hdr[2], hdr[3], hdr[4], hdr[5], hdr[6], hdr[7], (unsigned)hdr[8],
                                hdr[9], out, cl, cr, S, dl, dr);
        fwrite(&rc, sizeof rc, 1, stdout);
        if (rc == 0) fwrite(out, 2, npx, stdout);
        free(l); free(r); free(out); free(cl); free(cr); free(S); free(dl); free(dr);
    }
    return 0;
}
