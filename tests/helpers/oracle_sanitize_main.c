/* Host-only driver for the sanitizer run of the CPU oracle: the test builds
 * ff_oracle.c together with this file under AddressSanitizer and
 * UndefinedBehaviorSanitizer (any report aborts), runs one whole search and
 * the consistency-error and sparsification functions on a pair, and writes
 * every output so the test can compare them with the ordinary build.
 *
 * usage: oracle_sanitize_main IN OUT
 * IN : int32 W, H, C, levels, stride, iters, radius, eps, cost_kind,
 *      two_checks, sub_iters, sub_radius, sparse_s; uint64 seed, seed2;
 *      img1, img2 ([H][W][C] uint8 each)
 * OUT: flow_f, cost_f, mask_f, flow_b, cost_b, mask_b, err_f, keep_f    */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "ff_oracle.h"

static void* must(size_t n)
{
    void* p = malloc(n ? n : 1);
    if (!p) exit(3);
    return p;
}

int main(int argc, char** argv)
{
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t h[13];
    uint64_t seeds[2];
    if (fread(h, sizeof h, 1, f) != 1 || fread(seeds, sizeof seeds, 1, f) != 1) return 2;
    const int W = h[0], H = h[1], C = h[2];
    const size_t n = (size_t)W * H, nb = n * (size_t)C;
    uint8_t* i1 = (uint8_t*)must(nb);
    uint8_t* i2 = (uint8_t*)must(nb);
    if (fread(i1, 1, nb, f) != nb || fread(i2, 1, nb, f) != nb) return 2;
    fclose(f);
    ffo_params p;
    p.levels = h[3];
    p.seed_stride = h[4];
    p.iters = h[5];
    p.rs_radius = h[6];
    p.fb_eps = h[7];
    p.cost_kind = h[8];
    p.two_checks = h[9];
    p.sub_iters = h[10];
    p.sub_radius = h[11];
    p.seed = seeds[0];
    p.seed2 = seeds[1];
    int16_t* ff = (int16_t*)must(4 * n);
    int16_t* fbw = (int16_t*)must(4 * n);
    int32_t* cf = (int32_t*)must(4 * n);
    int32_t* cb = (int32_t*)must(4 * n);
    uint8_t* mf = (uint8_t*)must(n);
    uint8_t* mb = (uint8_t*)must(n);
    int32_t* ef = (int32_t*)must(4 * n);
    uint8_t* kf = (uint8_t*)must(n);
    if (ffo_match(&p, i1, i2, W, H, C, ff, cf, mf, fbw, cb, mb, NULL, NULL) != 0) return 4;
    ffo_fb_error_u(W, H, p.sub_iters > 0 ? 4 : 1, ff, cf, fbw, cb, ef);
    ffo_sparsify(W, H, mf, ef, h[12], kf);
    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    fwrite(ff, 4, n, o);
    fwrite(cf, 4, n, o);
    fwrite(mf, 1, n, o);
    fwrite(fbw, 4, n, o);
    fwrite(cb, 4, n, o);
    fwrite(mb, 1, n, o);
    fwrite(ef, 4, n, o);
    fwrite(kf, 1, n, o);
    fclose(o);
    free(i1); free(i2); free(ff); free(fbw); free(cf); free(cb); free(mf); free(mb); free(ef); free(kf);
    return 0;
}
