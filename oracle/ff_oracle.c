/*
 * ff_oracle.c -- plain single-threaded CPU oracle of the Flow Fields search.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  The
 * HIP library never links or calls this file, and the two share no code.
 *
 * The method (FlowFields++, Sec. 3.1 "Matches"): matching cost is a distance
 * between feature descriptors; initial matches come from Walsh-Hadamard
 * descriptors matched at the lowest resolution; propagation then spreads them
 * in four directions, several iterations per pyramid level from coarse to
 * fine, and a random search perturbs both flow components slightly after
 * each of an iteration's last three propagation steps; a forward-backward
 * consistency check with threshold epsilon (Table 3: epsilon = 1 for KITTI)
 * removes outliers.
 *
 * The paper leaves the exact arithmetic to the Flow Fields papers it cites.
 * The readings taken here (integer luma, 2x2 box pyramid, K = 16 sequency
 * ordered Walsh-Hadamard coefficients, SAD cost, exact seed search, scanline
 * sweeps, Philox-driven random search with halving radius, squared-Euclidean
 * consistency test) are each stated at the function that implements them.
 * Every step is written in the order the schedule runs it, with no blocking,
 * fusion or reordering, so it can be checked against that schedule by eye.
 */
#include "ff_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- gray -- */
/* Sec. 3.1 uses all CIELab channels; the integer reading is BT.601 luma with
 * 8-bit weights that sum to 256, rounded half up.  C = 1 passes through.   */
void ffo_gray(const uint8_t* img, int W, int H, int C, uint8_t* gray)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const uint8_t* p = img + ((size_t)y * W + x) * C;
            if (C == 1) {
                gray[(size_t)y * W + x] = p[0];
            } else {
                int v = (77 * p[0] + 150 * p[1] + 29 * p[2] + 128) >> 8;
                gray[(size_t)y * W + x] = (uint8_t)v;
            }
        }
}

/* ------------------------------------------------------------- pyramid -- */
/* The scales of the coarse-to-fine search (Sec. 3.1): factor-2 levels,
 * 2x2 box mean rounded half up, odd trailing row/column dropped.          */
void ffo_down2(const uint8_t* src, int W, int H, uint8_t* dst)
{
    int w = W >> 1, h = H >> 1;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            int s = src[(size_t)(2 * y) * W + 2 * x] + src[(size_t)(2 * y) * W + 2 * x + 1]
                  + src[(size_t)(2 * y + 1) * W + 2 * x] + src[(size_t)(2 * y + 1) * W + 2 * x + 1];
            dst[(size_t)y * w + x] = (uint8_t)((s + 2) >> 2);
        }
}

/* --------------------------------------------------------- descriptors -- */
/* Walsh-Hadamard descriptors (Sec. 3.1, initialisation).  The 1-D Walsh
 * functions on 8 samples in sequency order (number of sign changes 0..3):
 *   w0 = + + + + + + + +      w1 = + + + + - - - -
 *   w2 = + + - - - - + +      w3 = + + - - + + - -
 * The 2-D basis is W_uv(r, c) = w_u(r) w_v(c), u, v in 0..3, k = 4u + v.
 * The patch at (x, y) covers columns x-3..x+4 and rows y-3..y+4 with
 * coordinates clamped to the image (replicated border).                   */
static const int WALSH8[4][8] = {
    {+1, +1, +1, +1, +1, +1, +1, +1},
    {+1, +1, +1, +1, -1, -1, -1, -1},
    {+1, +1, -1, -1, -1, -1, +1, +1},
    {+1, +1, -1, -1, +1, +1, -1, -1},
};

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Floor division by 64 for any sign (the arithmetic shift the quantiser
 * reading uses), written without relying on >> of negative numbers.      */
static int floor_div64(int v) { return v >= 0 ? v / 64 : -((-v + 63) / 64); }
static int floor_div(int v, int d) { return v >= 0 ? v / d : -((-v + d - 1) / d); }

void ffo_descriptors(const uint8_t* P, int W, int H, int8_t* D)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int patch[8][8];
            for (int r = 0; r < 8; ++r)
                for (int c = 0; c < 8; ++c)
                    patch[r][c] = P[(size_t)clampi(y - 3 + r, 0, H - 1) * W + clampi(x - 3 + c, 0, W - 1)];
            int8_t* d = D + ((size_t)y * W + x) * FFO_K;
            for (int u = 0; u < 4; ++u)
                for (int v = 0; v < 4; ++v) {
                    int s = 0;
                    for (int r = 0; r < 8; ++r)
                        for (int c = 0; c < 8; ++c)
                            s += WALSH8[u][r] * WALSH8[v][c] * patch[r][c];
                    /* Quantise: floor(c / 64).  DC in 0..255 is shifted to
                     * int8 by -128; AC lies in [-8160, 8160] -> [-128, 127]. */
                    int q = floor_div64(s);
                    if (u == 0 && v == 0) q -= 128;
                    d[4 * u + v] = (int8_t)q;
                }
        }
}

/* ---------------------------------------------------------------- cost -- */
/* Matching cost: distance between descriptors (Sec. 3.1), read as the sum
 * of absolute differences of the 16 int8 coefficients.  A flow that leaves
 * image B has no cost: INF, never accepted by any comparison.             */
int32_t ffo_cost(const int8_t* DA, const int8_t* DB, int W, int H, int x, int y, int fx, int fy)
{
    int qx = x + fx, qy = y + fy;
    if (qx < 0 || qx >= W || qy < 0 || qy >= H) return FFO_INF;
    const int8_t* a = DA + ((size_t)y * W + x) * FFO_K;
    const int8_t* b = DB + ((size_t)qy * W + qx) * FFO_K;
    int32_t s = 0;
    for (int k = 0; k < FFO_K; ++k) s += abs((int)a[k] - (int)b[k]);
    return s;
}

/* ------------------------------------------------------------- Census --- */
/* The alternative matching cost of Sec. 3.1: the Hamming distance of the
 * binary patterns of the Census transform over a 7x7 patch (Zabih and
 * Woodfill).  Reading: on the luma plane (as every other step here), patch
 * centred on the pixel, border replicated, bit set when the neighbour is
 * strictly darker than the centre, neighbours in row-major order.          */
void ffo_census(const uint8_t* P, int W, int H, uint64_t* out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int c = P[(size_t)y * W + x];
            uint64_t bits = 0;
            int k = 0;
            for (int dy = -3; dy <= 3; ++dy)
                for (int dx = -3; dx <= 3; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    int v = P[(size_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
                    if (v < c) bits |= (uint64_t)1 << k;
                    ++k;
                }
            out[(size_t)y * W + x] = bits;
        }
}

int32_t ffo_cost_census(const uint64_t* CA, const uint64_t* CB, int W, int H, int x, int y, int fx, int fy)
{
    int qx = x + fx, qy = y + fy;
    if (qx < 0 || qx >= W || qy < 0 || qy >= H) return FFO_INF;
    uint64_t d = CA[(size_t)y * W + x] ^ CB[(size_t)qy * W + qx];
    int32_t n = 0;
    while (d) {
        n += (int32_t)(d & 1u);
        d >>= 1;
    }
    return n;
}

/* ---------------------------------------------------------- sub-pixel --- */
/* Sub-pixel matching (Sec. 3.1: sub-pixel locations are interpolated
 * bilinearly).  Reading: a refinement at level 0 on flows in quarter pixels;
 * the cost of a quarter-pixel target interpolates B's biased descriptor
 * bytes with integer bilinear weights and rounds half up, then takes the
 * SAD.  The 2x2 neighbour with zero weight is not read.                    */
int32_t ffo_cost_subpix(const int8_t* DA, const int8_t* DB, int W, int H, int x, int y, int u, int v)
{
    int tx = 4 * x + u, ty = 4 * y + v;
    if (tx < 0 || ty < 0) return FFO_INF;
    int ix = tx / 4, iy = ty / 4, ax = tx % 4, ay = ty % 4;
    if (ix > W - 1 || iy > H - 1 || (ix == W - 1 && ax != 0) || (iy == H - 1 && ay != 0)) return FFO_INF;
    int ix1 = ax ? ix + 1 : ix, iy1 = ay ? iy + 1 : iy;
    const int8_t* a = DA + ((size_t)y * W + x) * FFO_K;
    const int8_t* b00 = DB + ((size_t)iy * W + ix) * FFO_K;
    const int8_t* b10 = DB + ((size_t)iy * W + ix1) * FFO_K;
    const int8_t* b01 = DB + ((size_t)iy1 * W + ix) * FFO_K;
    const int8_t* b11 = DB + ((size_t)iy1 * W + ix1) * FFO_K;
    int w00 = (4 - ax) * (4 - ay), w10 = ax * (4 - ay), w01 = (4 - ax) * ay, w11 = ax * ay;
    int32_t s = 0;
    for (int k = 0; k < FFO_K; ++k) {
        int i = (w00 * (b00[k] + 128) + w10 * (b10[k] + 128) + w01 * (b01[k] + 128) + w11 * (b11[k] + 128) + 8) >> 4;
        s += abs(a[k] + 128 - i);
    }
    return s;
}

/* A level's matching-cost plane of one image: the descriptors (SAD, or the
 * sub-pixel SAD on quarter-pixel flows) or the Census strings (Hamming), as
 * params.cost_kind selects.                                                 */
typedef struct {
    int kind;
    const int8_t* desc;
    const uint64_t* cen;
} cplane;

static int32_t plane_cost(const cplane* A, const cplane* B, int W, int H, int x, int y, int fx, int fy)
{
    if (A->kind == FFO_COST_CENSUS) return ffo_cost_census(A->cen, B->cen, W, H, x, y, fx, fy);
    if (A->kind == FFO_COST_SUBPIX) return ffo_cost_subpix(A->desc, B->desc, W, H, x, y, fx, fy);
    return ffo_cost(A->desc, B->desc, W, H, x, y, fx, fy);
}

/* ------------------------------------------------------------ seed NN --- */
/* Initial matches at the lowest resolution (Sec. 3.1).  The paper matches
 * the Walsh-Hadamard descriptors with kd-trees; the reading here is the
 * exact answer a kd-tree approximates: for every seed s on the stride grid
 * of A, the pixel q of B with the smallest squared Euclidean descriptor
 * distance, the lowest linear index y*W+x on ties.                         */
void ffo_seed_nn(const int8_t* DA, const int8_t* DB, int W, int H, int stride, int32_t* idx)
{
    int nsx = (W + stride - 1) / stride, nsy = (H + stride - 1) / stride;
    for (int j = 0; j < nsy; ++j)
        for (int i = 0; i < nsx; ++i) {
            const int8_t* a = DA + ((size_t)(j * stride) * W + i * stride) * FFO_K;
            int32_t best = INT32_MAX, arg = -1;
            for (int q = 0; q < W * H; ++q) {
                const int8_t* b = DB + (size_t)q * FFO_K;
                int32_t d = 0;
                for (int k = 0; k < FFO_K; ++k) {
                    int t = (int)a[k] - (int)b[k];
                    d += t * t;
                }
                if (d < best) { best = d; arg = q; }
            }
            idx[j * nsx + i] = arg;
        }
}

int32_t ffo_nearest(const int8_t* a, const int8_t* DB, int N)
{
    int32_t best = INT32_MAX, arg = -1;
    for (int q = 0; q < N; ++q) {
        const int8_t* b = DB + (size_t)q * FFO_K;
        int32_t d = 0;
        for (int k = 0; k < FFO_K; ++k) {
            int t = (int)a[k] - (int)b[k];
            d += t * t;
        }
        if (d < best) { best = d; arg = q; }
    }
    return arg;
}

/* -------------------------------------------------------------- Philox -- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of a 4-word S-P network.  A round
 * multiplies words 0 and 2 by the Philox constants, takes the 64-bit
 * products' halves and xors the high halves with words 1 and 3 and the key;
 * the key is advanced by the Weyl constants between rounds.                */
void ffo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* --------------------------------------------------------- propagation -- */
/* Propagation in four directions (Sec. 3.1), read as four scanline
 * sweeps per iteration.  Within a sweep, pixels are visited in scan order;
 * each pixel compares its own flow with the flow its predecessor on the
 * line holds after that predecessor was visited, and takes the
 * predecessor's flow only if its cost is strictly lower.                   */
static void sweep_planes(const cplane* A, const cplane* B, int W, int H, int dir_code,
                         int16_t* flow, int32_t* cost)
{
    int horizontal = (dir_code == 0 || dir_code == 1);
    int lines = horizontal ? H : W;
    int len = horizontal ? W : H;
    for (int line = 0; line < lines; ++line) {
        for (int s = 1; s < len; ++s) {
            int x, y, px, py;          /* pixel and its predecessor */
            if (dir_code == 0)      { y = line; x = s;           px = x - 1; py = y; }
            else if (dir_code == 1) { y = line; x = len - 1 - s; px = x + 1; py = y; }
            else if (dir_code == 2) { x = line; y = s;           px = x; py = y - 1; }
            else                    { x = line; y = len - 1 - s; px = x; py = y + 1; }
            size_t p = (size_t)y * W + x, q = (size_t)py * W + px;
            int gx = flow[2 * q], gy = flow[2 * q + 1];
            int32_t e = plane_cost(A, B, W, H, x, y, gx, gy);
            if (e < cost[p]) {
                flow[2 * p] = (int16_t)gx;
                flow[2 * p + 1] = (int16_t)gy;
                cost[p] = e;
            }
        }
    }
}

void ffo_sweep(const int8_t* DA, const int8_t* DB, int W, int H, int dir_code,
               int16_t* flow, int32_t* cost)
{
    cplane A = {FFO_COST_WH, DA, NULL}, B = {FFO_COST_WH, DB, NULL};
    sweep_planes(&A, &B, W, H, dir_code, flow, cost);
}

void ffo_sweep_census(const uint64_t* CA, const uint64_t* CB, int W, int H, int dir_code,
                      int16_t* flow, int32_t* cost)
{
    cplane A = {FFO_COST_CENSUS, NULL, CA}, B = {FFO_COST_CENSUS, NULL, CB};
    sweep_planes(&A, &B, W, H, dir_code, flow, cost);
}

/* ------------------------------------------------------- random search -- */
/* Random search (Sec. 3.1): both flow components are perturbed by a small
 * random amount.  Reading: per pixel, J = floor(log2 R) + 1 trials with radius
 * r_j = R >> j around the flow v0 the pixel held before the pass; offsets
 * are uniform integers in [-r_j, r_j] (taken as u mod (2 r_j + 1) - r_j of
 * a Philox word); a trial replaces the current best only when its flow
 * differs from the best flow and its cost is strictly lower.  The Philox
 * counter is (y*W + x, level, (iter << 2) | pass, j >> 1) and the key is
 * the 64-bit seed split into (low, high) words; trial j uses words (0, 1)
 * when j is even and (2, 3) when j is odd.                                 */
static void random_search_planes(const cplane* A, const cplane* B, int W, int H, int level,
                                 int iter, int pass, int radius, uint64_t seed,
                                 int16_t* flow, int32_t* cost)
{
    int J = 0;
    while ((radius >> J) > 0) ++J;                 /* floor(log2 R) + 1 */
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            int v0x = flow[2 * p], v0y = flow[2 * p + 1];
            int bx = v0x, by = v0y;
            int32_t bc = cost[p];
            uint32_t u[4] = {0, 0, 0, 0};
            for (int j = 0; j < J; ++j) {
                int r = radius >> j;
                if ((j & 1) == 0) {
                    uint32_t ctr[4] = {(uint32_t)(y * W + x), (uint32_t)level,
                                       ((uint32_t)iter << 2) | (uint32_t)pass, (uint32_t)(j >> 1)};
                    ffo_philox4x32_10(ctr, key, u);
                }
                uint32_t ux = (j & 1) ? u[2] : u[0];
                uint32_t uy = (j & 1) ? u[3] : u[1];
                uint32_t span = 2u * (uint32_t)r + 1u;
                int dx = (int)(ux % span) - r;
                int dy = (int)(uy % span) - r;
                int cx = v0x + dx, cy = v0y + dy;
                if (cx == bx && cy == by) continue;
                int32_t c = plane_cost(A, B, W, H, x, y, cx, cy);
                if (c < bc) { bx = cx; by = cy; bc = c; }
            }
            flow[2 * p] = (int16_t)bx;
            flow[2 * p + 1] = (int16_t)by;
            cost[p] = bc;
        }
}

void ffo_random_search(const int8_t* DA, const int8_t* DB, int W, int H, int level,
                       int iter, int pass, int radius, uint64_t seed,
                       int16_t* flow, int32_t* cost)
{
    cplane A = {FFO_COST_WH, DA, NULL}, B = {FFO_COST_WH, DB, NULL};
    random_search_planes(&A, &B, W, H, level, iter, pass, radius, seed, flow, cost);
}

void ffo_random_search_census(const uint64_t* CA, const uint64_t* CB, int W, int H, int level,
                              int iter, int pass, int radius, uint64_t seed,
                              int16_t* flow, int32_t* cost)
{
    cplane A = {FFO_COST_CENSUS, NULL, CA}, B = {FFO_COST_CENSUS, NULL, CB};
    random_search_planes(&A, &B, W, H, level, iter, pass, radius, seed, flow, cost);
}

void ffo_sweep_subpix(const int8_t* DA, const int8_t* DB, int W, int H, int dir_code, int16_t* flow, int32_t* cost)
{
    cplane A = {FFO_COST_SUBPIX, DA, NULL}, B = {FFO_COST_SUBPIX, DB, NULL};
    sweep_planes(&A, &B, W, H, dir_code, flow, cost);
}

void ffo_random_search_subpix(const int8_t* DA, const int8_t* DB, int W, int H, int level, int iter, int pass,
                              int radius, uint64_t seed, int16_t* flow, int32_t* cost)
{
    cplane A = {FFO_COST_SUBPIX, DA, NULL}, B = {FFO_COST_SUBPIX, DB, NULL};
    random_search_planes(&A, &B, W, H, level, iter, pass, radius, seed, flow, cost);
}

/* --------------------------------------------------------- full search -- */
typedef struct {
    int W, H;
    uint8_t* pyr[2];       /* gray level of image 1 and image 2 */
    int8_t* desc[2];       /* descriptors of image 1 and image 2 */
    uint64_t* cen[2];      /* Census strings (cost_kind = FFO_COST_CENSUS)  */
} level_t;

static void trace_call(ffo_trace_fn trace, void* user, int dir, int level, int iter, int stage,
                       int W, int H, const int16_t* flow, const int32_t* cost)
{
    if (trace) trace(user, dir, level, iter, stage, W, H, flow, cost);
}

/* Coarse-to-fine search of one direction: A is the reference image, B the
 * image searched.  Writes the level-0 flow and cost.                        */
static void search_direction(const ffo_params* p, const level_t* lv, int ia, int ib, int dir,
                             int16_t* flow0, int32_t* cost0, ffo_trace_fn trace, void* user)
{
    int L = p->levels;
    int16_t* flow = NULL;
    int32_t* cost = NULL;
    int pw = 0, ph = 0;
    for (int l = L - 1; l >= 0; --l) {
        int W = lv[l].W, H = lv[l].H;
        const int8_t* DA = lv[l].desc[ia];
        const int8_t* DB = lv[l].desc[ib];
        /* seeds always match descriptors; every other cost uses the plane  */
        const cplane A = {p->cost_kind, DA, lv[l].cen[ia]}, B = {p->cost_kind, DB, lv[l].cen[ib]};
        int16_t* nflow = (l == 0) ? flow0 : (int16_t*)malloc(sizeof(int16_t) * 2 * (size_t)W * H);
        int32_t* ncost = (l == 0) ? cost0 : (int32_t*)malloc(sizeof(int32_t) * (size_t)W * H);
        if (l == L - 1) {
            /* Initialisation at the lowest resolution: exact seed matches,
             * each pixel takes the flow of the seed of its stride cell.     */
            int st = p->seed_stride;
            int nsx = (W + st - 1) / st, nsy = (H + st - 1) / st;
            int32_t* idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)nsx * nsy);
            ffo_seed_nn(DA, DB, W, H, st, idx);
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    int si = x / st, sj = y / st;
                    int q = idx[sj * nsx + si];
                    int fx = (q % W) - si * st, fy = (q / W) - sj * st;
                    size_t pp = (size_t)y * W + x;
                    nflow[2 * pp] = (int16_t)fx;
                    nflow[2 * pp + 1] = (int16_t)fy;
                    ncost[pp] = plane_cost(&A, &B, W, H, x, y, fx, fy);
                }
            free(idx);
        } else {
            /* Next finer scale: twice the coarse flow of the parent pixel
             * (nearest, clamped to the coarse grid), re-costed.            */
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    int cx = clampi(x >> 1, 0, pw - 1), cy = clampi(y >> 1, 0, ph - 1);
                    size_t cp = (size_t)cy * pw + cx, pp = (size_t)y * W + x;
                    int fx = 2 * flow[2 * cp], fy = 2 * flow[2 * cp + 1];
                    nflow[2 * pp] = (int16_t)fx;
                    nflow[2 * pp + 1] = (int16_t)fy;
                    ncost[pp] = plane_cost(&A, &B, W, H, x, y, fx, fy);
                }
            free(flow);
            free(cost);
        }
        flow = nflow;
        cost = ncost;
        pw = W;
        ph = H;
        trace_call(trace, user, dir, l, -1, 0, W, H, flow, cost);
        for (int t = 0; t < p->iters; ++t) {
            sweep_planes(&A, &B, W, H, 0, flow, cost);
            trace_call(trace, user, dir, l, t, 1, W, H, flow, cost);
            sweep_planes(&A, &B, W, H, 1, flow, cost);
            trace_call(trace, user, dir, l, t, 2, W, H, flow, cost);
            random_search_planes(&A, &B, W, H, l, t, 0, p->rs_radius, p->seed, flow, cost);
            trace_call(trace, user, dir, l, t, 3, W, H, flow, cost);
            sweep_planes(&A, &B, W, H, 2, flow, cost);
            trace_call(trace, user, dir, l, t, 4, W, H, flow, cost);
            random_search_planes(&A, &B, W, H, l, t, 1, p->rs_radius, p->seed, flow, cost);
            trace_call(trace, user, dir, l, t, 5, W, H, flow, cost);
            sweep_planes(&A, &B, W, H, 3, flow, cost);
            trace_call(trace, user, dir, l, t, 6, W, H, flow, cost);
            random_search_planes(&A, &B, W, H, l, t, 2, p->rs_radius, p->seed, flow, cost);
            trace_call(trace, user, dir, l, t, 7, W, H, flow, cost);
        }
    }
    if (p->sub_iters > 0) {
        /* Sub-pixel refinement at level 0 (Sec. 3.1): flows to quarter
         * pixels (costs unchanged: zero fraction), then sub_iters times the
         * same schedule with the interpolated cost; random search radius in
         * quarter pixels, Philox level index = number of pyramid levels.  */
        int W = lv[0].W, H = lv[0].H;
        for (size_t q = 0; q < (size_t)W * H; ++q) {
            flow[2 * q] = (int16_t)(4 * flow[2 * q]);
            flow[2 * q + 1] = (int16_t)(4 * flow[2 * q + 1]);
        }
        const cplane A = {FFO_COST_SUBPIX, lv[0].desc[ia], NULL}, B = {FFO_COST_SUBPIX, lv[0].desc[ib], NULL};
        trace_call(trace, user, dir, L, -1, 0, W, H, flow, cost);
        for (int t = 0; t < p->sub_iters; ++t) {
            sweep_planes(&A, &B, W, H, 0, flow, cost);
            trace_call(trace, user, dir, L, t, 1, W, H, flow, cost);
            sweep_planes(&A, &B, W, H, 1, flow, cost);
            trace_call(trace, user, dir, L, t, 2, W, H, flow, cost);
            random_search_planes(&A, &B, W, H, L, t, 0, p->sub_radius, p->seed, flow, cost);
            trace_call(trace, user, dir, L, t, 3, W, H, flow, cost);
            sweep_planes(&A, &B, W, H, 2, flow, cost);
            trace_call(trace, user, dir, L, t, 4, W, H, flow, cost);
            random_search_planes(&A, &B, W, H, L, t, 1, p->sub_radius, p->seed, flow, cost);
            trace_call(trace, user, dir, L, t, 5, W, H, flow, cost);
            sweep_planes(&A, &B, W, H, 3, flow, cost);
            trace_call(trace, user, dir, L, t, 6, W, H, flow, cost);
            random_search_planes(&A, &B, W, H, L, t, 2, p->sub_radius, p->seed, flow, cost);
            trace_call(trace, user, dir, L, t, 7, W, H, flow, cost);
        }
    }
}

/* Forward-backward consistency check (Sec. 3.1; threshold epsilon, Table 3):
 * p is kept when its own match and the match of its target q = p + F(p) are
 * both valid and the round trip F(p) + B(q) has squared length <= eps^2.   */
static void consistency(int W, int H, int eps, const int16_t* F, const int32_t* cF,
                        const int16_t* B, const int32_t* cB, uint8_t* mask)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            uint8_t m = 0;
            if (cF[p] != FFO_INF) {
                int qx = x + F[2 * p], qy = y + F[2 * p + 1];
                size_t q = (size_t)qy * W + qx;
                if (cB[q] != FFO_INF) {
                    int ex = F[2 * p] + B[2 * q], ey = F[2 * p + 1] + B[2 * q + 1];
                    m = (ex * ex + ey * ey <= eps * eps) ? 1 : 0;
                }
            }
            mask[p] = m;
        }
}

/* Consistency error (Sec. 3.1), the quantity the mask thresholds, for
 * flows in 1/unit pixels: q = p + F(p) rounded half up to whole pixels (an
 * identity for unit 1), error |F(p) + B(q)|^2 in 1/unit^2 px^2.          */
void ffo_fb_error_u(int W, int H, int unit, const int16_t* F, const int32_t* cF,
                    const int16_t* B, const int32_t* cB, int32_t* err)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            int32_t e = FFO_INF;
            if (cF[p] != FFO_INF) {
                int qx = x + floor_div(F[2 * p] + unit / 2, unit), qy = y + floor_div(F[2 * p + 1] + unit / 2, unit);
                size_t q = (size_t)qy * W + qx;
                if (cB[q] != FFO_INF) {
                    int ex = F[2 * p] + B[2 * q], ey = F[2 * p + 1] + B[2 * q + 1];
                    e = ex * ex + ey * ey;
                }
            }
            err[p] = e;
        }
}

void ffo_fb_error(int W, int H, const int16_t* F, const int32_t* cF,
                  const int16_t* B, const int32_t* cB, int32_t* err)
{
    ffo_fb_error_u(W, H, 1, F, cF, B, cB, err);
}

/* Two consistency checks (Sec. 3.1): the larger of the two errors.       */
void ffo_fb_error2_u(int W, int H, int unit, const int16_t* F, const int32_t* cF, const int16_t* B1,
                     const int32_t* cB1, const int16_t* B2, const int32_t* cB2, int32_t* err)
{
    int32_t* e2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)W * H);
    ffo_fb_error_u(W, H, unit, F, cF, B1, cB1, err);
    ffo_fb_error_u(W, H, unit, F, cF, B2, cB2, e2);
    for (size_t p = 0; p < (size_t)W * H; ++p)
        if (e2[p] > err[p]) err[p] = e2[p];
    free(e2);
}

void ffo_fb_error2(int W, int H, const int16_t* F, const int32_t* cF, const int16_t* B1, const int32_t* cB1,
                   const int16_t* B2, const int32_t* cB2, int32_t* err)
{
    ffo_fb_error2_u(W, H, 1, F, cF, B1, cB1, B2, cB2, err);
}

/* Sparsification (Sec. 3.1, s from Table 3): one kept match per 3x3 block
 * holding at least s consistent matches -- the lowest consistency error,
 * scanning the block in row-major order so the first minimum is the lowest
 * linear index.                                                           */
void ffo_sparsify(int W, int H, const uint8_t* mask, const int32_t* err, int s, uint8_t* keep)
{
    for (size_t p = 0; p < (size_t)W * H; ++p) keep[p] = 0;
    for (int by = 0; by < H; by += 3)
        for (int bx = 0; bx < W; bx += 3) {
            int count = 0;
            size_t best = 0;
            int32_t best_e = FFO_INF;
            for (int y = by; y < by + 3 && y < H; ++y)
                for (int x = bx; x < bx + 3 && x < W; ++x) {
                    size_t p = (size_t)y * W + x;
                    if (!mask[p]) continue;
                    ++count;
                    if (count == 1 || err[p] < best_e) {
                        best_e = err[p];
                        best = p;
                    }
                }
            if (count >= s) keep[best] = 1;
        }
}

int ffo_match(const ffo_params* p, const uint8_t* img1, const uint8_t* img2,
              int W, int H, int C,
              int16_t* flow_f, int32_t* cost_f, uint8_t* mask_f,
              int16_t* flow_b, int32_t* cost_b, uint8_t* mask_b,
              ffo_trace_fn trace, void* user)
{
    if (!p || !img1 || !img2 || !flow_f || !mask_f) return -1;
    if (C != 1 && C != 3) return -1;
    if (p->levels < 1 || p->levels > 16 || p->seed_stride < 1 || p->iters < 0 ||
        p->rs_radius < 0 || p->fb_eps < 0 || (p->cost_kind != FFO_COST_WH && p->cost_kind != FFO_COST_CENSUS))
        return -1;
    if (p->sub_iters < 0 || (p->sub_iters > 0 && (p->cost_kind != FFO_COST_WH || p->sub_radius < 0 || W > 2048 || H > 2048)))
        return -1;
    if (p->second_params && (p->iters2 < 0 || p->rs_radius2 < 0)) return -1;
    if (W < 1 || H < 1 || (W >> (p->levels - 1)) < 1 || (H >> (p->levels - 1)) < 1) return -1;

    int L = p->levels;
    level_t* lv = (level_t*)calloc((size_t)L, sizeof(level_t));
    const uint8_t* imgs[2] = {img1, img2};
    for (int i = 0; i < 2; ++i) {
        lv[0].W = W;
        lv[0].H = H;
        lv[0].pyr[i] = (uint8_t*)malloc((size_t)W * H);
        ffo_gray(imgs[i], W, H, C, lv[0].pyr[i]);
        for (int l = 1; l < L; ++l) {
            lv[l].W = lv[l - 1].W >> 1;
            lv[l].H = lv[l - 1].H >> 1;
            lv[l].pyr[i] = (uint8_t*)malloc((size_t)lv[l].W * lv[l].H);
            ffo_down2(lv[l - 1].pyr[i], lv[l - 1].W, lv[l - 1].H, lv[l].pyr[i]);
        }
        for (int l = 0; l < L; ++l) {
            lv[l].desc[i] = (int8_t*)malloc((size_t)lv[l].W * lv[l].H * FFO_K);
            ffo_descriptors(lv[l].pyr[i], lv[l].W, lv[l].H, lv[l].desc[i]);
            if (p->cost_kind == FFO_COST_CENSUS) {
                lv[l].cen[i] = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)lv[l].W * lv[l].H);
                ffo_census(lv[l].pyr[i], lv[l].W, lv[l].H, lv[l].cen[i]);
            }
        }
    }

    int32_t* cf = cost_f ? cost_f : (int32_t*)malloc(sizeof(int32_t) * (size_t)W * H);
    int16_t* fb = flow_b ? flow_b : (int16_t*)malloc(sizeof(int16_t) * 2 * (size_t)W * H);
    int32_t* cb = cost_b ? cost_b : (int32_t*)malloc(sizeof(int32_t) * (size_t)W * H);

    /* forward: reference image 1, searched image 2; backward: swapped */
    search_direction(p, lv, 0, 1, 0, flow_f, cf, trace, user);
    search_direction(p, lv, 1, 0, 1, fb, cb, trace, user);

    const int unit = p->sub_iters > 0 ? 4 : 1;          /* flows in quarter pixels after refinement */
    const int eps2 = p->fb_eps * p->fb_eps * unit * unit;
    if (!p->two_checks && unit == 1) {
        consistency(W, H, p->fb_eps, flow_f, cf, fb, cb, mask_f);
        if (mask_b) consistency(W, H, p->fb_eps, fb, cb, flow_f, cf, mask_b);
    } else if (!p->two_checks) {
        int32_t* e = (int32_t*)malloc(sizeof(int32_t) * (size_t)W * H);
        ffo_fb_error_u(W, H, unit, flow_f, cf, fb, cb, e);
        for (size_t q = 0; q < (size_t)W * H; ++q) mask_f[q] = e[q] <= eps2 ? 1 : 0;
        if (mask_b) {
            ffo_fb_error_u(W, H, unit, fb, cb, flow_f, cf, e);
            for (size_t q = 0; q < (size_t)W * H; ++q) mask_b[q] = e[q] <= eps2 ? 1 : 0;
        }
        free(e);
    } else {
        /* second pair of fields: the same search keyed by seed2; a match
         * must be consistent with both inverse fields (Sec. 3.1)          */
        ffo_params p2 = *p;
        p2.seed = p->seed2;
        if (p->second_params) {          /* other matching parameters too */
            p2.iters = p->iters2;
            p2.rs_radius = p->rs_radius2;
        }
        size_t n = (size_t)W * H;
        int16_t* f2 = (int16_t*)malloc(sizeof(int16_t) * 2 * n);
        int16_t* b2 = (int16_t*)malloc(sizeof(int16_t) * 2 * n);
        int32_t* cf2 = (int32_t*)malloc(sizeof(int32_t) * n);
        int32_t* cb2 = (int32_t*)malloc(sizeof(int32_t) * n);
        int32_t* e = (int32_t*)malloc(sizeof(int32_t) * n);
        search_direction(&p2, lv, 0, 1, 0, f2, cf2, NULL, NULL);
        search_direction(&p2, lv, 1, 0, 1, b2, cb2, NULL, NULL);
        ffo_fb_error2_u(W, H, unit, flow_f, cf, fb, cb, b2, cb2, e);
        for (size_t q = 0; q < n; ++q) mask_f[q] = e[q] <= eps2 ? 1 : 0;
        if (mask_b) {
            ffo_fb_error2_u(W, H, unit, fb, cb, flow_f, cf, f2, cf2, e);
            for (size_t q = 0; q < n; ++q) mask_b[q] = e[q] <= eps2 ? 1 : 0;
        }
        free(f2); free(b2); free(cf2); free(cb2); free(e);
    }

    if (!cost_f) free(cf);
    if (!flow_b) free(fb);
    if (!cost_b) free(cb);
    for (int l = 0; l < L; ++l)
        for (int i = 0; i < 2; ++i) {
            free(lv[l].pyr[i]);
            free(lv[l].desc[i]);
            free(lv[l].cen[i]);
        }
    free(lv);
    return 0;
}
