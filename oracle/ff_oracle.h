/*
 * ff_oracle.h -- CPU oracle of the Flow Fields dense correspondence search
 * (FlowFields++, Sec. 3.1 "Matches"): descriptors, seed initialisation at the
 * lowest resolution, coarse-to-fine propagation with random search, and the
 * forward-backward consistency check.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded reference
 * used by the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark.  The product path (the HIP library) never links, loads or calls
 * it, and it shares no code, header or table with that library.
 *
 * All arithmetic is integer; every output is defined exactly, so the HIP path
 * must reproduce it bit for bit.
 */
#ifndef FF_ORACLE_H
#define FF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFO_INF INT32_MAX
#define FFO_K   16          /* descriptor length */

typedef struct {
    int32_t  levels;        /* pyramid levels L >= 1                         */
    int32_t  seed_stride;   /* seed grid step at the coarsest level (3)      */
    int32_t  iters;         /* propagation iterations T per level (2)        */
    int32_t  rs_radius;     /* random-search radius R (16): R, R>>1, ..., 1   */
    int32_t  fb_eps;        /* consistency threshold epsilon in px (1)       */
    uint64_t seed;          /* random-search key                             */
    int32_t  cost_kind;     /* FFO_COST_WH (0) or FFO_COST_CENSUS (1)         */
    int32_t  two_checks;    /* 1: masks need a second check against the
                               inverse fields of a search keyed by seed2      */
    uint64_t seed2;         /* random-search key of the second search        */
    int32_t  sub_iters;     /* > 0: sub-pixel refinement iterations at level 0
                               (flows, errors and eps then in quarter pixels;
                               descriptor cost only)                          */
    int32_t  sub_radius;    /* its random-search radius in quarter pixels      */
    int32_t  second_params; /* with two_checks: 1 = the second search runs
                               iters2 iterations per level at random-search
                               radius rs_radius2 (0 = the first search's)    */
    int32_t  iters2;
    int32_t  rs_radius2;
} ffo_params;

#define FFO_COST_WH     0   /* SAD of the 16 Walsh-Hadamard coefficients     */
#define FFO_COST_CENSUS 1   /* Hamming distance of 7x7 Census bit strings    */
#define FFO_COST_SUBPIX 2   /* SAD against bilinearly interpolated descriptors,
                               flows in quarter pixels (refinement only)      */

/* Trace hook: called after every stage with the direction's state.
 * stage: 0 = level init, 1 = LR, 2 = RL, 3 = RS0, 4 = TB, 5 = RS1, 6 = BT,
 * 7 = RS2.  flow is [H][W][2] int16 (dx, dy), cost is [H][W] int32.        */
typedef void (*ffo_trace_fn)(void* user, int dir, int level, int iter, int stage,
                             int W, int H, const int16_t* flow, const int32_t* cost);

/* Sec. 3.1 input: colour to gray, Y = (77 R + 150 G + 29 B + 128) >> 8.  */
void ffo_gray(const uint8_t* img, int W, int H, int C, uint8_t* gray);
/* One 2x2 box-filter pyramid step, rounding half up, floor dimensions.  */
void ffo_down2(const uint8_t* src, int W, int H, uint8_t* dst);
/* 16 Walsh-Hadamard coefficients of the 8x8 patch at every pixel, int8.  */
void ffo_descriptors(const uint8_t* P, int W, int H, int8_t* D);
/* Exact nearest neighbour of every seed (stride grid) of A among all pixels
 * of B, squared L2 over the descriptors, ties to the lowest linear index.
 * idx has ceil(H/stride) * ceil(W/stride) entries, seed-row-major.       */
void ffo_seed_nn(const int8_t* DA, const int8_t* DB, int W, int H, int stride, int32_t* idx);
/* The same search for one query descriptor a against the N descriptors of
 * DB: index of the first minimum of the squared L2 distance.  Lets a test
 * check single seeds of a plane too large to search whole.               */
int32_t ffo_nearest(const int8_t* a, const int8_t* DB, int N);
/* 7x7 Census transform (Sec. 3.1; Zabih and Woodfill): bit k, for the k-th
 * of the 48 neighbours (dx, dy) in [-3, 3]^2 other than the centre taken in
 * row-major order (dy outer, dx inner), is 1 when the neighbour is strictly
 * darker than the centre; border replicated.  out is [H][W].              */
void ffo_census(const uint8_t* P, int W, int H, uint64_t* out);
/* Sub-pixel cost (Sec. 3.1, bilinear interpolation): (u, v) in quarter
 * pixels; the target (4x + u, 4y + v) must lie in [0, 4(W-1)] x [0, 4(H-1)];
 * B's biased coefficients (d + 128) are interpolated from the 2x2
 * neighbourhood with integer weights (4-ax)(4-ay), ax(4-ay), (4-ax)ay, ax ay
 * (ax, ay = fraction in quarters), rounded half up ((sum + 8) >> 4); SAD
 * against A's biased coefficients.  Zero fraction = the integer cost.     */
int32_t ffo_cost_subpix(const int8_t* DA, const int8_t* DB, int W, int H, int x, int y, int u, int v);
/* Census matching cost: Hamming distance (0..48), INF outside image B.   */
int32_t ffo_cost_census(const uint64_t* CA, const uint64_t* CB, int W, int H, int x, int y, int fx, int fy);
/* Philox4x32 with 10 rounds (Salmon et al., SC'11).                        */
void ffo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Matching cost: SAD of the two descriptors, INF when p+f leaves image B.  */
int32_t ffo_cost(const int8_t* DA, const int8_t* DB, int W, int H, int x, int y, int fx, int fy);
/* One directional sweep over the whole state of one level.
 * dir_code: 0 = LR, 1 = RL, 2 = TB, 3 = BT.  flow/cost updated in place.   */
void ffo_sweep(const int8_t* DA, const int8_t* DB, int W, int H, int dir_code,
               int16_t* flow, int32_t* cost);
/* One random-search pass over every pixel of one level.                    */
void ffo_random_search(const int8_t* DA, const int8_t* DB, int W, int H, int level,
                       int iter, int pass, int radius, uint64_t seed,
                       int16_t* flow, int32_t* cost);
/* The same two steps with the Census cost (planes from ffo_census).       */
void ffo_sweep_census(const uint64_t* CA, const uint64_t* CB, int W, int H, int dir_code,
                      int16_t* flow, int32_t* cost);
void ffo_random_search_census(const uint64_t* CA, const uint64_t* CB, int W, int H, int level,
                              int iter, int pass, int radius, uint64_t seed,
                              int16_t* flow, int32_t* cost);

/* Full search for one pair.  img1/img2 are [H][W][C] uint8, C in {1, 3}.
 * flow_* [H][W][2] int16, cost_* [H][W] int32, mask_* [H][W] uint8.
 * The backward outputs may be NULL.  Returns 0, or -1 on invalid input.   */
int ffo_match(const ffo_params* p, const uint8_t* img1, const uint8_t* img2,
              int W, int H, int C,
              int16_t* flow_f, int32_t* cost_f, uint8_t* mask_f,
              int16_t* flow_b, int32_t* cost_b, uint8_t* mask_b,
              ffo_trace_fn trace, void* user);

/* Consistency error of every pixel p (Sec. 3.1): with q = p + F(p), the
 * squared length |F(p) + B(q)|^2 when both matches are valid (finite cost),
 * FFO_INF otherwise.  The consistency mask is exactly err <= eps^2.       */
void ffo_fb_error(int W, int H, const int16_t* F, const int32_t* cF,
                  const int16_t* B, const int32_t* cB, int32_t* err);
/* The same for flows in 1/unit pixels (unit 1 or 4): q = p + F(p) rounded
 * half up to whole pixels, error in 1/unit^2 px^2.                         */
void ffo_fb_error_u(int W, int H, int unit, const int16_t* F, const int32_t* cF,
                    const int16_t* B, const int32_t* cB, int32_t* err);

/* Two consistency checks (Sec. 3.1): F against two inverse fields B1 and B2,
 * the second matched with other parameters.  err = the larger of the two
 * errors (FFO_INF when either is); a match passes both checks exactly when
 * err <= eps^2.                                                            */
void ffo_fb_error2(int W, int H, const int16_t* F, const int32_t* cF, const int16_t* B1, const int32_t* cB1,
                   const int16_t* B2, const int32_t* cB2, int32_t* err);
void ffo_fb_error2_u(int W, int H, int unit, const int16_t* F, const int32_t* cF, const int16_t* B1,
                     const int32_t* cB1, const int16_t* B2, const int32_t* cB2, int32_t* err);
/* The refinement's two steps on quarter-pixel flows (level index `level`
 * in the Philox counter is the number of pyramid levels).                 */
void ffo_sweep_subpix(const int8_t* DA, const int8_t* DB, int W, int H, int dir_code, int16_t* flow, int32_t* cost);
void ffo_random_search_subpix(const int8_t* DA, const int8_t* DB, int W, int H, int level, int iter, int pass,
                              int radius, uint64_t seed, int16_t* flow, int32_t* cost);

/* Sparsification (Sec. 3.1; minimum matches s from Table 3): the image is
 * cut into 3x3 blocks from the origin, the last column and row of blocks
 * partial when W or H is not a multiple of 3.  A block that holds at least
 * s consistent matches (mask = 1) keeps the one with the lowest consistency
 * error, the lowest y*W + x among equals; every other pixel is dropped.
 * keep is [H][W], 1 = kept match.                                         */
void ffo_sparsify(int W, int H, const uint8_t* mask, const int32_t* err, int s, uint8_t* keep);

#ifdef __cplusplus
}
#endif
#endif
