// ff_kernels.hip -- gfx950 kernels of the Flow Fields search (FlowFields++,
// Sec. 3.1 "Matches").  Every kernel is grouped over a batch: blockIdx.y (or
// .z) selects the pair and the image or direction, the other grid axes cover
// the largest level of the batch and blocks beyond a pair's own size exit
// (the per-pixel kernels cap that axis for batches of many small pairs and
// stride over the image; the line phases of uneven batches run a work list).
//
// All arithmetic is integer and follows the schedule stated in include/ff.h;
// the parallel forms used here (windowed relaxation of the scanline sweeps,
// all random-search trials gathered before the sequential selection, MFMA
// scoring of the seed search) reproduce that schedule's result exactly.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "ff_internal.h"

namespace ff {

typedef int v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ helpers ---
__device__ __forceinline__ uint32_t pack_flow(int fx, int fy)
{
    return (uint32_t)(uint16_t)fx | ((uint32_t)(uint16_t)fy << 16);
}
__device__ __forceinline__ int flow_x(uint32_t f) { return (int)(int16_t)(f & 0xFFFFu); }
__device__ __forceinline__ int flow_y(uint32_t f) { return (int)(int16_t)(f >> 16); }

// Global-address-space pointers.  Buffer pointers arrive through the
// per-pair table as generic pointers; converting the base pointer once makes
// every access below a global_load / global_store instead of a flat one.
#define FF_GLOBAL __attribute__((address_space(1)))
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef FF_GLOBAL const uint8_t gcu8;
typedef FF_GLOBAL const u32x4 gcu4;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef FF_GLOBAL const u32x2 gcu2;
typedef FF_GLOBAL i32x2 gi2;

// One line's search state in LDS between a phase's passes: flows as u32 and
// costs as u16 in two planes (6 bytes a pixel instead of 8, so more lines fit
// per CU).  Every finite cost fits: SAD of 16 bytes <= 4080, Hamming <= 48;
// INF is stored as 0xFFFF.  Pixels below hi are held here; a long row keeps
// its last windows (p >= hi) in global memory instead, so that LDS does not
// cap the number of waves per CU -- the first pass writes them last and the
// second pass (right to left) reads them first, while they are still in L2.
struct LdsLine {
    __attribute__((address_space(3))) uint32_t* f;
    __attribute__((address_space(3))) uint16_t* c;
    int hi;
    __device__ __forceinline__ bool has(int p) const { return p < hi; }
    __device__ __forceinline__ i32x2 get(int p) const
    {
        const uint32_t cc = c[p];
        return i32x2{(int)f[p], cc == 0xFFFFu ? kInf : (int)cc};
    }
    __device__ __forceinline__ void set(int p, i32x2 v) const
    {
        f[p] = (uint32_t)v.x;
        c[p] = (uint16_t)(v.y == kInf ? 0xFFFFu : (uint32_t)v.y);
    }
};

__device__ __forceinline__ uint4 ld16(gcu8* p)
{
    const u32x4 v = *(gcu4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}

// SAD of two 16-byte descriptors held biased (unsigned) -- four v_sad_u8.
__device__ __forceinline__ int32_t sad16(uint4 a, uint4 b)
{
    uint32_t s = __builtin_amdgcn_sad_u8(a.x, b.x, 0u);
    s = __builtin_amdgcn_sad_u8(a.y, b.y, s);
    s = __builtin_amdgcn_sad_u8(a.z, b.z, s);
    s = __builtin_amdgcn_sad_u8(a.w, b.w, s);
    return (int32_t)s;
}

// Blocks are dispatched to the 8 XCDs round-robin by linear block id; the
// remap gives each XCD a contiguous range of logical blocks.  Line phases:
// the lines of one pair and direction (which gather from the same descriptor
// plane) run on one XCD and share its L2.  Tiled kernels: neighbouring tiles
// run on one XCD, so the cache lines their edges share are completed in one
// L2 before they are written back.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Logical (x, y, z) block of a 3-D grid under xcd_remap.
__device__ __forceinline__ int3 xcd_block3()
{
    const int nxy = gridDim.x * gridDim.y;
    const int lb = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y + nxy * blockIdx.z, nxy * gridDim.z);
    const int z = lb / nxy, r = lb - z * nxy;
    return make_int3(r % gridDim.x, r / gridDim.x, z);
}

// Index of pixel (x, y) in a row-major feature plane whose rows are CS
// entries apart (CS = the level's Wp), or in a column-major one whose
// columns are CS entries apart (CS = the level's Hp): W or H rounded up so
// that every line of the plane starts on a 128-byte line.
template <bool COL>
__device__ __forceinline__ size_t pix(int x, int y, int CS)
{
    return COL ? (size_t)x * CS + y : (size_t)y * CS + x;
}

__device__ __forceinline__ uint4 load_desc(gcu8* __restrict__ D, size_t idx)
{
    return ld16(D + idx * 16);
}

// The two matching features of Sec. 3.1 the search can run on: the 16
// Walsh-Hadamard coefficients (biased bytes; cost = SAD, four v_sad_u8) or
// the 48-bit 7x7 Census string (cost = Hamming distance, two v_bcnt).
template <int CK> struct Feat;
template <> struct Feat<0> {
    using T = uint4;
    __device__ static T load(gcu8* __restrict__ base, size_t idx) { return ld16(base + idx * 16); }
    __device__ static T zero() { return make_uint4(0, 0, 0, 0); }
    __device__ static int32_t dist(T a, T b) { return sad16(a, b); }
};
template <> struct Feat<1> {
    using T = uint2;
    __device__ static T load(gcu8* __restrict__ base, size_t idx)
    {
        const u32x2 v = *(gcu2*)(base + idx * 8);
        return make_uint2(v.x, v.y);
    }
    __device__ static T zero() { return make_uint2(0, 0); }
    __device__ static int32_t dist(T a, T b) { return (int32_t)(__popc(a.x ^ b.x) + __popc(a.y ^ b.y)); }
};

// Sub-pixel refinement (Sec. 3.1): flows in quarter pixels, own feature =
// the pixel's descriptor; the cost is computed by subpix_cost below.
template <> struct Feat<2> {
    using T = uint4;
    __device__ static T load(gcu8* __restrict__ base, size_t idx) { return ld16(base + idx * 16); }
    __device__ static T zero() { return make_uint4(0, 0, 0, 0); }
};

// Bilinear interpolation of one word of four biased descriptor bytes with
// integer weights summing to 16, rounded half up: even and odd bytes as
// 16-bit lanes (each lane's sum <= 16 * 255 + 8, so 32-bit arithmetic on the
// packed pairs never carries between lanes).
__device__ __forceinline__ uint32_t bilerp_word(uint32_t b00, uint32_t b10, uint32_t b01, uint32_t b11, uint32_t w00,
                                                uint32_t w10, uint32_t w01, uint32_t w11)
{
    const uint32_t m = 0x00FF00FFu;
    const uint32_t ev = (b00 & m) * w00 + (b10 & m) * w10 + (b01 & m) * w01 + (b11 & m) * w11 + 0x00080008u;
    const uint32_t od = ((b00 >> 8) & m) * w00 + ((b10 >> 8) & m) * w10 + ((b01 >> 8) & m) * w01 +
                        ((b11 >> 8) & m) * w11 + 0x00080008u;
    return ((ev >> 4) & m) | (((od >> 4) & m) << 8);
}

// Cost of pixel (x, y) with own descriptor a under quarter-pixel flow f: the
// target (4x + u, 4y + v) must lie in [0, 4(W-1)] x [0, 4(H-1)]; B's 2x2
// neighbourhood is interpolated with weights (4-ax)(4-ay), ax(4-ay),
// (4-ax)ay, ax ay.  A neighbour of zero weight is replaced by the pixel
// itself, so no read leaves the image (four loads whatever the fraction:
// skipping them per lane measured slower).  INF outside.
template <bool COL>
__device__ __forceinline__ int32_t subpix_cost(gcu8* __restrict__ DB, int W, int H, int CS, int x, int y, uint32_t f,
                                               uint4 a)
{
    const int tx = 4 * x + flow_x(f), ty = 4 * y + flow_y(f);
    if (tx < 0 || ty < 0) return kInf;
    const int ix = tx >> 2, iy = ty >> 2, ax = tx & 3, ay = ty & 3;
    if (ix > W - 1 || iy > H - 1 || (ix == W - 1 && ax) || (iy == H - 1 && ay)) return kInf;
    const int ix1 = ax ? ix + 1 : ix, iy1 = ay ? iy + 1 : iy;
    const uint4 b00 = ld16(DB + pix<COL>(ix, iy, CS) * 16), b10 = ld16(DB + pix<COL>(ix1, iy, CS) * 16);
    const uint4 b01 = ld16(DB + pix<COL>(ix, iy1, CS) * 16), b11 = ld16(DB + pix<COL>(ix1, iy1, CS) * 16);
    const uint32_t w00 = (4 - ax) * (4 - ay), w10 = ax * (4 - ay), w01 = (4 - ax) * ay, w11 = ax * ay;
    const uint4 i = make_uint4(bilerp_word(b00.x, b10.x, b01.x, b11.x, w00, w10, w01, w11),
                               bilerp_word(b00.y, b10.y, b01.y, b11.y, w00, w10, w01, w11),
                               bilerp_word(b00.z, b10.z, b01.z, b11.z, w00, w10, w01, w11),
                               bilerp_word(b00.w, b10.w, b01.w, b11.w, w00, w10, w01, w11));
    return sad16(a, i);
}

// Matching cost of pixel (x, y) of A, feature a, under flow f against the
// feature plane DB of B (layout by COL, column stride CS); INF when the
// target leaves the image, and then no load is issued.
template <bool COL, int CK>
__device__ __forceinline__ int32_t feat_cost(gcu8* __restrict__ DB, int W, int H, int CS, int x, int y, uint32_t f,
                                             typename Feat<CK>::T a)
{
    if constexpr (CK == 2) {
        return subpix_cost<COL>(DB, W, H, CS, x, y, f, a);
    } else {
        const int qx = x + flow_x(f), qy = y + flow_y(f);
        if ((unsigned)qx >= (unsigned)W || (unsigned)qy >= (unsigned)H) return kInf;
        return Feat<CK>::dist(a, Feat<CK>::load(DB, pix<COL>(qx, qy, CS)));
    }
}

// A sweep's predecessor values: every lane takes its lower (higher)
// neighbour's v, lane 0 (63) takes edge -- DPP wave_shr:1 (wave_shl:1), a
// register-to-register shift of the whole wave with the edge lane left at the
// `old` operand, instead of a permute through LDS.
__device__ __forceinline__ uint32_t lane_from_lower(uint32_t v, uint32_t edge)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_from_higher(uint32_t v, uint32_t edge)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xF, 0xF, false);
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of the 4-word S-P network,
// key advanced by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Random search of one pixel (Sec. 3.1: both flow components perturbed by a
// small random amount).  Trials j = 0..J-1 with radius R >> j around the pre-pass
// flow v0; offsets come from the Philox block at counter
// (y*W + x, level, iter << 2 | pass, j >> 1), words (0,1) for even j and
// (2,3) for odd j.  All trial costs are gathered first (independent loads),
// then selected in trial order with a strict '<', which equals the
// sequential rule because a trial equal to the running best costs the same.
// A trial with a zero offset repeats v0, whose cost bounds the running best
// from above, so it can never be taken and is not evaluated.
// `cost(flow)` evaluates one trial (a global gather, or an LDS read when the
// caller staged the target neighbourhood).
template <int RC, typename CostFn>
__device__ __forceinline__ void random_search(uint32_t& bf, int32_t& bc, int W, int x, int y, uint32_t level,
                                              uint32_t ctr2, const SearchConst& sc, CostFn cost)
{
    const int vx = flow_x(bf), vy = flow_y(bf);
    const uint32_t ctr0 = (uint32_t)(y * W + x);
    if constexpr (RC > 0) {
        constexpr int JC = 31 - __builtin_clz((unsigned)RC) + 1;
        uint32_t cand[JC];
        int32_t e[JC];
        uint4 u = make_uint4(0, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < JC; ++j) {
            if ((j & 1) == 0) u = philox4x32_10(make_uint4(ctr0, level, ctr2, (uint32_t)(j >> 1)), sc.key0, sc.key1);
            const uint32_t ux = (j & 1) ? u.z : u.x;
            const uint32_t uy = (j & 1) ? u.w : u.y;
            const int r = RC >> j;
            const uint32_t span = 2u * (uint32_t)r + 1u;
            const int dx = (int)(ux % span) - r, dy = (int)(uy % span) - r;
            cand[j] = pack_flow(vx + dx, vy + dy);
            e[j] = (dx | dy) != 0 ? cost(cand[j]) : kInf;        // zero offset: never selected
        }
#pragma unroll
        for (int j = 0; j < JC; ++j)
            if (e[j] < bc) { bc = e[j]; bf = cand[j]; }
    } else {
        uint4 u = make_uint4(0, 0, 0, 0);
        for (int j = 0; j < sc.trials; ++j) {
            if ((j & 1) == 0) u = philox4x32_10(make_uint4(ctr0, level, ctr2, (uint32_t)(j >> 1)), sc.key0, sc.key1);
            const uint32_t ux = (j & 1) ? u.z : u.x;
            const uint32_t uy = (j & 1) ? u.w : u.y;
            const int r = sc.radius >> j;
            const uint32_t span = 2u * (uint32_t)r + 1u;
            const int dx = (int)(ux % span) - r, dy = (int)(uy % span) - r;
            const uint32_t c = pack_flow(vx + dx, vy + dy);
            const int32_t ej = (dx | dy) != 0 ? cost(c) : kInf;
            if (ej < bc) { bc = ej; bf = c; }
        }
    }
}

// ------------------------------------------------------------- ingest ---
// Level-0 luma of both images: Y = (77 R + 150 G + 29 B + 128) >> 8, C = 1
// copies.  16 pixels per thread: 48 (or 16) input bytes in 16-byte loads
// when the image is 16-byte aligned, one 16-byte store; the plane's ragged
// end and unaligned images go byte by byte.  grid (blocks per image, 2 * pairs),
// each block striding over its image's 4096-pixel spans.
__device__ __forceinline__ uint32_t luma4(const uint32_t* w, int k0)
{
    // pixels k0 .. k0+3 of a 48-byte group held as 12 little-endian words
    uint32_t out = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int j = 3 * (k0 + k);
        const uint32_t r = (w[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        const uint32_t g = (w[(j + 1) >> 2] >> (8 * ((j + 1) & 3))) & 0xFFu;
        const uint32_t b = (w[(j + 2) >> 2] >> (8 * ((j + 2) & 3))) & 0xFFu;
        out |= ((77u * r + 150u * g + 29u * b + 128u) >> 8) << (8 * k);
    }
    return out;
}

// Luma of the 16 pixels from i0 (fewer at the plane's end): 16-byte loads
// and one 16-byte store when the image is 16-byte aligned, else byte by byte.
__device__ __forceinline__ void gray16(const uint8_t* __restrict__ src, uint8_t* __restrict__ dst, int C, int n,
                                       int i0)
{
    if (i0 + 16 <= n && ((uintptr_t)src & 15u) == 0) {
        u32x4 o;
        if (C == 3) {
            gcu4* s4 = (gcu4*)(src + (size_t)i0 * 3);
            const u32x4 a = s4[0], b = s4[1], c = s4[2];
            const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
            o = u32x4{luma4(w, 0), luma4(w, 4), luma4(w, 8), luma4(w, 12)};
        } else {
            o = *(gcu4*)(src + i0);
        }
        *(FF_GLOBAL u32x4*)(dst + i0) = o;
        return;
    }
    for (int i = i0; i < min(i0 + 16, n); ++i) {
        uint8_t v;
        if (C == 3) {
            const uint8_t* p = src + (size_t)i * 3;
            v = (uint8_t)((77u * p[0] + 150u * p[1] + 29u * p[2] + 128u) >> 8);
        } else {
            v = src[i];
        }
        dst[i] = v;
    }
}

// grid (blocks per image, 2 * pairs): each block strides over its image's
// 16-pixel groups (few blocks per image for batches of many small pairs).
__global__ __launch_bounds__(256) void k_gray(const PairDev* __restrict__ pairs)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int img = blockIdx.y & 1;
    const int n = P.lv[0].W * P.lv[0].H;
    const uint8_t* src = P.img[img];
    uint8_t* dst = P.lv[0].gray[img];
    for (int i0 = (blockIdx.x * 256 + threadIdx.x) * 16; i0 < n; i0 += gridDim.x * 256 * 16)
        gray16(src, dst, P.C, n, i0);
}

// One pyramid step: 2x2 box mean rounded half up, floor dimensions.  grid
// (blocks per image, 2 * pairs), each block striding over its image.
__global__ __launch_bounds__(256) void k_down2(const PairDev* __restrict__ pairs, int level)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int img = blockIdx.y & 1;
    const LevelDev& S = P.lv[level - 1];
    const LevelDev& D = P.lv[level];
    const int n = D.W * D.H;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const int x = i % D.W, y = i / D.W;
        const uint8_t* s = S.gray[img] + (size_t)(2 * y) * S.W + 2 * x;
        const uint32_t sum = (uint32_t)s[0] + s[1] + s[S.W] + s[S.W + 1];
        D.gray[img][i] = (uint8_t)((sum + 2u) >> 2);
    }
}

// -------------------------------------------------------- descriptors ---
// 16 Walsh-Hadamard coefficients of the 8x8 patch at every pixel (Sec. 3.1),
// separable: the four lowest-sequency Walsh functions on 8 samples are
// constant on sample pairs, so a 1-D transform is 4 pair sums and one
// 4-point butterfly.  A block covers 64 x 32 outputs.  Its 71 x 39 input
// window (replicated border) and the 39 x 64 row transforms (4 x int16) live
// in LDS; thread (c, g) takes column c, rows 8g .. 8g+7, and runs the column
// transform on packed int16 pairs (every partial sum stays within 16 320):
// 15 row transforms give the 14 vertical pair sums its 8 outputs share.
// Written row-major straight from registers (lanes along x) and
// column-major through LDS (lanes along y), both coalesced.
constexpr int kDescTX = 64, kDescTY = 32;
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t desc_word(s16x2 lo, s16x2 hi, uint32_t bias)
{
    // floor(c / 64) of the four coefficients, low bytes packed, biased by +128
    // except the DC byte (already 0..255)
    const s16x2 ql = lo >> (short)6, qh = hi >> (short)6;
    return __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, qh), __builtin_bit_cast(uint32_t, ql), 0x06040200u) ^ bias;
}

template <bool STREAM>
__global__ __launch_bounds__(256) void k_desc(const PairDev* __restrict__ pairs, int level)
{
    const int3 tb = xcd_block3();
    const PairDev& P = pairs[tb.z >> 1];
    const int img = tb.z & 1;
    const LevelDev& L = P.lv[level];
    const int W = L.W, H = L.H;
    const int x0 = tb.x * kDescTX, y0 = tb.y * kDescTY;
    if (x0 >= W || y0 >= H) return;
    constexpr int TR = kDescTY + 7;                              // input rows
    __shared__ union {
        struct {
            uint8_t tile[TR][kDescTX + 8];                      // 39 x 72 bytes (8-byte multiple)
            uint2 rowt[TR][kDescTX];                            // 4 x int16 row transforms
        } in;
        uint4 res[kDescTY / 2][kDescTX + 1];                    // half of the finished descriptors
    } sm;
    // input window: all loads issued before the first LDS write
    gcu8* __restrict__ src = (gcu8*)L.gray[img];
    constexpr int NT = TR * (kDescTX + 7), NI = (NT + 255) / 256;
    uint8_t v[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int r = i / (kDescTX + 7), c = i % (kDescTX + 7);
        const int gy = min(max(y0 - 3 + r, 0), H - 1);
        const int gx = min(max(x0 - 3 + c, 0), W - 1);
        v[k] = i < NT ? src[(uint32_t)gy * (uint32_t)W + (uint32_t)gx] : 0;
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < NT) sm.in.tile[i / (kDescTX + 7)][i % (kDescTX + 7)] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < (TR * kDescTX + 255) / 256; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i >= TR * kDescTX) break;
        const int r = i / kDescTX, c = i % kDescTX;
        const uint8_t* t = &sm.in.tile[r][c];
        const int q0 = t[0] + t[1], q1 = t[2] + t[3], q2 = t[4] + t[5], q3 = t[6] + t[7];
        const int a = q0 + q1, b = q2 + q3, d = q0 - q1, e = q2 - q3;
        // sequency order: (a + b, a - b, d - e, d + e)
        sm.in.rowt[r][c] = make_uint2(((uint32_t)(a + b) & 0xFFFFu) | ((uint32_t)(a - b) << 16),
                                      ((uint32_t)(d - e) & 0xFFFFu) | ((uint32_t)(d + e) << 16));
    }
    __syncthreads();
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    // vertical pair sums P_k = rowt[8g + k] + rowt[8g + k + 1], k = 0 .. 13,
    // as (v0, v1) and (v2, v3) packed pairs
    s16x2 pl[14], ph[14];
    {
        uint2 prev = sm.in.rowt[8 * g][c];
#pragma unroll
        for (int k = 0; k < 14; ++k) {
            const uint2 nxt = sm.in.rowt[8 * g + k + 1][c];
            pl[k] = __builtin_bit_cast(s16x2, prev.x) + __builtin_bit_cast(s16x2, nxt.x);
            ph[k] = __builtin_bit_cast(s16x2, prev.y) + __builtin_bit_cast(s16x2, nxt.y);
            prev = nxt;
        }
    }
    uint4 out[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // column butterfly over the pair sums at rows i, i+2, i+4, i+6
        const s16x2 al = pl[i] + pl[i + 2], bl = pl[i + 4] + pl[i + 6];
        const s16x2 dl = pl[i] - pl[i + 2], el = pl[i + 4] - pl[i + 6];
        const s16x2 ah = ph[i] + ph[i + 2], bh = ph[i + 4] + ph[i + 6];
        const s16x2 dh = ph[i] - ph[i + 2], eh = ph[i + 4] - ph[i + 6];
        out[i] = make_uint4(desc_word(al + bl, ah + bh, 0x80808000u), desc_word(al - bl, ah - bh, 0x80808080u),
                            desc_word(dl - el, dh - eh, 0x80808080u), desc_word(dl + el, dh + eh, 0x80808080u));
    }
    // Row-major copy: whole 1 KB runs per store instruction.  STREAM (level 0:
    // the largest planes, read only by later kernels): non-temporal stores,
    // which stream through L2 without displacing other data; the coarser
    // levels' planes are read right after (seed records, coarse line
    // phases) and stay cached.  The column-major copy's 256-byte runs share
    // cache lines with the neighbouring tile's and need L2 to merge them:
    // ordinary stores.
    const int x = x0 + c;
    FF_GLOBAL u32x4* dst = (FF_GLOBAL u32x4*)L.desc[img];
#pragma unroll
    for (int i = 0; i < 8; ++i) {                                // row-major: lanes along x
        const int y = y0 + 8 * g + i;
        if (x < W && y < H) {
            FF_GLOBAL u32x4* q = dst + ((uint32_t)y * (uint32_t)L.Wp + (uint32_t)x);
            const u32x4 v = u32x4{out[i].x, out[i].y, out[i].z, out[i].w};
            if constexpr (STREAM) __builtin_nontemporal_store(v, q);
            else *q = v;
        }
    }
    FF_GLOBAL u32x4* dstT = (FF_GLOBAL u32x4*)L.descT[img];
    for (int half = 0; half < 2; ++half) {                       // column-major, 16 rows at a time
        __syncthreads();                                         // row transforms / previous half consumed
        if ((g >> 1) == half) {
#pragma unroll
            for (int i = 0; i < 8; ++i) sm.res[8 * (g & 1) + i][c] = out[i];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {                            // lanes along y: 16 rows x 4 columns a wave
            const int i = threadIdx.x + 256 * k;
            const int r = i % 16, cc = i / 16;
            const int xx = x0 + cc, yy = y0 + 16 * half + r;
            if (xx < W && yy < H) {
                const uint4 w = sm.res[r][cc];
                dstT[(uint32_t)xx * (uint32_t)L.Hp + (uint32_t)yy] = u32x4{w.x, w.y, w.z, w.w};
            }
        }
    }
}

// ------------------------------------------------------------- Census ---
// 7x7 Census strings (Sec. 3.1, the Census matching cost): bit k, for the
// k-th of the 48 neighbours (dx, dy) in [-3, 3]^2 other than the centre in
// row-major order, is set when the neighbour is strictly darker than the
// centre; border replicated.  A block covers 64 x 32 outputs with its
// 70 x 38 input window in LDS (all byte loads in flight before the first
// LDS write); thread (c, g) builds column c, rows 8g .. 8g+7.  Stored as
// u64 row-major from registers and column-major through LDS, 16 rows at a
// time, both coalesced.  grid (ceil(W/64), ceil(H/32), 2 * pairs).
constexpr int kCenTX = 64, kCenTY = 32;

__global__ __launch_bounds__(256) void k_census(const PairDev* __restrict__ pairs, int level)
{
    const PairDev& P = pairs[blockIdx.z >> 1];
    const int img = blockIdx.z & 1;
    const LevelDev& L = P.lv[level];
    const int W = L.W, H = L.H;
    const int x0 = blockIdx.x * kCenTX, y0 = blockIdx.y * kCenTY;
    if (x0 >= W || y0 >= H) return;
    constexpr int TR = kCenTY + 6, TC = kCenTX + 6;
    __shared__ union {
        uint8_t tile[TR][kCenTX + 8];
        uint2 res[kCenTY / 2][kCenTX + 1];
    } sm;
    gcu8* __restrict__ src = (gcu8*)L.gray[img];
    constexpr int NT = TR * TC, NI = (NT + 255) / 256;
    uint8_t v[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        const int r = i / TC, c = i % TC;
        const int gy = min(max(y0 - 3 + r, 0), H - 1);
        const int gx = min(max(x0 - 3 + c, 0), W - 1);
        v[k] = i < NT ? src[(uint32_t)gy * (uint32_t)W + (uint32_t)gx] : 0;
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int i = threadIdx.x + 256 * k;
        if (i < NT) sm.tile[i / TC][i % TC] = v[k];
    }
    __syncthreads();
    const int c = threadIdx.x & 63, g = threadIdx.x >> 6;
    uint32_t rows[14][2];                                        // window rows 8g .. 8g+13, bytes c .. c+7
#pragma unroll
    for (int r = 0; r < 14; ++r) {
        const uint8_t* t = &sm.tile[8 * g + r][c];
        rows[r][0] = (uint32_t)t[0] | ((uint32_t)t[1] << 8) | ((uint32_t)t[2] << 16) | ((uint32_t)t[3] << 24);
        rows[r][1] = (uint32_t)t[4] | ((uint32_t)t[5] << 8) | ((uint32_t)t[6] << 16);
    }
    uint2 out[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint32_t centre = (rows[i + 3][0] >> 24) & 0xFFu;       // byte 3 of row i+3
        uint32_t lo = 0, hi = 0;
        int k = 0;
#pragma unroll
        for (int dy = 0; dy < 7; ++dy) {
#pragma unroll
            for (int dx = 0; dx < 7; ++dx) {
                if (dy == 3 && dx == 3) continue;
                const uint32_t nb = (rows[i + dy][dx >> 2] >> (8 * (dx & 3))) & 0xFFu;
                const uint32_t bit = nb < centre ? 1u : 0u;
                if (k < 32) lo |= bit << k;
                else hi |= bit << (k - 32);
                ++k;
            }
        }
        out[i] = make_uint2(lo, hi);
    }
    const int x = x0 + c;
    FF_GLOBAL u32x2* dst = (FF_GLOBAL u32x2*)L.cen[img];
#pragma unroll
    for (int i = 0; i < 8; ++i) {                                // row-major: lanes along x
        const int y = y0 + 8 * g + i;
        if (x < W && y < H) dst[(uint32_t)y * (uint32_t)L.Wp + (uint32_t)x] = u32x2{out[i].x, out[i].y};
    }
    FF_GLOBAL u32x2* dstT = (FF_GLOBAL u32x2*)L.cenT[img];
    for (int half = 0; half < 2; ++half) {                       // column-major, 16 rows at a time
        __syncthreads();
        if ((g >> 1) == half) {
#pragma unroll
            for (int i = 0; i < 8; ++i) sm.res[8 * (g & 1) + i][c] = out[i];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; ++k) {                            // lanes along y
            const int i = threadIdx.x + 256 * k;
            const int r = i % 16, cc = i / 16;
            const int xx = x0 + cc, yy = y0 + 16 * half + r;
            if (xx < W && yy < H) {
                const uint2 w = sm.res[r][cc];
                dstT[(uint32_t)xx * (uint32_t)L.Hp + (uint32_t)yy] = u32x2{w.x, w.y};
            }
        }
    }
}

// ------------------------------------------------------------ seed NN ---
// Database records for the exact seed search at the coarsest level.  The
// score 2 a.b - |b|^2 (maximised; equivalent to minimising |a - b|^2) is one
// v_mfma_i32_16x16x64_i8 per 16 x 16 tile: the 64-deep K axis holds
//   A row  = [ a, a, g0, g1 ]      B column = [ b, b, beta0, beta1 ]
// with constants g = (127 x 31, 1) and digits beta (31 in [-128, 0], the last
// in [0, 126]) such that g . beta = -|b|^2 exactly.  Also clears the keys.
__global__ __launch_bounds__(256) void k_seed_records(const PairDev* __restrict__ pairs, int level)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int img = blockIdx.y & 1;
    const LevelDev& L = P.lv[level];
    const int N = L.W * L.H, Q = P.nsx * P.nsy;                // Q <= N: seeds are pixels
    // a thread builds one record in LDS; the block then stores its 256
    // records (16 KiB) as consecutive 16-byte pieces, so every store
    // instruction writes 1 KiB of consecutive memory
    __shared__ u32x4 recs[256 * 4];
    FF_GLOBAL u32x4* out = (FF_GLOBAL u32x4*)P.dbrec[img];
    // grid (blocks per image, 2 * pairs): each block strides over its image
    for (int base = blockIdx.x * 256; base < N; base += gridDim.x * 256) {   // uniform per block
        const int n = base + (int)threadIdx.x;
        if (n < N) {
            if (n < Q) ((FF_GLOBAL unsigned long long*)P.keys[img])[n] = 0ull;
            const uint4 db = load_desc((gcu8*)L.desc[img], (size_t)(n / L.W) * L.Wp + (size_t)(n % L.W));
            const uint4 b = make_uint4(db.x ^ 0x80808080u, db.y ^ 0x80808080u, db.z ^ 0x80808080u, db.w ^ 0x80808080u);
            const uint32_t bw[4] = {b.x, b.y, b.z, b.w};
            int nb = 0;
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int v = (int)(int8_t)(bw[k >> 2] >> (8 * (k & 3)));
                nb += v * v;
            }
            const int neg = -nb;                                    // in [-262144, 0]
            const int X = -((-neg + 126) / 127);                    // floor(neg / 127), neg <= 0
            const int rmd = neg - 127 * X;                          // 0..126
            uint32_t beta[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            int rem = X;
#pragma unroll
            for (int k = 0; k < 31; ++k) {
                const int v = max(rem, -128);
                rem -= v;
                beta[k >> 2] |= (uint32_t)(v & 0xFF) << (8 * (k & 3));
            }
            beta[7] |= (uint32_t)(rmd & 0xFF) << 24;
            recs[threadIdx.x * 4 + 0] = u32x4{b.x, b.y, b.z, b.w};
            recs[threadIdx.x * 4 + 1] = u32x4{b.x, b.y, b.z, b.w};
            recs[threadIdx.x * 4 + 2] = u32x4{beta[0], beta[1], beta[2], beta[3]};
            recs[threadIdx.x * 4 + 3] = u32x4{beta[4], beta[5], beta[6], beta[7]};
        }
        __syncthreads();
        const int pieces = min(256, N - base) * 4;                 // 16-byte pieces of this block's records
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int e = (int)threadIdx.x + 256 * k;
            if (e < pieces) out[(size_t)base * 4 + (size_t)e] = recs[e];
        }
        __syncthreads();                                          // records stored before the next round overwrites them
    }
}

// Exact nearest neighbour of every seed of A among all coarsest pixels of B
// (Sec. 3.1 initial matches; the exact answer the kd-tree approximates).
// A block of 4 waves holds 4 x 16*MQ seeds as MFMA A operands and streams
// one split of the database: chunks of kSeedChunk tiles are copied once per
// block into LDS (direct global -> LDS loads) and read by all four waves, so
// the database crosses L2 once per block instead of once per wave.  Each
// tile sits in LDS in lane order -- slot 16 g + n holds group g of record n,
// the 16 bytes lane n + 16 g feeds to the MFMA -- so a wave reads a tile as
// 64 consecutive 16-byte slots, free of bank conflicts (the copy permutes
// its source addresses inside the tile's kilobyte instead).  A wave scores
// only its seed tiles that hold seeds: a wave, or the tail of one, past the
// last seed issues no MFMA.  Per lane and seed row a wave keeps each chunk's
// largest score (one v_max3 per two scores) and folds it into
// max((score << 11) | (2047 - chunk)), so equal scores prefer the earlier
// chunk; splits merge (score, chunk) per seed and k_seed_resolve picks the
// lowest index inside the winning chunk -- the lowest index wins every tie.
// grid (ceil(seed tiles / (4 MQ)), splits, 2 * pairs), 256 threads.
// Largest value over the 16 lanes of each row of the wave: DPP within the
// row -- two quad swaps, then rotations of the row by 4 and by 8 lanes (every
// source lane lies in the row, so no lane reads the bound value).
__device__ __forceinline__ int row16_max(int k)
{
    k = max(k, __builtin_amdgcn_mov_dpp(k, 0xB1, 0xF, 0xF, true));    // quad_perm [1, 0, 3, 2]
    k = max(k, __builtin_amdgcn_mov_dpp(k, 0x4E, 0xF, 0xF, true));    // quad_perm [2, 3, 0, 1]
    k = max(k, __builtin_amdgcn_mov_dpp(k, 0x124, 0xF, 0xF, true));   // row_ror:4
    k = max(k, __builtin_amdgcn_mov_dpp(k, 0x128, 0xF, 0xF, true));   // row_ror:8
    return k;
}

constexpr int kSeedChunk = 16;                                   // tiles (16 KiB) per LDS chunk
constexpr int kNoScore = -(1 << 20);                             // below every score; << 11 gives INT32_MIN

template <int MQ>
__global__ __launch_bounds__(256) void k_seed_nn(const PairDev* __restrict__ pairs, int level,
                                                int stride, int tiles_per_split)
{
    // XCD-aware order: the seed blocks streaming one split (consecutive x)
    // run on one XCD and share the split through its L2
    const int3 bk = xcd_block3();
    const PairDev& P = pairs[bk.z >> 1];
    const int dir = bk.z & 1;
    const LevelDev& L = P.lv[level];
    const int N = L.W * L.H, Q = P.nsx * P.nsy;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    if (bk.x * 4 * 16 * MQ >= Q) return;                         // no seeds in this block: uniform
    const int ntiles = (N + 15) >> 4;
    const int t0 = bk.y * tiles_per_split;
    if (t0 >= ntiles) return;                                    // uniform
    const int t1 = min(t0 + tiles_per_split, ntiles);
    const int qbase = (bk.x * 4 + wave) * 16 * MQ;               // may exceed Q: the wave still copies
    const int live = min(MQ, max(0, (Q - qbase + 15) >> 4));    // seed tiles of this wave holding seeds
    const int m = lane & 15, g = lane >> 4;
    __shared__ v4i tiles[kSeedChunk * 64];

    // a seed's grid cell (q % nsx, q / nsx) from one division per wave: q =
    // y0 nsx + r0 + 16 mq + m, and the lane takes whole rows off its offset
    const int nsx = P.nsx, y0 = qbase / nsx, r0 = qbase - y0 * nsx;
    v4i A[MQ];
#pragma unroll
    for (int mq = 0; mq < MQ; ++mq) {
        const int q = qbase + 16 * mq + m;
        if (g >= 2) {
            A[mq] = v4i{0x7F7F7F7F, 0x7F7F7F7F, 0x7F7F7F7F, g == 2 ? 0x7F7F7F7F : 0x017F7F7F};
        } else if (q < Q) {
            int cx = r0 + 16 * mq + m, cy = y0;
            while (cx >= nsx) {
                cx -= nsx;
                ++cy;
            }
            const int sx = cx * stride, sy = cy * stride;
            const uint4 d = load_desc((gcu8*)L.desc[dir], (size_t)sy * L.Wp + sx);
            A[mq] = v4i{(int)(d.x ^ 0x80808080u), (int)(d.y ^ 0x80808080u), (int)(d.z ^ 0x80808080u),
                        (int)(d.w ^ 0x80808080u)};
        } else {
            A[mq] = v4i{0, 0, 0, 0};
        }
    }
    int best[MQ][4];
#pragma unroll
    for (int mq = 0; mq < MQ; ++mq)
#pragma unroll
        for (int i = 0; i < 4; ++i) best[mq][i] = INT32_MIN;

    const FF_GLOBAL v4i* rec = (const FF_GLOBAL v4i*)P.dbrec[dir ^ 1];
    const v4i zero = v4i{0, 0, 0, 0};
    const uint32_t nrec4 = (uint32_t)N * 4u;                     // valid 16-byte groups of the database
    // LDS slot e of a chunk holds the chunk's 16-byte group src(e): tile
    // e / 64, record e % 16, group (e / 16) % 4
    const uint32_t esrc = (uint32_t)(threadIdx.x & ~63u) | ((threadIdx.x & 15u) << 2) | ((threadIdx.x >> 4) & 3u);
    for (int tb = t0, c = 0; tb < t1; tb += kSeedChunk, ++c) {
        const int nt = min(kSeedChunk, t1 - tb);
        // copy tiles tb .. tb+nt-1 into LDS: thread e fills slots e, e + 256,
        // ...; a wave's 64 lanes land on 64 consecutive LDS slots
        for (int e = threadIdx.x, k = 0; e < nt * 64; e += 256, k += 256) {
            const uint32_t gidx = (uint32_t)tb * 64u + esrc + (uint32_t)k;
            if (gidx < nrec4)
                __builtin_amdgcn_global_load_lds((const FF_GLOBAL void*)(rec + gidx),
                                                 (__attribute__((address_space(3))) void*)&tiles[e - lane], 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const v4i* __restrict__ T = tiles;
        // the chunk's largest score per lane and seed row: one v_max3 per two
        // scores, full tiles two at a time; instantiated per number of live
        // seed tiles so the MFMA chain has no branches
        auto score = [&](auto LIVE) {
            constexpr int LV = decltype(LIVE)::value;
            const int tfull = min(tb + nt, N >> 4);
            // the first two full tiles start the running maxima
            int cm[LV][4];
            int t = tb;
            if (t + 1 < tfull) {
                const v4i B0 = T[(uint32_t)lane];
                const v4i B1 = T[64u + (uint32_t)lane];
#pragma unroll
                for (int mq = 0; mq < LV; ++mq) {
                    const v4i acc0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mq], B0, zero, 0, 0, 0);
                    const v4i acc1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mq], B1, zero, 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) cm[mq][i] = max(acc0[i], acc1[i]);
                }
                t += 2;
            } else {
#pragma unroll
                for (int mq = 0; mq < LV; ++mq)
#pragma unroll
                    for (int i = 0; i < 4; ++i) cm[mq][i] = kNoScore;
            }
            for (; t + 1 < tfull; t += 2) {
                const v4i B0 = T[(uint32_t)(t - tb) * 64u + (uint32_t)lane];
                const v4i B1 = T[(uint32_t)(t - tb) * 64u + 64u + (uint32_t)lane];
#pragma unroll
                for (int mq = 0; mq < LV; ++mq) {
                    const v4i acc0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mq], B0, zero, 0, 0, 0);
                    const v4i acc1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mq], B1, zero, 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) cm[mq][i] = max(cm[mq][i], max(acc0[i], acc1[i]));
                }
            }
            // remaining tile of the chunk, possibly the ragged last one of the plane
            for (; t < tb + nt; ++t) {
                const bool nvalid = t * 16 + m < N;
                const v4i B = T[(uint32_t)(t - tb) * 64u + (uint32_t)lane];
#pragma unroll
                for (int mq = 0; mq < LV; ++mq) {
                    const v4i acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mq], B, zero, 0, 0, 0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) cm[mq][i] = max(cm[mq][i], nvalid ? acc[i] : kNoScore);
                }
            }
            // key = (score << 11) | (2047 - chunk): equal scores prefer the earlier chunk
            const uint32_t tag = (uint32_t)(2047 - c);
#pragma unroll
            for (int mq = 0; mq < LV; ++mq)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    best[mq][i] = max(best[mq][i], (int)(((uint32_t)cm[mq][i] << 11) | tag));
        };
        static_assert(MQ == 4, "the live-count dispatch below covers MQ = 4");
        if (live == 4) score(std::integral_constant<int, 4>{});
        else if (live == 3) score(std::integral_constant<int, 3>{});
        else if (live == 2) score(std::integral_constant<int, 2>{});
        else if (live == 1) score(std::integral_constant<int, 1>{});
        __syncthreads();                                         // chunk consumed before it is overwritten
    }
    if (live == 0) return;
    // Per seed: the best key over its 16 columns; splits merge (score, first
    // tile of the chunk) with a 64-bit atomicMax on (score + 2^20) << 32 |
    // low word, so the merged key names the earliest chunk reaching the best
    // score.  Low word: (0xFFFF - tile) << 16 | the mask of columns reaching
    // the key (a chunk lies in one split, so the mask never decides the max);
    // with more than 65536 tiles, ~tile and every column.  k_seed_resolve then
    // finds the lowest index inside that chunk.
#pragma unroll
    for (int mq = 0; mq < MQ; ++mq) {
        if (mq >= live) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = row16_max(best[mq][i]);
            const uint32_t cols = (uint32_t)(__ballot(best[mq][i] == k) >> (16 * g)) & 0xFFFFu;
            const int q = qbase + 16 * mq + 4 * g + i;
            if (m == 0 && q < Q && (k >> 11) != kNoScore) {
                const uint32_t tb = (uint32_t)(t0 + (2047 - (k & 2047)) * kSeedChunk);
                const uint32_t lo = ntiles > 65536 ? 0xFFFFFFFFu - tb : ((0xFFFFu - tb) << 16) | cols;
                const unsigned long long key =
                    ((unsigned long long)(uint32_t)((k >> 11) + (1 << 20)) << 32) | (unsigned long long)lo;
                atomicMax(&P.keys[dir][q], key);
            }
        }
    }
}

// The lowest database index reaching each seed's best score: the merged key
// holds the score, the first tile of the earliest chunk reaching it and the
// columns that reach it there, so the answer is the first of those columns'
// entries in the chunk's 16 tiles with the score, evaluated from the int8
// descriptors as 2 a.b - |b|^2 with v_dot4 (the integer the MFMA forms).
// Entries past the chunk's split come later than every entry of the chunk,
// so scanning all 16 tiles finds the same first one.  The key's low word
// becomes ~index.  4 lanes per seed, lane s taking tiles 4s .. 4s+3 of each
// listed column in turn, 64 seeds at a time; grid (blocks per image,
// 2 * pairs), 256 threads, each block striding over its seeds.
__global__ __launch_bounds__(256) void k_seed_resolve(const PairDev* __restrict__ pairs, int level, int stride)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int dir = blockIdx.y & 1;
    const LevelDev& L = P.lv[level];
    const int W = L.W, N = L.W * L.H, Q = P.nsx * P.nsy;
    const int sub = threadIdx.x & 3;                             // tiles 4 sub .. 4 sub + 3 of the chunk
    // grid (blocks per image, 2 * pairs): each block strides over its
    // pair-direction's seeds, 64 at a time (the bound is uniform per block, so
    // every lane of a seed's group takes part in the shuffles below)
    for (int base = blockIdx.x * 64; base < Q; base += gridDim.x * 64) {
        const int q = base + (threadIdx.x >> 2);                 // 4 lanes per seed
        const bool live = q < Q;
        const unsigned long long key = live ? P.keys[dir][q] : 0ull;
        const int S = (int)(uint32_t)(key >> 32) - (1 << 20);
        const bool wide = (N + 15) / 16 > 65536;
        const uint32_t tb = wide ? 0xFFFFFFFFu - (uint32_t)key : 0xFFFFu - (((uint32_t)key >> 16) & 0xFFFFu);
        uint32_t cols = !live ? 0u : wide ? 0xFFFFu : (uint32_t)key & 0xFFFFu;
        int a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        if (live) {
            const int sx = (q % P.nsx) * stride, sy = (q / P.nsx) * stride;
            const uint4 ad = load_desc((gcu8*)L.desc[dir], (size_t)sy * L.Wp + sx);
            a0 = (int)(ad.x ^ 0x80808080u), a1 = (int)(ad.y ^ 0x80808080u), a2 = (int)(ad.z ^ 0x80808080u),
            a3 = (int)(ad.w ^ 0x80808080u);
        }
        gcu8* __restrict__ DBd = (gcu8*)L.desc[dir ^ 1];
        uint32_t nmin = 0xFFFFFFFFu;
        while (cols) {                                               // uniform within the seed's 4 lanes
            const uint32_t j = (uint32_t)__builtin_ctz(cols);
            cols &= cols - 1u;
            uint4 bd[4];                                             // the lane's four tiles: loads in flight together
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t n = (tb + (uint32_t)(4 * sub + k)) * 16u + j;
                bd[k] = n < (uint32_t)N ? load_desc(DBd, (size_t)(n / (uint32_t)W) * L.Wp + (n % (uint32_t)W))
                                        : make_uint4(0, 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t n = (tb + (uint32_t)(4 * sub + k)) * 16u + j;
                const int b0 = (int)(bd[k].x ^ 0x80808080u), b1 = (int)(bd[k].y ^ 0x80808080u),
                          b2 = (int)(bd[k].z ^ 0x80808080u), b3 = (int)(bd[k].w ^ 0x80808080u);
                int ab = __builtin_amdgcn_sdot4(a0, b0, 0, false);
                ab = __builtin_amdgcn_sdot4(a1, b1, ab, false);
                ab = __builtin_amdgcn_sdot4(a2, b2, ab, false);
                ab = __builtin_amdgcn_sdot4(a3, b3, ab, false);
                int bb = __builtin_amdgcn_sdot4(b0, b0, 0, false);
                bb = __builtin_amdgcn_sdot4(b1, b1, bb, false);
                bb = __builtin_amdgcn_sdot4(b2, b2, bb, false);
                bb = __builtin_amdgcn_sdot4(b3, b3, bb, false);
                if (n < (uint32_t)N && 2 * ab - bb == S) nmin = min(nmin, n);
            }
        }
        nmin = min(nmin, (uint32_t)__shfl_xor((int)nmin, 1, 64));
        nmin = min(nmin, (uint32_t)__shfl_xor((int)nmin, 2, 64));
        if (live && sub == 0) P.keys[dir][q] = (key & 0xFFFFFFFF00000000ull) | (unsigned long long)(0xFFFFFFFFu - nmin);
    }
}

// ----------------------------------------------------------- level init --
// Coarsest level: every pixel takes the flow of the seed of its stride cell.
// Finer levels: twice the flow of the parent pixel (clamped to the coarse
// grid).  Cost re-evaluated on the descriptors or, with census set, on the
// Census strings.  grid (pixels / 256, 2 * pairs).
// Init flow of pixel (x, y) at `level`: the seed of its stride cell at the
// coarsest level, else twice the final flow of its parent (clamped to the
// coarse grid).
__device__ __forceinline__ uint32_t init_flow(const PairDev& P, int dir, int level, bool coarsest, int stride, int W,
                                              int x, int y)
{
    if (coarsest) {
        const int si = x / stride, sj = y / stride;
        const unsigned long long key = P.keys[dir][sj * P.nsx + si];
        const uint32_t q = 0xFFFFFFFFu - (uint32_t)key;
        return pack_flow((int)(q % (uint32_t)W) - si * stride, (int)(q / (uint32_t)W) - sj * stride);
    }
    const LevelDev& C = P.lv[level + 1];
    const int cx = min(x >> 1, C.W - 1), cy = min(y >> 1, C.H - 1);
    const uint32_t cf = (uint32_t)((const gi2*)C.state[dir])[(uint32_t)cy * (uint32_t)C.Wp + (uint32_t)cx].x;
    return pack_flow(2 * flow_x(cf), 2 * flow_y(cf));
}

__global__ __launch_bounds__(256) void k_init(const PairDev* __restrict__ pairs, int level, int coarsest,
                                              int stride, int census)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int dir = blockIdx.y & 1;
    const LevelDev& L = P.lv[level];
    const int W = L.W, H = L.H;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= W * H) return;
    const int x = i % W, y = i / W;
    const uint32_t f = init_flow(P, dir, level, coarsest != 0, stride, W, x, y);
    const size_t ip = (size_t)y * L.Wp + x;                     // row-major planes: rows Wp apart
    const int32_t c = census
                          ? feat_cost<false, 1>((gcu8*)L.cen[dir ^ 1], W, H, L.Wp, x, y, f, Feat<1>::load((gcu8*)L.cen[dir], ip))
                          : feat_cost<false, 0>((gcu8*)L.desc[dir ^ 1], W, H, L.Wp, x, y, f, Feat<0>::load((gcu8*)L.desc[dir], ip));
    L.state[dir][(size_t)y * L.Wp + x] = make_int2((int)f, c);
}

// ------------------------------------------------------- line phases ----

// One phase of one iteration, one wave per line.
//   row phase (COL = false, lines = rows, row-major buffers):
//       LR sweep; RL sweep followed by random-search pass 0
//   col phase (COL = true, lines = columns, column-major buffers):
//       TB sweep followed by pass 1; BT sweep followed by pass 2
// Sweep semantics (propagation, Sec. 3.1): scanning the line, a pixel takes
// its predecessor's post-update flow iff that flow's cost is strictly lower
// than the pixel's own pre-sweep cost.  The result is the unique h with
// h_p = rule(pre_p, h_{p-1}); a window of CH x 64 pixels (lane l holds
// positions w0 + 64c + l) solves it by relaxation -- every pixel re-applies
// the rule to its own pre-sweep value and its predecessor's current value
// until no predecessor value changes -- with the boundary value carried in
// from the previous window.  Rounds = 1 + longest propagation run in the
// window; only pixels whose predecessor changed gather again.  A pixel's
// random search needs only its own swept state, so it runs on the window
// right after convergence, before the write.  Both passes use the same
// window partition, so every lane re-reads exactly what it wrote.
//
// STG (staged random search): the WPB waves of a block take the windows of
// their WPB adjacent lines in lockstep.  After the sweep of a window every
// wave publishes the flow of one sample pixel; the block takes the median
// of those flows as the window's displacement and loads B's descriptors of
// a fixed RI x RJ neighbourhood -- the window's lines and positions moved
// by that displacement, widened on both sides -- into LDS with coalesced
// loads.  Trials that land inside it read LDS; trials outside it (large
// radii, pixels whose flow departs from the median) load from global
// memory as before.  The trials, their order and their costs are unchanged.
//
// upto (for intermediate captures): row 1 = LR, 2 = +RL, 3 = +RS0;
// col 4 = TB, 5 = +RS1, 6 = +BT, 7 = +RS2.
// WPB lines (waves) per block; grid (ceil(lines / WPB), 2 * pairs).  CH, WPB
// and STG only change scheduling and data movement, never the result.
// One sweep pass of one line, software-pipelined across windows (plain
// path, compile-time radius).  Window w+1's state and own descriptors are
// loaded while window w relaxes; window w's random-search trials are
// gathered at its end and selected during window w+1's first relaxation
// round, so their memory latency overlaps other work.  The trials, their
// order and the selection rule are those of random_search().
// With `lock` (schedule mode 2) the waves of a block take their windows in
// lockstep (a barrier at the start of each window; waves past the block's
// last line pass the same barriers without a line): adjacent lines then
// gather from the same neighbourhood of B at the same time and share its
// cache lines in L1 and L2 (column phase on the 1242x375 batch: 790 -> 748
// us per launch; on short lines the waits can cost more than that gains).
template <int RC, bool COL, int CH, int CK>
__device__ __forceinline__ void line_pass_pipelined(gcu8* __restrict__ DA, gcu8* __restrict__ DB,
                                                    const gi2* __restrict__ Sin, int sstr, gi2* __restrict__ S,
                                                    bool lin, bool lout, LdsLine lline, int W, int H, int CS, int len,
                                                    int line,
                                                    int lane,
                                                    bool fwd, bool rs, uint32_t level, uint32_t ctr2,
                                                    const SearchConst& sc, const PairDev& P, int dir, int initc,
                                                    bool lock)
{
    using FT = typename Feat<CK>::T;
    constexpr int WIN = 64 * CH;
    constexpr int JC = 31 - __builtin_clz((unsigned)RC) + 1;
    const int nwin = (len + WIN - 1) / WIN;
    auto wstart = [&](int wi) { return (fwd ? wi : nwin - 1 - wi) * WIN; };

    uint32_t f0[CH], nf0[CH];
    int32_t c0[CH], nc0[CH];
    FT a[CH], na[CH];
    auto load_window = [&](int w0, uint32_t* F, int32_t* C, FT* A) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int p = w0 + 64 * c + lane;
            const bool valid = p < len;
            A[c] = valid ? Feat<CK>::load(DA, p) : Feat<CK>::zero();
            i32x2 st = i32x2{0, kInf};
            if (valid) {
                if (initc) {                                     // row phase, first pass of iteration 0
                    const uint32_t f = init_flow(P, dir, (int)level, initc == 2, sc.stride, W, p, line);
                    st = i32x2{(int)f, feat_cost<false, CK>(DB, W, H, CS, p, line, f, A[c])};
                } else {
                    st = (lin && lline.has(p)) ? lline.get(p) : Sin[(uint32_t)p * (uint32_t)sstr];
                }
            }
            F[c] = (uint32_t)st.x;
            C[c] = st.y;
        }
    };
    load_window(wstart(0), f0, c0, a);

    // random search of the previous window, gathered but not yet selected
    bool pend = false;
    int pw0 = 0;
    uint32_t pbf[CH], pcand[CH][JC];
    int32_t pbc[CH];
    FT pdesc[CH][JC], pa[CH];
    uint32_t pin[CH];                                            // bit j: trial j lands inside image B
    auto finish = [&]() {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int p = pw0 + 64 * c + lane;
            if (p >= len) continue;
            uint32_t bf = pbf[c];
            int32_t bc = pbc[c];
#pragma unroll
            for (int j = 0; j < JC; ++j) {
                const int32_t e = ((pin[c] >> j) & 1u) ? Feat<CK>::dist(pa[c], pdesc[c][j]) : kInf;
                if (e < bc) { bc = e; bf = pcand[c][j]; }
            }
            if (lout && lline.has(p)) lline.set(p, i32x2{(int)bf, bc});
            else S[p] = i32x2{(int)bf, bc};
        }
    };

    uint32_t carry = 0;
    for (int wi = 0; wi < nwin; ++wi) {
        if (lock) __syncthreads();                               // windows in lockstep across the block
        const int w0 = wstart(wi);
        if (wi + 1 < nwin) load_window(wstart(wi + 1), nf0, nc0, na);
        uint32_t lp[CH], h[CH];
        int32_t le[CH];
        bool hp[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int p = w0 + 64 * c + lane;
            hp[c] = p < len && (fwd ? p > 0 : p + 1 < len);
            lp[c] = f0[c];
            le[c] = c0[c];
            h[c] = f0[c];
        }
        while (true) {
            uint32_t pred[CH];
            bool need[CH];
            bool anyn = false;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                if (fwd) {
                    const uint32_t edge = c == 0 ? carry : (uint32_t)__builtin_amdgcn_readlane((int)h[c > 0 ? c - 1 : 0], 63);
                    pred[c] = lane_from_lower(h[c], edge);
                } else {
                    const uint32_t edge = c == CH - 1 ? carry
                                                      : (uint32_t)__builtin_amdgcn_readlane((int)h[c < CH - 1 ? c + 1 : c], 0);
                    pred[c] = lane_from_higher(h[c], edge);
                }
                need[c] = hp[c] && pred[c] != lp[c];
                anyn |= need[c];
            }
            const bool go = __any(anyn);
            if (go) {
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (need[c]) {
                        const int p = w0 + 64 * c + lane;
                        lp[c] = pred[c];
                        le[c] = pred[c] == f0[c] ? c0[c]
                                                 : feat_cost<COL, CK>(DB, W, H, CS, COL ? line : p, COL ? p : line, pred[c], a[c]);
                    }
                }
            }
            if (pend) {
                finish();
                pend = false;
            }
            if (!go) break;
#pragma unroll
            for (int c = 0; c < CH; ++c) h[c] = le[c] < c0[c] ? lp[c] : f0[c];
        }
        carry = fwd ? (uint32_t)__builtin_amdgcn_readlane((int)h[CH - 1], 63)
                    : (uint32_t)__builtin_amdgcn_readlane((int)h[0], 0);
        if (rs) {
            // issue this window's trials (Philox offsets, gathers); select later
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int p = w0 + 64 * c + lane;
                pbf[c] = h[c];
                pbc[c] = le[c] < c0[c] ? le[c] : c0[c];
                pa[c] = a[c];
                pin[c] = 0;
                if (p >= len) continue;
                const int x = COL ? line : p, y = COL ? p : line;
                const int vx = flow_x(h[c]), vy = flow_y(h[c]);
                const uint32_t ctr0 = (uint32_t)(y * W + x);
                uint4 u = make_uint4(0, 0, 0, 0);
#pragma unroll
                for (int j = 0; j < JC; ++j) {
                    if ((j & 1) == 0) u = philox4x32_10(make_uint4(ctr0, level, ctr2, (uint32_t)(j >> 1)), sc.key0, sc.key1);
                    const uint32_t ux = (j & 1) ? u.z : u.x;
                    const uint32_t uy = (j & 1) ? u.w : u.y;
                    const int r = RC >> j;
                    const uint32_t span = 2u * (uint32_t)r + 1u;
                    const int qdx = (int)(ux % span) - r, qdy = (int)(uy % span) - r;
                    pcand[c][j] = pack_flow(vx + qdx, vy + qdy);
                    const int qx = x + flow_x(pcand[c][j]), qy = y + flow_y(pcand[c][j]);
                    // a zero offset repeats the swept flow, whose cost is the
                    // running best's upper bound: never selected, not gathered
                    const bool in = (unsigned)qx < (unsigned)W && (unsigned)qy < (unsigned)H && (qdx | qdy) != 0;
                    pin[c] |= in ? (1u << j) : 0u;
                    pdesc[c][j] = in ? Feat<CK>::load(DB, pix<COL>(qx, qy, CS)) : Feat<CK>::zero();
                }
            }
            pend = true;
            pw0 = w0;
        } else {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int p = w0 + 64 * c + lane;
                if (p >= len) continue;
                const int32_t bc = le[c] < c0[c] ? le[c] : c0[c];
                if (lout && lline.has(p)) lline.set(p, i32x2{(int)h[c], bc});
                else S[p] = i32x2{(int)h[c], bc};
            }
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            f0[c] = nf0[c];
            c0[c] = nc0[c];
            a[c] = na[c];
        }
    }
    if (pend) finish();
}

// Staged neighbourhood: RJ lines (the block's WPB lines widened by 12 on
// each side, 8 for 16-line blocks) by RI positions (the window widened to
// fill 51 KiB of LDS for 64-px windows -- three blocks per CU -- or 72 KiB
// for 128-px windows).
template <int CH, int WPB>
struct StageDims {
    static constexpr int RJ = WPB + (WPB >= 16 ? 16 : 24);
    static constexpr int RI = (CH == 1 ? 3264 : 4608) / RJ;
    static constexpr int CAP = RI * RJ;
};

template <int RC, bool COL, int CH, int WPB, bool STG, int CK>
__global__ __launch_bounds__(64 * WPB) void k_line_phase(const PairDev* __restrict__ pairs, int level,
                                                         int iter, int upto, SearchConst sc, int xw, int finit,
                                                         const uint32_t* __restrict__ items, int lock)
{
    static_assert(!STG || CK == 0, "the staged random search holds descriptors");
    const uint32_t rlev = sc.rng_level >= 0 ? (uint32_t)sc.rng_level : (uint32_t)level;   // Philox level word
    using FT = typename Feat<CK>::T;
    constexpr size_t FB = CK == 1 ? 8 : 16;                      // feature bytes per pixel
    // The block's pair-direction and line block: from the batch's work list
    // (items: pair-direction << 16 | line block, every block of every pair
    // and nothing past a pair's own size; a 1-D grid) or, for a single pair
    // or pairs of one size, from the 2-D grid (line blocks x pair-directions).
    // Either way in XCD-aware order, so the lines of one pair-direction
    // (which gather from the same descriptor plane) share one L2.
    int pd, bx;
    if (items) {
        const uint32_t it = items[xcd_remap(blockIdx.x, gridDim.x)];
        pd = (int)(it >> 16);
        bx = (int)(it & 0xFFFFu);
    } else {
        const int lb = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
        pd = lb / gridDim.x;
        bx = lb % gridDim.x;
    }
    const PairDev& P = pairs[pd >> 1];
    const int dir = pd & 1;
    const LevelDev& L = P.lv[level];
    const int W = L.W, H = L.H;
    const int len = COL ? H : W, nlines = COL ? W : H;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int line0 = bx * WPB;
    const int line = line0 + wave;
    if (line0 >= nlines) return;                                 // whole block idle: uniform
    const bool active = line < nlines;
    // Lines' state in LDS between the passes (xw > 0: pixels held per line).
    // Column phase: the block copies its WPB columns of the row-major state
    // into LDS, both passes read and write them there, and the block stores
    // them back row-major (otherwise the first pass reads the row-major state
    // in place and the passes write stateT).  Row phase: the first pass reads
    // the state from global memory and leaves its result in LDS, the second
    // pass reads it there and writes global memory; a row longer than xw
    // keeps its last windows in global memory between the passes.
    const bool xwk = xw != 0;
    const bool xwc = COL && xwk;                                 // block-wide copies: every wave takes part
    // the pipelined pass with lock keeps the block's windows in lockstep:
    // every wave stays to pass its barriers
    constexpr bool PIPE = !STG && RC > 0 && CH <= 2 && CK != 2;
    const bool lk = PIPE && lock != 0;
    if (!lk && !STG && !active && !xwc) return;
    const int CS = COL ? L.Hp : L.Wp;                            // feature-plane line stride
    gcu8* __restrict__ DA = (gcu8*)(CK == 1 ? (COL ? L.cenT[dir] : L.cen[dir]) : (COL ? L.descT[dir] : L.desc[dir])) +
                            (size_t)line * CS * FB;
    gcu8* __restrict__ DB = (gcu8*)(CK == 1 ? (COL ? L.cenT[dir ^ 1] : L.cen[dir ^ 1])
                                            : (COL ? L.descT[dir ^ 1] : L.desc[dir ^ 1]));
    gi2* __restrict__ S = (gi2*)(COL ? L.stateT[dir] : L.state[dir]) + (size_t)line * (COL ? len : L.Wp);
    constexpr int WIN = 64 * CH;
    const int nwin = (len + WIN - 1) / WIN;

    using SD = StageDims<CH, WPB>;
    constexpr int RI = SD::RI, RJ = SD::RJ;
    __shared__ uint4 region[STG ? SD::CAP : 1];
    __shared__ int sample[2][WPB][2];                            // per parity: a flow sample (i, j) per line
    __shared__ int sample_ok[2][WPB];
    extern __shared__ uint32_t lbuf_[];                          // xw: WPB lines x xw pixels, two planes
    const int hi = (!COL && len > xw) ? xw / WIN * WIN : len;  // whole windows in LDS
    auto line_lds = [&](int k) {
        __attribute__((address_space(3))) uint32_t* const f = (__attribute__((address_space(3))) uint32_t*)lbuf_;
        return LdsLine{f + k * xw, (__attribute__((address_space(3))) uint16_t*)(f + WPB * xw) + k * xw, hi};
    };
    const LdsLine lline = line_lds(wave);
    if (xwc) {
        const gi2* __restrict__ src = (const gi2*)L.state[dir];
        const int nl = min(WPB, nlines - line0);
        for (int e = threadIdx.x; e < WPB * len; e += 64 * WPB) {
            const int k = e % WPB, p = e / WPB;
            if (k < nl) line_lds(k).set(p, src[(uint32_t)p * (uint32_t)L.Wp + (uint32_t)(line0 + k)]);
        }
        __syncthreads();
    }
    int gw = 0;                                                  // windows staged so far (slot parity)

    for (int pass = 0; pass < 2; ++pass) {
        const bool fwd = pass == 0;
        bool rs;
        uint32_t rs_pass;
        if (!COL) {
            if (!fwd && upto < 2) break;
            rs = !fwd && upto >= 3;
            rs_pass = 0;
        } else {
            if (!fwd && upto < 6) break;
            rs = fwd ? upto >= 5 : upto >= 7;
            rs_pass = fwd ? 1 : 2;
        }
        const uint32_t ctr2 = ((uint32_t)iter << 2) | rs_pass;
        // the column phase's first pass reads the row-major state in place
        const gi2* __restrict__ Sin = (COL && fwd) ? (const gi2*)L.state[dir] + line : S;
        const int sstr = (COL && fwd) ? L.Wp : 1;
        const bool lin = xwk && (COL || !fwd);
        const bool lout = xwk && (COL || (fwd && upto >= 2));
        const bool quarter = CK == 2 && !COL && fwd && finit;

        if constexpr (PIPE) {                                    // the sub-pixel refinement: generic pass
            if (active)
                line_pass_pipelined<RC, COL, CH, CK>(DA, DB, Sin, sstr, S, lin, lout, lline, W, H, CS, len, line, lane, fwd,
                                                     rs,
                                                 (uint32_t)level, ctr2, sc, P, dir,
                                                 (!COL && fwd && finit) ? (level == sc.levels - 1 ? 2 : 1) : 0, lk);
            else if (lk)
                for (int wi = 0; wi < nwin; ++wi) __syncthreads();   // the active waves' barriers, one a window
            continue;
        }
        uint32_t carry = 0;
        for (int wi = 0; wi < nwin; ++wi) {
            const int w0 = (fwd ? wi : nwin - 1 - wi) * WIN;
            uint32_t f0[CH], lp[CH], h[CH];
            int32_t c0[CH], le[CH];
            FT a[CH];
            bool hp[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int p = w0 + 64 * c + lane;
                const bool valid = active && p < len;
                const i32x2 st = !valid                    ? i32x2{0, kInf}
                                 : (lin && lline.has(p)) ? lline.get(p)
                                                         : Sin[(uint32_t)p * (uint32_t)sstr];
                a[c] = valid ? Feat<CK>::load(DA, p) : Feat<CK>::zero();
                f0[c] = (uint32_t)st.x;
                // first row pass of the refinement: whole-pixel flows to
                // quarter pixels on load (costs unchanged, zero fraction)
                if constexpr (CK == 2)
                    if (quarter) f0[c] = pack_flow(4 * flow_x(f0[c]), 4 * flow_y(f0[c]));
                c0[c] = st.y;
                hp[c] = valid && (fwd ? p > 0 : p + 1 < len);
                lp[c] = f0[c];
                le[c] = c0[c];
                h[c] = f0[c];
            }
            // ---- staging of the window's random-search neighbourhood, issued
            // before the sweep so the copy overlaps the relaxation rounds
            int si0 = 0, sj0 = 0;
            if (STG && rs) {
                const int slot = gw & 1;
                if (lane == 32) {                                // sample: lane 32 of the first chunk
                    sample[slot][wave][0] = COL ? flow_y(f0[0]) : flow_x(f0[0]);
                    sample[slot][wave][1] = COL ? flow_x(f0[0]) : flow_y(f0[0]);
                    sample_ok[slot][wave] = (active && w0 + 32 < len) ? 1 : 0;
                }
                __syncthreads();
                // lower median of the published samples, per component: lane k < WPB
                // holds sample k and counts the samples ordered before it (ties by
                // index), so exactly one lane holds each rank
                const bool okk = lane < WPB && sample_ok[slot][lane < WPB ? lane : 0];
                const int vi = okk ? sample[slot][lane][0] : 0, vj = okk ? sample[slot][lane][1] : 0;
                const unsigned long long okmask = __ballot(okk);
                const int nv = __popcll(okmask);
                int rank_i = 0, rank_j = 0;
#pragma unroll
                for (int k = 0; k < WPB; ++k) {
                    if (!((okmask >> k) & 1ull)) continue;
                    const int ik = __builtin_amdgcn_readlane(vi, k), jk = __builtin_amdgcn_readlane(vj, k);
                    rank_i += (ik < vi || (ik == vi && k < lane)) ? 1 : 0;
                    rank_j += (jk < vj || (jk == vj && k < lane)) ? 1 : 0;
                }
                const int mid = (nv - 1) >> 1;
                const unsigned long long hi = __ballot(okk && rank_i == mid), hj = __ballot(okk && rank_j == mid);
                const int mi = nv ? __builtin_amdgcn_readlane(vi, __ffsll((long long)hi) - 1) : 0;
                const int mj = nv ? __builtin_amdgcn_readlane(vj, __ffsll((long long)hj) - 1) : 0;
                si0 = w0 + mi - (RI - WIN) / 2;
                sj0 = line0 + mj - (RJ - WPB) / 2;
                // direct global -> LDS copies (global_load_lds_dwordx4): lane l of a
                // row chunk lands at LDS base + 16 l, lanes outside the image or the
                // row stay masked off
                for (int rj = wave; rj < RJ; rj += WPB) {
                    const int gj = sj0 + rj;
                    if (gj < 0 || gj >= nlines) continue;
#pragma unroll
                    for (int k = 0; k < (RI + 63) / 64; ++k) {
                        const int ri = 64 * k + lane, gi = si0 + ri;
                        if (ri < RI && gi >= 0 && gi < len)
                            __builtin_amdgcn_global_load_lds(
                                (const FF_GLOBAL void*)(DB + ((size_t)gj * CS + gi) * 16),
                                (__attribute__((address_space(3))) void*)&region[rj * RI + 64 * k], 16, 0, 0);
                    }
                }
                ++gw;
            }
            while (active) {
                uint32_t pred[CH];
                bool need[CH];
                bool anyn = false;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (fwd) {
                        const uint32_t edge = c == 0 ? carry : (uint32_t)__builtin_amdgcn_readlane((int)h[c > 0 ? c - 1 : 0], 63);
                        pred[c] = lane_from_lower(h[c], edge);
                    } else {
                        const uint32_t edge = c == CH - 1 ? carry
                                                          : (uint32_t)__builtin_amdgcn_readlane((int)h[c < CH - 1 ? c + 1 : c], 0);
                        pred[c] = lane_from_higher(h[c], edge);
                    }
                    need[c] = hp[c] && pred[c] != lp[c];
                    anyn |= need[c];
                }
                if (!__any(anyn)) break;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (need[c]) {
                        const int p = w0 + 64 * c + lane;
                        lp[c] = pred[c];
                        le[c] = pred[c] == f0[c] ? c0[c]
                                                 : feat_cost<COL, CK>(DB, W, H, CS, COL ? line : p, COL ? p : line, pred[c], a[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) h[c] = le[c] < c0[c] ? lp[c] : f0[c];
            }
            carry = fwd ? (uint32_t)__builtin_amdgcn_readlane((int)h[CH - 1], 63)
                        : (uint32_t)__builtin_amdgcn_readlane((int)h[0], 0);

            if (STG && rs) {
                __builtin_amdgcn_s_waitcnt(0);                   // staged descriptors have landed in LDS
                __syncthreads();
            }

#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int p = w0 + 64 * c + lane;
                if (!(active && p < len)) continue;
                uint32_t bf = h[c];
                int32_t bc = le[c] < c0[c] ? le[c] : c0[c];
                const int x = COL ? line : p, y = COL ? p : line;
                if (rs) {
                    const FT ac = a[c];
                    if constexpr (STG) {
                        random_search<RC>(bf, bc, W, x, y, rlev, ctr2, sc, [&](uint32_t f) -> int32_t {
                            const int qx = x + flow_x(f), qy = y + flow_y(f);
                            if ((unsigned)qx >= (unsigned)W || (unsigned)qy >= (unsigned)H) return kInf;
                            const int ri = (COL ? qy : qx) - si0, rj = (COL ? qx : qy) - sj0;
                            if ((unsigned)ri < (unsigned)RI && (unsigned)rj < (unsigned)RJ)
                                return sad16(ac, region[rj * RI + ri]);
                            return sad16(ac, ld16(DB + pix<COL>(qx, qy, CS) * 16));
                        });
                    } else {
                        random_search<RC>(bf, bc, W, x, y, rlev, ctr2, sc,
                                          [&](uint32_t f) { return feat_cost<COL, CK>(DB, W, H, CS, x, y, f, ac); });
                    }
                }
                if (lout && lline.has(p)) lline.set(p, i32x2{(int)bf, bc});
                else S[p] = i32x2{(int)bf, bc};
            }
        }
    }
    if (xwc) {
        // WPB adjacent columns: for every row, WPB consecutive state entries
        __syncthreads();
        gi2* __restrict__ dst = (gi2*)L.state[dir];
        const int nl = min(WPB, nlines - line0);
        for (int e = threadIdx.x; e < WPB * len; e += 64 * WPB) {
            const int k = e % WPB, p = e / WPB;
            if (k < nl) dst[(uint32_t)p * (uint32_t)L.Wp + (uint32_t)(line0 + k)] = line_lds(k).get(p);
        }
    }
}

// State transpose between the row-major and column-major copies of every
// pair and direction at one level (32 x 32 tiles through LDS).
// to_t = 1: state -> stateT, grid (ceil(W/32), ceil(H/32), 2 * pairs);
// to_t = 0: stateT -> state, grid (ceil(H/32), ceil(W/32), 2 * pairs).
__global__ __launch_bounds__(256) void k_transpose_state(const PairDev* __restrict__ pairs, int level, int to_t)
{
    const PairDev& P = pairs[blockIdx.z >> 1];
    const int dir = blockIdx.z & 1;
    const LevelDev& L = P.lv[level];
    const int SW = to_t ? L.W : L.H, SH = to_t ? L.H : L.W;     // source is [SH][SW]
    const int sp = to_t ? L.Wp : L.H, dp = to_t ? L.H : L.Wp;   // source / destination row strides
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32;
    if (x0 >= SW || y0 >= SH) return;
    const int2* __restrict__ src = to_t ? L.state[dir] : L.stateT[dir];
    int2* __restrict__ dst = to_t ? L.stateT[dir] : L.state[dir];
    __shared__ int2 t[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int y = y0 + r, x = x0 + tx;
        if (y < SH && x < SW) t[r][tx] = src[(size_t)y * sp + x];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int xx = x0 + r, yy = y0 + tx;                     // destination is [SW][SH]
        if (xx < SW && yy < SH) dst[(size_t)xx * dp + yy] = t[tx][r];
    }
}

// ------------------------------------------------------- consistency ----
// Forward-backward check at level 0 (Sec. 3.1, threshold epsilon): p is kept
// when its match and the match of q = p + F(p) are valid and
// |F(p) + B(q)|^2 <= eps^2.  Writes the caller's flow / cost / mask.
// Consistency error |F(p) + B(q)|^2, q = p + F(p); INF when either match is
// invalid (a finite cost means q lies inside the image).  mask = err <= eps^2.
// Flows in 1 / 2^shift pixels (shift 2 after the sub-pixel refinement): q is
// then rounded half up to whole pixels and the error is in 1 / 4^shift px^2.
__device__ __forceinline__ int32_t fb_err(const gi2* __restrict__ other, int Wp, int x, int y, i32x2 s, int shift)
{
    if (s.y == kInf) return kInf;
    const uint32_t F = (uint32_t)s.x;
    const int half = shift ? 1 << (shift - 1) : 0;
    const int qx = x + ((flow_x(F) + half) >> shift), qy = y + ((flow_y(F) + half) >> shift);
    const i32x2 t = other[(uint32_t)qy * (uint32_t)Wp + (uint32_t)qx];
    if (t.y == kInf) return kInf;
    const int ex = flow_x(F) + flow_x((uint32_t)t.x), ey = flow_y(F) + flow_y((uint32_t)t.x);
    return ex * ex + ey * ey;
}

// The consistency kernels: four pixels per thread, 64 apart, so that a wave
// covers 256 consecutive pixels and each of its load, gather and store
// instructions touches 64 consecutive ones (the gathers at q = p + F(p) of
// neighbouring lanes then share cache lines).  Neighbouring blocks run on
// one XCD, so those gathers find the other field's rows in the L2 that
// fetched them.  TWO: the two-check form (own = the first search's field,
// inverse fields = the first search's and the second search's).  The error
// plane is written when the table holds one.  grid (pixels / 1024, 2 * pairs).
template <bool TWO>
__device__ __forceinline__ void fb_pixels(const PairDev* __restrict__ pairs, int eps2, int shift)
{
    const int lb = xcd_remap(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
    const int bx = lb % gridDim.x, by = lb / gridDim.x;
    const PairDev& P = pairs[by >> 1];
    const int dir = by & 1;
    const LevelDev& L = P.lv[0];
    const int W = L.W, n = L.W * L.H;
    const int i0 = bx * 1024 + (threadIdx.x >> 6) * 256 + (threadIdx.x & 63);
    if (i0 >= n) return;
    const gi2* __restrict__ own = (const gi2*)(TWO ? P.save[dir] : L.state[dir]);
    const gi2* __restrict__ inv1 = (const gi2*)(TWO ? P.save[dir ^ 1] : L.state[dir ^ 1]);
    const gi2* __restrict__ inv2 = (const gi2*)L.state[dir ^ 1];
    FF_GLOBAL uint32_t* fl = (FF_GLOBAL uint32_t*)P.flow[dir];
    FF_GLOBAL int32_t* co = (FF_GLOBAL int32_t*)P.cost[dir];
    FF_GLOBAL uint8_t* mk = (FF_GLOBAL uint8_t*)P.mask[dir];
    FF_GLOBAL int32_t* er = (FF_GLOBAL int32_t*)P.fberr[dir];
    const int Wp = L.Wp;                                         // state rows are Wp apart
    i32x2 st[4];
    int px[4], py[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int i = i0 + 64 * k;
        py[k] = i / W;
        px[k] = i - py[k] * W;
        st[k] = i < n ? own[(uint32_t)py[k] * (uint32_t)Wp + (uint32_t)px[k]] : i32x2{0, kInf};   // INF: nothing gathered
    }
    int32_t e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t e1 = fb_err(inv1, Wp, px[k], py[k], st[k], shift);
        e[k] = TWO ? max(e1, fb_err(inv2, Wp, px[k], py[k], st[k], shift)) : e1;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t i = (uint32_t)(i0 + 64 * k);
        if ((int)i >= n) continue;
        if (fl) fl[i] = (uint32_t)st[k].x;
        if (co) co[i] = st[k].y;
        if (mk) mk[i] = e[k] <= eps2 ? 1 : 0;
        if (er) er[i] = e[k];
    }
}

// Forward-backward check of one search (Sec. 3.1).
__global__ __launch_bounds__(256) void k_fb(const PairDev* __restrict__ pairs, int eps2, int shift)
{
    fb_pixels<false>(pairs, eps2, shift);
}

// ---------------------------------------------- sub-pixel refinement ----
// Level-0 flows of both directions to quarter pixels; costs are unchanged
// (a whole-pixel target has zero fraction).  grid (pixels / 256, 2 * pairs).
__global__ __launch_bounds__(256) void k_to_quarter(const PairDev* __restrict__ pairs)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int dir = blockIdx.y & 1;
    const LevelDev& L = P.lv[0];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= L.W * L.H) return;
    const int y = i / L.W, x = i - y * L.W;
    gi2* s = (gi2*)L.state[dir] + ((size_t)y * L.Wp + x);
    const uint32_t f = (uint32_t)(*s).x;
    (*s).x = (int)pack_flow(4 * flow_x(f), 4 * flow_y(f));
}

// --------------------------------------------- second consistency check --
// Keep the first search's level-0 state while the second search (keyed by
// seed2) reuses the state planes.  grid (pixels / 256, 2 * pairs).
__global__ __launch_bounds__(256) void k_save_state(const PairDev* __restrict__ pairs)
{
    const PairDev& P = pairs[blockIdx.y >> 1];
    const int dir = blockIdx.y & 1;
    const LevelDev& L = P.lv[0];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= L.W * L.H) return;
    const size_t j = (size_t)(i / L.W) * L.Wp + (size_t)(i % L.W);  // both planes rows Wp apart
    ((gi2*)P.save[dir])[j] = ((const gi2*)L.state[dir])[j];
}

// Two consistency checks (Sec. 3.1): p of the first search's field F is
// checked against the first search's inverse field B and the second
// search's B2; the error is the larger of the two (INF when either match is
// invalid) and the mask is error <= eps^2.  Flow and cost come from the first
// search.  grid (pixels / 1024, 2 * pairs).
__global__ __launch_bounds__(256) void k_fb2(const PairDev* __restrict__ pairs, int eps2, int shift)
{
    fb_pixels<true>(pairs, eps2, shift);
}

// ----------------------------------------------------- sparsification --
// Sec. 3.1 (minimum matches s from Table 3): the level-0 image is cut into
// 3x3 blocks from the origin, partial at the right and bottom borders.  A
// block with at least s consistent matches (error <= eps^2) keeps the one of
// lowest error, the lowest y*W + x among equals; all nine keep bytes of the
// block are written.  A wave covers kSparseBands bands of 3 rows over 63
// columns (21 blocks per band; lane 63 idle): each lane reads and writes its
// own column, so every load and store instruction touches 63 consecutive
// pixels of a row, and all the wave's loads are in flight together.  Per
// band a lane folds its column into a count and the smallest key (error << 4
// | 3 dy + dx; error <= eps^2 <= 2^24, so the key fits), and the block's
// three lanes combine theirs with shuffles.
// grid (ceil(ceil(W/63)/4), ceil(H/(3 kSparseBands)), 2 * pairs)
constexpr int kSparseBands = 4;

__global__ __launch_bounds__(256) void k_sparse(const PairDev* __restrict__ pairs, int eps2, int s)
{
    const PairDev& P = pairs[blockIdx.z >> 1];
    const int dir = blockIdx.z & 1;
    FF_GLOBAL uint8_t* keep = (FF_GLOBAL uint8_t*)P.sparse[dir];
    if (!keep) return;                                           // output not requested
    const LevelDev& L = P.lv[0];
    const int W = L.W, H = L.H;
    const int lane = threadIdx.x & 63;
    const int x0 = (blockIdx.x * 4 + (int)(threadIdx.x >> 6)) * 63, y0 = 3 * kSparseBands * blockIdx.y;
    if (x0 >= W || y0 >= H) return;                              // uniform per wave
    const int x = x0 + lane, dx = lane % 3, lead = lane - dx;     // lead: the block's first lane
    const bool col = lane < 63 && x < W;
    const FF_GLOBAL int32_t* err = (const FF_GLOBAL int32_t*)P.fberr[dir];
    int32_t e[3 * kSparseBands];
#pragma unroll
    for (int r = 0; r < 3 * kSparseBands; ++r)
        e[r] = col && y0 + r < H ? err[(uint32_t)(y0 + r) * (uint32_t)W + (uint32_t)x] : kInf;
#pragma unroll
    for (int band = 0; band < kSparseBands; ++band) {
        const int yb = y0 + 3 * band;
        if (yb >= H) break;                                      // uniform
        int count = 0;
        uint32_t key = 0xFFFFFFFFu;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
            if (e[3 * band + dy] <= eps2) {
                ++count;
                key = min(key, ((uint32_t)e[3 * band + dy] << 4) | (uint32_t)(3 * dy + dx));
            }
        const int total = __shfl(count, lead, 64) + __shfl(count, lead + 1, 64) + __shfl(count, lead + 2, 64);
        const uint32_t kb = min(min((uint32_t)__shfl((int)key, lead, 64), (uint32_t)__shfl((int)key, lead + 1, 64)),
                                (uint32_t)__shfl((int)key, lead + 2, 64));
        const int best = total >= s && kb != 0xFFFFFFFFu ? (int)(kb & 15u) : -1;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
            if (col && yb + dy < H)
                keep[(uint32_t)(yb + dy) * (uint32_t)W + (uint32_t)x] = 3 * dy + dx == best ? 1 : 0;
    }
}

// ------------------------------------------------------------- debug ----
// Descriptors of one level as signed bytes, packed [H][W][16] (the plane's
// rows are Wp entries apart).
__global__ void k_copy_desc_signed(const uint8_t* __restrict__ src, int8_t* __restrict__ dst, int W, int H, int Wp)
{
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (size_t)W * H * 16) return;
    const size_t px = i >> 4, y = px / (size_t)W, x = px - y * (size_t)W;
    dst[i] = (int8_t)(src[(y * (size_t)Wp + x) * 16 + (i & 15)] ^ 0x80u);
}

__global__ void k_keys_to_index(const unsigned long long* __restrict__ keys, int32_t* __restrict__ dst, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = (int32_t)(0xFFFFFFFFu - (uint32_t)keys[i]);
}

// ------------------------------------------- allocation-free scratch ----
// Workspace of ff_match_pair_noalloc: one pair's pyramids, descriptors,
// search state and seed tables plus its device table, in a fixed array that
// every GPU the library runs on holds until the process ends.  In host code
// the array's name is only a stand-in for the device address: the address
// comes from hipGetSymbolAddress, taken once per device (with that device
// current) when a handle is created there, and only that address is handed
// to kernels and copies.  Calls on one device are ordered through an event
// recorded after each call (the next call's stream waits for it) under a
// host lock, so calls from several streams, handles or threads never use the
// array at the same time.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_setup;
std::mutex g_scratch_use[kNoAllocDevices];
void* g_scratch_ptr[kNoAllocDevices];
hipEvent_t g_scratch_done[kNoAllocDevices];
}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Once per device, with `device` current: the array's device address and
// the event that orders the calls using it.
hipError_t noalloc_setup(int device)
{
    if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_setup);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return e != hipSuccess ? e : hipErrorInvalidSymbol;
    }
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_scratch_done[device] = ev;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

bool noalloc_lookup(int device, void** ptr, hipEvent_t* done)
{
    if (device < 0 || device >= kNoAllocDevices) return false;
    std::lock_guard<std::mutex> g(g_scratch_setup);
    *ptr = g_scratch_ptr[device];
    *done = g_scratch_done[device];
    return *ptr != nullptr;
}

void noalloc_lock(int device) { g_scratch_use[device].lock(); }
void noalloc_unlock(int device) { g_scratch_use[device].unlock(); }

// ------------------------------------------------------------ launchers --
#define FF_GRID1(n) dim3((unsigned)(((n) + 255) / 256))

// Blocks per image of the per-pixel kernels (grid (blocks, 2 * pairs), each
// block striding over its image): enough to cover the largest image in one
// pass, but for batches of many small images at most what keeps the grid
// near kPixelBlocks, so that blocks are not mostly started and retired.
constexpr long long kPixelBlocks = 16384;
unsigned blocks_per_image(long long natural, int npairs)
{
    const long long cap = std::max<long long>(1, kPixelBlocks / (2LL * npairs));
    return (unsigned)std::max<long long>(1, std::min(natural, cap));
}
void launch_gray(const PairDev* d, int npairs, int maxpx, hipStream_t st)
{
    const long long groups = (maxpx + 15) / 16;                  // threads of 16 pixels
    hipLaunchKernelGGL(k_gray, dim3(blocks_per_image((groups + 255) / 256, npairs), 2 * npairs), dim3(256), 0, st, d);
}
void launch_down2(const PairDev* d, int npairs, int level, int maxpx, hipStream_t st)
{
    hipLaunchKernelGGL(k_down2, dim3(blocks_per_image((maxpx + 255) / 256, npairs), 2 * npairs), dim3(256), 0, st, d,
                       level);
}
void launch_desc(const PairDev* d, int npairs, int level, int maxW, int maxH, hipStream_t st)
{
    const dim3 grid((maxW + kDescTX - 1) / kDescTX, (maxH + kDescTY - 1) / kDescTY, 2 * npairs);
    if (level == 0) hipLaunchKernelGGL(k_desc<true>, grid, dim3(256), 0, st, d, level);
    else hipLaunchKernelGGL(k_desc<false>, grid, dim3(256), 0, st, d, level);
}
void launch_census(const PairDev* d, int npairs, int level, int maxW, int maxH, hipStream_t st)
{
    hipLaunchKernelGGL(k_census, dim3((maxW + kCenTX - 1) / kCenTX, (maxH + kCenTY - 1) / kCenTY, 2 * npairs),
                       dim3(256), 0, st, d, level);
}
void launch_seed_resolve(const PairDev* d, int npairs, int level, int stride, int maxQ, hipStream_t st)
{
    hipLaunchKernelGGL(k_seed_resolve, dim3(blocks_per_image((maxQ + 63) / 64, npairs), 2 * npairs), dim3(256), 0, st, d,
                       level, stride);
}
void launch_seed_records(const PairDev* d, int npairs, int level, int maxN, hipStream_t st)
{
    hipLaunchKernelGGL(k_seed_records, dim3(blocks_per_image((maxN + 255) / 256, npairs), 2 * npairs), dim3(256), 0, st,
                       d, level);
}
// Database splits: few, so that each block streams a long split and pays its
// prologue, first chunk and epilogue rarely, yet enough to fill the GPU's
// block slots (four 256-thread blocks per CU at the kernel's register
// count) in whole rounds: among 1x..4x the smallest count that fills the
// slots once, the one wasting the fewest slots in its last round (the
// smaller on ties); whole chunks per split and at most 2048 chunks per split
// (the chunk tag's range).
void launch_seed_nn(const PairDev* d, int npairs, int level, int stride, int maxQ, int maxN, hipStream_t st)
{
    constexpr int MQ = 4;
    constexpr long long kSlots = 256 * 5;
    const int qblocks = (maxQ + 4 * 16 * MQ - 1) / (4 * 16 * MQ);
    const int nchunks = (maxN + 16 * kSeedChunk - 1) / (16 * kSeedChunk);
    const long long per_split = (long long)qblocks * 2 * npairs;
    const long long s0 = std::max<long long>({1, (kSlots + per_split - 1) / per_split, (nchunks + 2047) / 2048});
    long long splits = std::min<long long>(s0, nchunks);
    double best_eff = -1.0;
    for (long long s = s0; s <= 4 * s0 && s <= nchunks; ++s) {
        const long long blocks = s * per_split, rounds = (blocks + kSlots - 1) / kSlots;
        const double eff = (double)blocks / (double)(rounds * kSlots);
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            splits = s;
        }
    }
    const int cps = (int)((nchunks + splits - 1) / splits);      // chunks per split
    const int tps = cps * kSeedChunk;
    const int nsplit = ((maxN + 15) / 16 + tps - 1) / tps;
    hipLaunchKernelGGL(k_seed_nn<MQ>, dim3(qblocks, nsplit, 2 * npairs), dim3(256), 0, st, d, level, stride, tps);
}
void launch_init(const PairDev* d, int npairs, int level, int coarsest, int stride, int census, int maxpx,
                 hipStream_t st)
{
    hipLaunchKernelGGL(k_init, dim3((maxpx + 255) / 256, 2 * npairs), dim3(256), 0, st, d, level, coarsest, stride,
                       census);
}
// A line phase keeps its WPB lines' state in LDS (6 bytes a pixel) between
// its passes when they fit in 64 KiB (lines up to 1365 px at 8 lines per
// block, 2730 px at 4).
constexpr size_t kLdsBytesPerPx = 6;
bool line_cross_write(int wpb, int maxlen)
{
    return (size_t)wpb * (size_t)maxlen * kLdsBytesPerPx <= 65536;
}

// Pixels of a row held in LDS: as many whole windows as let 24 waves per CU
// share the CU's 160 KiB of LDS (sizing for the 28 that the registers allow
// measured slower: more of each row goes through global memory); the rest of
// a longer row goes through global memory between the passes.
template <int CH, int WPB>
int row_lds_pixels(int maxlen)
{
    constexpr int kWaves = 24, blocks = (kWaves + WPB - 1) / WPB;
    constexpr int cap = (int)(160 * 1024 / blocks / WPB / kLdsBytesPerPx) / (64 * CH) * (64 * CH);
    static_assert(cap >= 64 * CH, "at least one window per row in LDS");
    return maxlen < cap ? maxlen : cap;
}

template <int RC, bool COL, int CH, int WPB, bool STG, int CK>
void launch_line_t(const PairDev* d, int npairs, int level, int iter, int upto, const SearchConst& sc, int nlines,
                   int maxlen, int finit, const LineWork& wk, int lock, hipStream_t st)
{
    const int xw = !line_cross_write(WPB, maxlen) ? 0 : COL ? maxlen : row_lds_pixels<CH, WPB>(maxlen);
    const size_t dyn = (size_t)WPB * xw * kLdsBytesPerPx;
    const dim3 grid = wk.items ? dim3((unsigned)wk.n) : dim3((nlines + WPB - 1) / WPB, 2 * npairs);
    hipLaunchKernelGGL((k_line_phase<RC, COL, CH, WPB, STG, CK>), grid, dim3(64 * WPB), dyn, st, d, level, iter, upto,
                       sc, xw, finit, wk.items, lock);
}

template <int RC, bool COL, int CK>
bool launch_line_rc(int ch, int wpb, int stg, const PairDev* d, int npairs, int level, int iter, int upto,
                    const SearchConst& sc, int nlines, int maxlen, int finit, const LineWork& wk, hipStream_t st)
{
    // stg: 0 free-running, 1 staged (lockstep, LDS neighbourhood), 2 lockstep
    // (the pipelined pass's windows; the other passes run free)
#define FF_LINE_CASE(C, B, G)                                                                        \
    if (ch == C && wpb == B && (stg == G || (G == 0 && stg == 2))) {                                 \
        launch_line_t<RC, COL, C, B, G != 0, CK>(d, npairs, level, iter, upto, sc, nlines, maxlen, finit, wk, \
                                                 stg == 2 ? 1 : 0, st);                              \
        return true;                                                                                 \
    }
    if constexpr (CK == 2) {                                     // the refinement's fixed schedule
        FF_LINE_CASE(1, 4, 0) FF_LINE_CASE(1, 8, 0)
    } else {
        FF_LINE_CASE(1, 2, 0) FF_LINE_CASE(1, 4, 0) FF_LINE_CASE(1, 8, 0)
        FF_LINE_CASE(2, 2, 0) FF_LINE_CASE(2, 4, 0) FF_LINE_CASE(2, 8, 0)
        FF_LINE_CASE(4, 2, 0) FF_LINE_CASE(4, 4, 0) FF_LINE_CASE(4, 8, 0)
        FF_LINE_CASE(8, 2, 0) FF_LINE_CASE(8, 4, 0) FF_LINE_CASE(8, 8, 0)
    }
    if constexpr (CK == 0) {
        FF_LINE_CASE(1, 4, 1) FF_LINE_CASE(1, 8, 1) FF_LINE_CASE(1, 16, 1) FF_LINE_CASE(2, 8, 1)
    }
#undef FF_LINE_CASE
    return false;
}

template <int CK>
bool launch_line_ck(bool col, int ch, int wpb, int stg, const PairDev* d, int npairs, int level, int iter,
                    int upto, const SearchConst& sc, int nlines, int maxlen, int finit, const LineWork& wk,
                    hipStream_t st)
{
    if constexpr (CK == 2) {
        // the refinement: radius 2 (two trials) unrolled, so both trials'
        // neighbourhood loads are in flight together; other radii in a loop
        if (sc.radius == 2)
            return col ? launch_line_rc<2, true, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, 0,
                                                     wk, st)
                       : launch_line_rc<2, false, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen,
                                                      finit, wk, st);
        return col ? launch_line_rc<0, true, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, 0, wk,
                                                 st)
                   : launch_line_rc<0, false, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, finit,
                                                  wk, st);
    } else {
        if (sc.radius == 16)
            return col ? launch_line_rc<16, true, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, 0,
                                                      wk, st)
                       : launch_line_rc<16, false, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen,
                                                       finit, wk, st);
        return col ? launch_line_rc<0, true, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, 0, wk,
                                                 st)
                   : launch_line_rc<0, false, CK>(ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, 0, wk,
                                                  st);
    }
}

// One row or column phase of every pair and direction at one level.  ch =
// chunks of 64 px per relaxation window, wpb = lines per block, stg = staged
// random search, ck = cost (0 descriptor SAD, 1 Census, 2 sub-pixel SAD on
// quarter-pixel flows: generic pass, (ch, wpb) in {(1, 4), (1, 8)} only);
// supported: stg 0 with ch in {1, 2, 4, 8} and wpb in {2, 4, 8} (ch <= 2
// runs the software-pipelined pass at radius 16); stg 1, descriptor cost
// only, with (ch, wpb) in {(1, 4), (1, 8), (1, 16), (2, 8)}.  Returns false
// otherwise.
// nlines / maxlen: the batch's largest line count and line length.  The
// column phase reads the row-major state and, when line_cross_write()
// allows it, also writes it (otherwise its result stays in stateT).
// finit: the row phase of iteration 0 computes the level init itself (the
// first pass loads each pixel's init flow and costs it instead of reading a
// state written by k_init); only the software-pipelined pass supports it --
// see line_fused_init().
// wk: the batch's work list for this phase and level (items null: the 2-D
// grid over the batch's largest line count).
bool launch_line_phase(bool col, int ch, int wpb, int stg, int ck, const PairDev* d, int npairs, int level,
                       int iter, int upto, const SearchConst& sc, int nlines, int maxlen, int finit,
                       const LineWork& wk, hipStream_t st)
{
    if (ck == 2)
        return stg == 0 &&
               launch_line_ck<2>(col, ch, wpb, 0, d, npairs, level, iter, upto, sc, nlines, maxlen, finit, wk, st);
    return ck ? launch_line_ck<1>(col, ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, finit, wk, st)
              : launch_line_ck<0>(col, ch, wpb, stg, d, npairs, level, iter, upto, sc, nlines, maxlen, finit, wk, st);
}

// Whether the row phase with this schedule can take over the level init.
bool line_fused_init(int ch, int stg, const SearchConst& sc)
{
    return sc.radius == 16 && stg != 1 && ch <= 2;
}
void launch_transpose_state(const PairDev* d, int npairs, int level, int to_t, int maxW, int maxH, hipStream_t st)
{
    const int sw = to_t ? maxW : maxH, sh = to_t ? maxH : maxW;
    hipLaunchKernelGGL(k_transpose_state, dim3((sw + 31) / 32, (sh + 31) / 32, 2 * npairs), dim3(256), 0, st, d,
                       level, to_t);
}
void launch_fb(const PairDev* d, int npairs, int eps2, int shift, int maxpx, hipStream_t st)
{
    hipLaunchKernelGGL(k_fb, dim3((maxpx + 1023) / 1024, 2 * npairs), dim3(256), 0, st, d, eps2, shift);
}
void launch_to_quarter(const PairDev* d, int npairs, int maxpx, hipStream_t st)
{
    hipLaunchKernelGGL(k_to_quarter, dim3((maxpx + 255) / 256, 2 * npairs), dim3(256), 0, st, d);
}
void launch_save_state(const PairDev* d, int npairs, int maxpx, hipStream_t st)
{
    hipLaunchKernelGGL(k_save_state, dim3((maxpx + 255) / 256, 2 * npairs), dim3(256), 0, st, d);
}
void launch_fb2(const PairDev* d, int npairs, int eps2, int shift, int maxpx, hipStream_t st)
{
    hipLaunchKernelGGL(k_fb2, dim3((maxpx + 1023) / 1024, 2 * npairs), dim3(256), 0, st, d, eps2, shift);
}
void launch_sparse(const PairDev* d, int npairs, int eps2, int s, int maxW, int maxH, hipStream_t st)
{
    const int waves = (maxW + 62) / 63, nby = (maxH + 3 * kSparseBands - 1) / (3 * kSparseBands);
    hipLaunchKernelGGL(k_sparse, dim3((waves + 3) / 4, nby, 2 * npairs), dim3(256), 0, st, d, eps2, s);
}
void launch_copy_desc_signed(const uint8_t* src, int8_t* dst, int W, int H, int Wp, hipStream_t st)
{
    const size_t n = (size_t)W * H * 16;
    hipLaunchKernelGGL(k_copy_desc_signed, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, W, H, Wp);
}
void launch_keys_to_index(const unsigned long long* keys, int32_t* dst, int n, hipStream_t st)
{
    hipLaunchKernelGGL(k_keys_to_index, dim3((n + 255) / 256), dim3(256), 0, st, keys, dst, n);
}

}  // namespace ff
