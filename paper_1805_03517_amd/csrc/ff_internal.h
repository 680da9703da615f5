// ff_internal.h -- device-side layout of one batch, shared by the HIP kernels
// and the host runtime of libff (nothing outside libff includes it).
//
// HBM layout per pair (all buffers 256-byte aligned, carved from one arena):
//   gray[l][i]   uint8  [H_l][W_l]        pyramid level l of image i
//   desc[l][i]   uint8  [H_l][Wp_l][16]   descriptors, stored biased (d + 128),
//                                         rows padded to Wp_l entries
//                                         so the SAD unit works on unsigned bytes
//   descT[l][i]  uint8  [W_l][Hp_l][16]   the same descriptors column-major; each
//                                         column padded to Hp_l = H_l rounded up to
//                                         16 entries, so every column starts on a
//                                         128-byte line (padding never read)
//   state[l][d]  int2   [H_l][Wp_l]       search state of direction d, rows padded
//                                         to Wp_l = W_l rounded up to 16 entries
//                                         (every row of every row-major plane then
//                                         starts on a 128-byte line; padding never
//                                         read):
//                                         .x = flow (int16 dx | int16 dy << 16),
//                                         .y = cost (INT32_MAX = invalid)
//   stateT[l][d] int2   [W_l][H_l]        column-major copy used by the column phase
//   dbrec[i]     int8   [N][64]           seed-search database records of image i
//                                         at the coarsest level (see k_seed_records)
//   keys[d]      uint64 [nsy][nsx]        packed (score, ~index) of the best seed match
// The column phase runs the same line kernel as the row phase on the
// column-major copies, so its lanes walk consecutive y with coalesced loads.
#pragma once
#include <stdint.h>

namespace ff {

constexpr int kMaxLevels = 8;
constexpr int kMaxSide = 8192;
constexpr int32_t kInf = 0x7FFFFFFF;
// Column stride of the column-major feature planes: H rounded up to 16
// entries, so that every column starts on a 128-byte line.
inline int padded_height(int H) { return (H + 15) & ~15; }
// Row stride of the row-major state, descriptor and Census planes: W rounded
// up to 16, so that every row starts on a 128-byte line.
inline int padded_width(int W) { return (W + 15) & ~15; }

struct LevelDev {
    int W, H;
    int Hp;                          // column stride of descT / cenT (H rounded up to 16)
    int Wp;                          // row stride of state, desc and cen (W rounded up to 16)
    uint8_t* gray[2];
    uint8_t* desc[2];
    uint8_t* descT[2];
    int2* state[2];
    int2* stateT[2];
    uint8_t* cen[2];                 // 7x7 Census strings, u64 per pixel, rows Wp apart (Census cost only)
    uint8_t* cenT[2];                // column-major copy, columns Hp apart
};

struct PairDev {
    const uint8_t* img[2];
    int C;
    int nsx, nsy;                    // seed grid at the coarsest level
    LevelDev lv[kMaxLevels];
    int8_t* dbrec[2];
    unsigned long long* keys[2];
    int16_t* flow[2];                // outputs (fwd, bwd); bwd entries may be null
    int32_t* cost[2];
    uint8_t* mask[2];
    int32_t* fberr[2];               // consistency error (caller's buffer, or the workspace's when sparsifying)
    uint8_t* sparse[2];              // 3x3-block selection (caller's); null = not computed
    int2* save[2];                   // first search's level-0 state (second consistency check)
};

// A line phase's work list over a batch (device memory; see k_line_phase):
// n items pair-direction << 16 | line block, or items null.
struct LineWork {
    const uint32_t* items;
    int n;
};

struct SearchConst {
    int levels;
    int stride;
    int iters;
    int radius;
    int trials;                      // floor(log2 radius) + 1, 0 when radius == 0
    int eps2;
    uint32_t key0, key1;             // Philox key words
    int rng_level;                   // >= 0: level word of the Philox counter (sub-pixel refinement)
};

}  // namespace ff
