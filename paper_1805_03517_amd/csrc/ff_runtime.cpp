// ff_runtime.cpp -- host runtime of libff: handle, workspace arena, batch
// planner and the C ABI declared in include/ff.h.
//
// A call validates its pairs, sizes the workspace for the batch (one arena,
// grown on demand and kept), writes the per-pair device table, and enqueues
// the fixed launch sequence on the caller's stream:
//   gray -> pyramid (L-1) -> descriptors (L) -> seed records -> seed NN
//   -> for each level, coarsest first: init, then iters x (row phase,
//      state -> column-major, col phase, state -> row-major)
//   -> forward-backward check.
// Every launch covers all pairs of the batch, so a batch costs the same
// number of launches as one pair.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ff.h"
#include "ff_internal.h"

namespace ff {
void launch_gray(const PairDev*, int, int, hipStream_t);
void launch_down2(const PairDev*, int, int, int, hipStream_t);
void launch_desc(const PairDev*, int, int, int, int, hipStream_t);
void launch_seed_records(const PairDev*, int, int, int, hipStream_t);
void launch_seed_nn(const PairDev*, int, int, int, int, int, hipStream_t);
void launch_seed_resolve(const PairDev*, int, int, int, int, hipStream_t);
void launch_init(const PairDev*, int, int, int, int, int, int, hipStream_t);
void launch_census(const PairDev*, int, int, int, int, hipStream_t);
bool launch_line_phase(bool, int, int, int, int, const PairDev*, int, int, int, int, const SearchConst&, int, int,
                       int, const LineWork&, hipStream_t);
bool line_fused_init(int ch, int stg, const SearchConst& sc);
bool line_cross_write(int wpb, int maxlen);
void launch_transpose_state(const PairDev*, int, int, int, int, int, hipStream_t);
void launch_fb(const PairDev*, int, int, int, int, hipStream_t);
void launch_to_quarter(const PairDev*, int, int, hipStream_t);
void launch_sparse(const PairDev*, int, int, int, int, int, hipStream_t);
void launch_save_state(const PairDev*, int, int, hipStream_t);
void launch_fb2(const PairDev*, int, int, int, int, hipStream_t);
void launch_copy_desc_signed(const uint8_t*, int8_t*, int, int, int, hipStream_t);
void launch_keys_to_index(const unsigned long long*, int32_t*, int, hipStream_t);
size_t noalloc_scratch_bytes();
hipError_t noalloc_setup(int device);
bool noalloc_lookup(int device, void** ptr, hipEvent_t* done);
void noalloc_lock(int device);
void noalloc_unlock(int device);
}  // namespace ff

using namespace ff;

// Launch geometry of one batch: the largest level sizes over its pairs.
struct Dims {
    int n = 0;
    int maxW[kMaxLevels] = {0}, maxH[kMaxLevels] = {0}, maxPx[kMaxLevels] = {0};
    int maxQ = 0;
    // the line phases' work lists (phase 0 rows, 1 columns) for a batch of
    // uneven pairs: nitems blocks, at byte offset item_off in the device
    // table; nitems 0 = the 2-D grid over the largest pair
    int nitems[2][kMaxLevels] = {{0}};
    size_t item_off[2][kMaxLevels] = {{0}};
};

struct ff_ctx {
    ff_params prm{};
    int device = 0;
    std::string err;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    PairDev* d_table = nullptr;      // device copy of the per-pair table (and the work lists after it)
    size_t d_table_cap = 0;          // bytes
    // pinned staging ring for table uploads: the host refills slot k only
    // after the copy that last read it has finished, so it can run several
    // calls ahead of the device
    static constexpr int kStaging = 4;
    char* h_table[kStaging] = {};
    size_t h_table_cap[kStaging] = {};   // bytes
    hipEvent_t table_ev[kStaging] = {};
    unsigned staging_next = 0;
    // captured launch sequences, keyed by the batch's launch geometry
    struct GraphEntry {
        std::vector<long long> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<GraphEntry> graphs;
    std::vector<std::vector<long long>> seen;   // geometries launched once, not yet captured
    hipStream_t cap_stream = nullptr;
    bool use_graphs = true;
    std::vector<char> last;          // what d_table holds now
    // the last call's pair array as the caller passed it, with its launch
    // geometry: a call with byte-identical pairs on the same arena reuses
    // the validated plan and the device table as they are
    std::vector<ff_pair> last_pairs;
    void* last_arena = nullptr;
    Dims last_dims;
    bool last_valid = false;
    unsigned last_tune_gen = 0;
    unsigned tune_gen = 0;           // bumped whenever the schedule changes (the work lists depend on it)
    // stream ordering between calls: every call records run_done on its
    // stream, and a call on another stream first waits for it, since all
    // calls share the arena and the device table
    hipEvent_t run_done = nullptr;
    hipStream_t run_stream = nullptr;
    bool run_any = false;
    // allocation fault injection (tests): with fault_after = n >= 0, the
    // first n device or pinned allocations made for this handle (its serving
    // lanes included) succeed and every later one fails as out of memory
    ff_ctx* fault_root = this;
    long long fault_after = -1;
    long long allocs = 0;
    // tracing: event pairs around every launch while enabled
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct ProfRec {
        int kernel, level;
        size_t ev;                                // first of its two events
    };
    std::vector<ProfRec> prof;
    struct ServeState* serve = nullptr;         // serving engine, created on first use
    // line-kernel schedule per phase (0 row, 1 col) and level: chunks of 64 px
    // per relaxation window, lines per block and LDS staging of the random
    // search (set by ff_autotune / ff_tune_set)
    int tune_ch[2][kMaxLevels] = {{1, 1, 1, 1, 1, 1, 1, 1}, {1, 1, 1, 1, 1, 1, 1, 1}};
    int tune_wpb[2][kMaxLevels] = {{4, 4, 4, 4, 4, 4, 4, 4}, {8, 8, 8, 8, 8, 8, 8, 8}};
    int tune_stg[2][kMaxLevels] = {};          // mode: 0 free-running, 1 staged LDS neighbourhood, 2 lockstep windows
};

// Serving: continuous batching over `lanes` concurrent cohorts.  Each lane
// owns a stream, a completion event and a sub-context (its own arena and
// pair table).  Submitted requests wait in a FIFO; whenever a lane is idle
// the requests at the head of the FIFO that fit the lane's arena form a
// cohort and run as one grouped batch on that lane's stream, overlapping
// with the cohorts already running on the other lanes.
struct ServeReq {
    ff_pair pair;
    uint64_t tag;
    size_t bytes;
    hipEvent_t ready;                // recorded on the submitter's stream
};
struct ServeLane {
    ff_ctx* exec = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> tags;
};
struct ServeState {
    std::vector<ServeLane> lanes;
    size_t lane_bytes = 0;
    int max_cohort = 0;
    std::deque<ServeReq> pending;
    std::deque<uint64_t> done;
    std::vector<hipEvent_t> ev_pool;
};

namespace {

const char* g_static_err = "invalid handle";

ff_status fail(ff_ctx* h, ff_status s, const std::string& msg)
{
    if (h) h->err = msg;
    return s;
}

ff_status hip_fail(ff_ctx* h, hipError_t e, const char* what)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return fail(h, FF_ERR_HIP, buf);
}

#define FF_HIP(h, call)                                   \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(h, e_, #call); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

struct PairPlan {
    int W[kMaxLevels], H[kMaxLevels];
    int nsx, nsy;
    size_t bytes;
};

PairPlan plan_pair(const ff_params& p, int W, int H)
{
    PairPlan pl{};
    size_t b = 0;
    for (int l = 0; l < p.levels; ++l) {
        pl.W[l] = l == 0 ? W : pl.W[l - 1] >> 1;
        pl.H[l] = l == 0 ? H : pl.H[l - 1] >> 1;
        const size_t n = (size_t)pl.W[l] * pl.H[l], nT = (size_t)pl.W[l] * padded_height(pl.H[l]),
                     nR = (size_t)padded_width(pl.W[l]) * pl.H[l];
        b += 2 * align_up(n);            // gray planes
        b += 2 * align_up(nR * 16) + 2 * align_up(nT * 16);   // descriptors, row- and column-major
        b += 2 * align_up(nR * 8) + 2 * align_up(n * 8);      // state, row- and column-major
        if (p.flags & FF_COST_CENSUS) b += 2 * align_up(nR * 8) + 2 * align_up(nT * 8);   // Census strings
    }
    const int c = p.levels - 1;
    pl.nsx = (pl.W[c] + p.seed_stride - 1) / p.seed_stride;
    pl.nsy = (pl.H[c] + p.seed_stride - 1) / p.seed_stride;
    b += 2 * align_up((size_t)pl.W[c] * pl.H[c] * 64);
    b += 2 * align_up((size_t)pl.nsx * pl.nsy * 8);
    if (p.flags & FF_SPARSIFY) b += 2 * align_up((size_t)W * H * 4);   // consistency errors
    if (p.flags & FF_SECOND_CHECK) b += 2 * align_up((size_t)padded_width(W) * H * 8);   // first search's level-0 state
    pl.bytes = b;
    return pl;
}

ff_status validate_params(ff_ctx* h, const ff_params& p)
{
    if (p.levels < 1 || p.levels > kMaxLevels) return fail(h, FF_ERR_INVALID, "levels must be in 1..8");
    if (p.seed_stride < 1 || p.seed_stride > 64) return fail(h, FF_ERR_INVALID, "seed_stride must be in 1..64");
    if (p.iters < 0 || p.iters > 64) return fail(h, FF_ERR_INVALID, "iters must be in 0..64");
    if (p.rs_radius < 0 || p.rs_radius > 1024) return fail(h, FF_ERR_INVALID, "rs_radius must be in 0..1024");
    if (p.fb_eps < 0 || p.fb_eps > 1024) return fail(h, FF_ERR_INVALID, "fb_eps must be in 0..1024");
    if (p.flags & ~(FF_SPARSIFY | FF_COST_CENSUS | FF_SECOND_CHECK | FF_SECOND_PARAMS | FF_SUBPIXEL))
        return fail(h, FF_ERR_INVALID, "unknown flag bits");
    if (p.flags & FF_SECOND_PARAMS) {
        if (!(p.flags & FF_SECOND_CHECK)) return fail(h, FF_ERR_INVALID, "FF_SECOND_PARAMS needs FF_SECOND_CHECK");
        if (p.iters2 < 0 || p.iters2 > 64) return fail(h, FF_ERR_INVALID, "iters2 must be in 0..64");
        if (p.rs_radius2 < 0 || p.rs_radius2 > 1024) return fail(h, FF_ERR_INVALID, "rs_radius2 must be in 0..1024");
    }
    if (p.flags & FF_SUBPIXEL) {
        if (p.flags & FF_COST_CENSUS) return fail(h, FF_ERR_INVALID, "FF_SUBPIXEL needs the descriptor cost");
        if (p.sub_iters < 1 || p.sub_iters > 16) return fail(h, FF_ERR_INVALID, "sub_iters must be in 1..16");
        if (p.sub_radius < 0 || p.sub_radius > 64) return fail(h, FF_ERR_INVALID, "sub_radius must be in 0..64");
    }
    if ((p.flags & FF_SPARSIFY) && (p.sparse_min < 1 || p.sparse_min > 9))
        return fail(h, FF_ERR_INVALID, "sparse_min must be in 1..9");
    return FF_OK;
}

ff_status validate_pair(ff_ctx* h, const ff_pair& q)
{
    const ff_params& p = h->prm;
    if (!q.img1 || !q.img2 || !q.flow_fwd || !q.mask_fwd)
        return fail(h, FF_ERR_INVALID, "img1, img2, flow_fwd and mask_fwd are required");
    if (q.channels != 1 && q.channels != 3) return fail(h, FF_ERR_INVALID, "channels must be 1 or 3");
    if (q.width < 1 || q.height < 1 || q.width > kMaxSide || q.height > kMaxSide)
        return fail(h, FF_ERR_INVALID, "width and height must be in 1..8192");
    if ((q.width >> (p.levels - 1)) < 1 || (q.height >> (p.levels - 1)) < 1)
        return fail(h, FF_ERR_INVALID, "image too small for the number of levels");
    if ((p.flags & FF_SUBPIXEL) && (q.width > 2048 || q.height > 2048))
        return fail(h, FF_ERR_INVALID, "FF_SUBPIXEL: quarter-pixel flows need width and height <= 2048");
    if (((uintptr_t)q.flow_fwd & 3) || ((uintptr_t)q.flow_bwd & 3) || ((uintptr_t)q.cost_fwd & 3) ||
        ((uintptr_t)q.cost_bwd & 3) || ((uintptr_t)q.fberr_fwd & 3) || ((uintptr_t)q.fberr_bwd & 3))
        return fail(h, FF_ERR_INVALID, "flow, cost and fberr outputs must be 4-byte aligned");
    if (p.flags & FF_SPARSIFY) {
        if (!q.sparse_fwd) return fail(h, FF_ERR_INVALID, "sparse_fwd is required with FF_SPARSIFY");
    } else if (q.sparse_fwd || q.sparse_bwd) {
        return fail(h, FF_ERR_INVALID, "sparse outputs need FF_SPARSIFY");
    }
    return FF_OK;
}

// Bytes the handle's serving lanes hold (0 when serving is not configured).
size_t serve_bytes(const ff_ctx* h);

// Every device or pinned allocation of the runtime goes through these two,
// which apply the handle's fault injection.
bool alloc_faulted(ff_ctx* h)
{
    ff_ctx* r = h->fault_root;
    if (r->fault_after >= 0 && r->allocs >= r->fault_after) return true;
    ++r->allocs;
    return false;
}

hipError_t dev_malloc(ff_ctx* h, void** p, size_t bytes)
{
    if (alloc_faulted(h)) return hipErrorOutOfMemory;
    return hipMalloc(p, bytes);
}

hipError_t pinned_malloc(ff_ctx* h, void** p, size_t bytes)
{
    if (alloc_faulted(h)) return hipErrorOutOfMemory;
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

ff_status ensure_arena(ff_ctx* h, size_t need, bool exact = false)
{
    // one budget per handle: its own arena and its serving lanes together
    const size_t lanes = serve_bytes(h);
    if (h->prm.hbm_budget && need + lanes > h->prm.hbm_budget) {
        char buf[200];
        snprintf(buf, sizeof buf, "workspace of %zu bytes (plus %zu held by serving lanes) exceeds the budget of %llu bytes",
                 need, lanes, (unsigned long long)h->prm.hbm_budget);
        return fail(h, FF_ERR_BUDGET, buf);
    }
    if (need <= h->arena_bytes) return FF_OK;
    if (h->arena) {
        FF_HIP(h, hipDeviceSynchronize());
        FF_HIP(h, hipFree(h->arena));
        h->arena = nullptr;
        h->arena_bytes = 0;
        h->last.clear();
        h->last_pairs.clear();
    }
    size_t want = exact ? need : need + need / 8;           // head-room against regrowth
    if (h->prm.hbm_budget) want = std::min<size_t>(want, h->prm.hbm_budget - lanes);
    hipError_t e = dev_malloc(h, &h->arena, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = dev_malloc(h, &h->arena, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            h->arena = nullptr;
            return fail(h, FF_ERR_OOM, "hipMalloc of the workspace arena failed");
        }
        h->arena_bytes = need;
    } else {
        h->arena_bytes = want;
    }
    return FF_OK;
}

// Fill the per-pair table: carve each pair's buffers out of the workspace
// at `base` (the handle's arena, or the allocation-free path's scratch).
void build_table(const ff_params& p, char* base, const ff_pair* pairs, int n, PairDev* tab, const PairPlan* plans)
{
    for (int i = 0; i < n; ++i) tab[i] = PairDev{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* r = base + off;
        off += align_up(bytes);
        return r;
    };
    for (int i = 0; i < n; ++i) {
        const PairPlan& pl = plans[i];
        PairDev& d = tab[i];
        d.img[0] = pairs[i].img1;
        d.img[1] = pairs[i].img2;
        d.C = pairs[i].channels;
        d.nsx = pl.nsx;
        d.nsy = pl.nsy;
        for (int l = 0; l < p.levels; ++l) {
            const size_t np = (size_t)pl.W[l] * pl.H[l];
            LevelDev& L = d.lv[l];
            L.W = pl.W[l];
            L.H = pl.H[l];
            L.Hp = padded_height(pl.H[l]);
            L.Wp = padded_width(pl.W[l]);
            const size_t npT = (size_t)L.W * L.Hp;
            for (int k = 0; k < 2; ++k) L.gray[k] = (uint8_t*)take(np);
            const size_t npR = (size_t)L.Wp * L.H;                 // row-major planes, rows Wp apart
            for (int k = 0; k < 2; ++k) L.desc[k] = (uint8_t*)take(npR * 16);
            for (int k = 0; k < 2; ++k) L.descT[k] = (uint8_t*)take(npT * 16);
            for (int k = 0; k < 2; ++k) L.state[k] = (int2*)take(npR * 8);
            for (int k = 0; k < 2; ++k) L.stateT[k] = (int2*)take(np * 8);
            if (p.flags & FF_COST_CENSUS) {
                for (int k = 0; k < 2; ++k) L.cen[k] = (uint8_t*)take(npR * 8);
                for (int k = 0; k < 2; ++k) L.cenT[k] = (uint8_t*)take(npT * 8);
            }
        }
        const int c = p.levels - 1;
        for (int k = 0; k < 2; ++k) d.dbrec[k] = (int8_t*)take((size_t)pl.W[c] * pl.H[c] * 64);
        for (int k = 0; k < 2; ++k) d.keys[k] = (unsigned long long*)take((size_t)pl.nsx * pl.nsy * 8);
        d.flow[0] = pairs[i].flow_fwd;
        d.flow[1] = pairs[i].flow_bwd;
        d.cost[0] = pairs[i].cost_fwd;
        d.cost[1] = pairs[i].cost_bwd;
        d.mask[0] = pairs[i].mask_fwd;
        d.mask[1] = pairs[i].mask_bwd;
        d.fberr[0] = pairs[i].fberr_fwd;
        d.fberr[1] = pairs[i].fberr_bwd;
        d.sparse[0] = pairs[i].sparse_fwd;
        d.sparse[1] = pairs[i].sparse_bwd;
        if (p.flags & FF_SECOND_CHECK)
            for (int k = 0; k < 2; ++k) d.save[k] = (int2*)take((size_t)padded_width(pl.W[0]) * pl.H[0] * 8);
        if (p.flags & FF_SPARSIFY) {
            const size_t np = (size_t)pl.W[0] * pl.H[0];
            for (int k = 0; k < 2; ++k) {
                int32_t* own = (int32_t*)take(np * 4);
                if (!d.fberr[k]) d.fberr[k] = own;
            }
        }
    }
}

ff_status upload_table(ff_ctx* h, const std::vector<char>& tab, hipStream_t st)
{
    const size_t n = tab.size();                       // bytes
    if (h->last.size() == n && std::memcmp(h->last.data(), tab.data(), n) == 0)
        return FF_OK;                                  // device table already current
    // from here until the copy is enqueued the device table's contents are
    // unknown (a new allocation, or a copy that failed): forget them, so a
    // later call never skips its upload on the strength of a stale record
    h->last.clear();
    if (n > h->d_table_cap) {
        if (h->d_table) {
            FF_HIP(h, hipDeviceSynchronize());
            FF_HIP(h, hipFree(h->d_table));
            h->d_table = nullptr;
        }
        const size_t cap = std::max<size_t>(n, 16 * sizeof(PairDev));
        h->d_table_cap = 0;
        if (dev_malloc(h, (void**)&h->d_table, cap) != hipSuccess) {
            (void)hipGetLastError();
            h->d_table = nullptr;
            return fail(h, FF_ERR_OOM, "hipMalloc of the device pair table failed");
        }
        h->d_table_cap = cap;
    }
    const int k = (int)(h->staging_next++ % ff_ctx::kStaging);
    FF_HIP(h, hipEventSynchronize(h->table_ev[k]));   // the copy that last read slot k is done
    if (n > h->h_table_cap[k]) {
        // the slot keeps its old buffer until the larger one exists, so every
        // slot always holds at least the 16 pairs it was created with (the
        // allocation-free entry point relies on that)
        const size_t cap = std::max<size_t>(n, 16 * sizeof(PairDev));
        char* grown = nullptr;
        if (pinned_malloc(h, (void**)&grown, cap) != hipSuccess) {
            (void)hipGetLastError();
            return fail(h, FF_ERR_OOM, "pinned staging allocation failed");
        }
        if (h->h_table[k]) (void)hipHostFree(h->h_table[k]);
        h->h_table[k] = grown;
        h->h_table_cap[k] = cap;
    }
    std::memcpy(h->h_table[k], tab.data(), n);
    FF_HIP(h, hipMemcpyAsync(h->d_table, h->h_table[k], n, hipMemcpyHostToDevice, st));
    FF_HIP(h, hipEventRecord(h->table_ev[k], st));
    h->last = tab;
    return FF_OK;
}

struct Stop {
    bool active = false;
    ff_stage st{};
    void* dst = nullptr;
};

SearchConst search_const(const ff_params& p)
{
    SearchConst sc{};
    sc.levels = p.levels;
    sc.stride = p.seed_stride;
    sc.iters = p.iters;
    sc.radius = p.rs_radius;
    int J = 0;
    while ((p.rs_radius >> J) > 0) ++J;
    sc.trials = J;
    sc.eps2 = p.fb_eps * p.fb_eps;
    sc.key0 = (uint32_t)p.seed;
    sc.key1 = (uint32_t)(p.seed >> 32);
    sc.rng_level = -1;
    return sc;
}

const char* const kKernelNames[] = {"gray",      "down2",     "desc",       "seed_records", "seed_nn",
                                    "init",      "row_phase", "col_phase",  "transpose",    "fb",
                                    "sparse",    "census",    "save_state", "to_quarter",   "sub_row_phase",
                                    "sub_col_phase", "seed_resolve"};
enum { KN_GRAY, KN_DOWN2, KN_DESC, KN_SEED_REC, KN_SEED_NN, KN_INIT, KN_ROW, KN_COL, KN_TRANS, KN_FB, KN_SPARSE,
       KN_CENSUS, KN_SAVE, KN_QUARTER, KN_SUB_ROW, KN_SUB_COL, KN_SEED_RES, KN_COUNT };

// Record the opening event of a traced launch; returns the pair index or -1.
long prof_begin(ff_ctx* h, int kernel, int level, hipStream_t st)
{
    if (!h->prof_on) return -1;
    while (h->ev_used + 2 > h->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        h->ev_pool.push_back(e);
    }
    const size_t i = h->ev_used;
    h->ev_used += 2;
    (void)hipEventRecord(h->ev_pool[i], st);
    h->prof.push_back(ff_ctx::ProfRec{kernel, level, i});
    return (long)i;
}

void prof_end(ff_ctx* h, long i, hipStream_t st)
{
    if (i >= 0) (void)hipEventRecord(h->ev_pool[(size_t)i + 1], st);
}

#define FF_TRACED(kernel, level, call)          \
    do {                                        \
        const long pi_ = prof_begin(h, kernel, level, st); \
        call;                                   \
        prof_end(h, pi_, st);                   \
    } while (0)

// Enqueue the whole search (or, for a debug stop, the part up to it).

// Enqueue the launch sequence on `st`.  With an active stop, enqueue only up
// to that point and copy the intermediate of pair 0 (tab0 / plan0).
ff_status enqueue(ff_ctx* h, const PairDev* d, const Dims& D, hipStream_t st, const Stop& stop,
                  const PairDev* tab0, const PairPlan* plan0)
{
    const ff_params& p = h->prm;
    const int n = D.n;
    const int L = p.levels, c = L - 1;
    const SearchConst sc = search_const(p);
    auto level_px = [&](int l) { return (size_t)plan0->W[l] * plan0->H[l]; };
    auto work = [&](int ph, int l) {
        return D.nitems[ph][l] ? LineWork{(const uint32_t*)((const char*)d + D.item_off[ph][l]), D.nitems[ph][l]}
                               : LineWork{nullptr, 0};
    };
    // a level's state for a debug stop: rows Wp apart on the device, packed [H][W] for the caller
    auto copy_state = [&](int l) {
        const LevelDev& V = tab0->lv[l];
        return hipMemcpy2DAsync(stop.dst, (size_t)V.W * 8, V.state[stop.st.dir], (size_t)V.Wp * 8, (size_t)V.W * 8,
                                (size_t)V.H, hipMemcpyDeviceToDevice, st);
    };

    FF_TRACED(KN_GRAY, 0, launch_gray(d, n, D.maxPx[0], st));
    if (stop.active && stop.st.kind == FF_STAGE_GRAY) {
        FF_HIP(h, hipMemcpyAsync(stop.dst, tab0->lv[0].gray[stop.st.image], level_px(0), hipMemcpyDeviceToDevice, st));
        return FF_OK;
    }
    for (int l = 1; l < L; ++l) FF_TRACED(KN_DOWN2, l, launch_down2(d, n, l, D.maxPx[l], st));
    if (stop.active && stop.st.kind == FF_STAGE_PYRAMID) {
        const int l = stop.st.level;
        FF_HIP(h, hipMemcpyAsync(stop.dst, tab0->lv[l].gray[stop.st.image], level_px(l), hipMemcpyDeviceToDevice, st));
        return FF_OK;
    }
    const bool census = (p.flags & FF_COST_CENSUS) != 0;
    // with the Census cost only the seed level needs descriptors (unless a
    // debug stop asks for another level's)
    for (int l = 0; l < L; ++l)
        if (!census || l == c || (stop.active && stop.st.kind == FF_STAGE_DESC))
            FF_TRACED(KN_DESC, l, launch_desc(d, n, l, D.maxW[l], D.maxH[l], st));
    if (census)
        for (int l = 0; l < L; ++l) FF_TRACED(KN_CENSUS, l, launch_census(d, n, l, D.maxW[l], D.maxH[l], st));
    if (stop.active && stop.st.kind == FF_STAGE_CENSUS) {
        const int l = stop.st.level;
        const LevelDev& V = tab0->lv[l];
        FF_HIP(h, hipMemcpy2DAsync(stop.dst, (size_t)V.W * 8, V.cen[stop.st.image], (size_t)V.Wp * 8, (size_t)V.W * 8,
                                   (size_t)V.H, hipMemcpyDeviceToDevice, st));
        return FF_OK;
    }
    if (stop.active && stop.st.kind == FF_STAGE_DESC) {
        const int l = stop.st.level;
        const LevelDev& V = tab0->lv[l];
        launch_copy_desc_signed(V.desc[stop.st.image], (int8_t*)stop.dst, V.W, V.H, V.Wp, st);
        return FF_OK;
    }
    FF_TRACED(KN_SEED_REC, c, launch_seed_records(d, n, c, D.maxPx[c], st));
    FF_TRACED(KN_SEED_NN, c, launch_seed_nn(d, n, c, p.seed_stride, D.maxQ, D.maxPx[c], st));
    FF_TRACED(KN_SEED_RES, c, launch_seed_resolve(d, n, c, p.seed_stride, D.maxQ, st));
    if (stop.active && stop.st.kind == FF_STAGE_SEEDS) {
        launch_keys_to_index(tab0->keys[stop.st.dir], (int32_t*)stop.dst, plan0->nsx * plan0->nsy, st);
        return FF_OK;
    }
    // The search; with FF_SECOND_CHECK it runs again keyed by seed2 after
    // the first search's level-0 state is saved (debug stops name the first).
    const bool second = (p.flags & FF_SECOND_CHECK) != 0;
    const bool subpix = (p.flags & FF_SUBPIXEL) != 0;
    // the second search: keyed by seed2, and with FF_SECOND_PARAMS run with
    // its own iteration count and random-search radius
    SearchConst sc2 = sc;
    sc2.key0 = (uint32_t)p.seed2;
    sc2.key1 = (uint32_t)(p.seed2 >> 32);
    if (p.flags & FF_SECOND_PARAMS) {
        sc2.iters = p.iters2;
        sc2.radius = p.rs_radius2;
        sc2.trials = 0;
        while ((p.rs_radius2 >> sc2.trials) > 0) ++sc2.trials;
    }
    for (int run_k = 0; run_k < (second ? 2 : 1); ++run_k) {
        const SearchConst& scr = run_k ? sc2 : sc;
        const int iters = scr.iters;
        if (run_k == 1) FF_TRACED(KN_SAVE, 0, launch_save_state(d, n, D.maxPx[0], st));
        for (int l = c; l >= 0; --l) {
            const bool stop_here = run_k == 0 && stop.active && stop.st.kind == FF_STAGE_STATE && stop.st.level == l;
            // the row phase of iteration 0 takes over the init when its
            // schedule allows (and no stop asks for the init state itself)
            const bool fuse = iters > 0 && line_fused_init(h->tune_ch[0][l], h->tune_stg[0][l], scr) &&
                              !(stop_here && stop.st.step == 0);
            if (!fuse)
                FF_TRACED(KN_INIT, l, launch_init(d, n, l, l == c ? 1 : 0, p.seed_stride, census ? 1 : 0, D.maxPx[l], st));
            if (stop_here && stop.st.step == 0) {
                FF_HIP(h, copy_state(l));
                return FF_OK;
            }
            for (int t = 0; t < iters; ++t) {
                const bool last = stop_here && stop.st.iter == t;
                const int upto = last ? stop.st.step : 7;
                FF_TRACED(KN_ROW, l, launch_line_phase(false, h->tune_ch[0][l], h->tune_wpb[0][l], h->tune_stg[0][l], census ? 1 : 0, d, n, l, t,
                                                    std::min(upto, 3), scr, D.maxH[l], D.maxW[l], fuse && t == 0, work(0, l), st));
                if (upto >= 4) {
                    // the column phase reads the row-major state; its result comes
                    // back row-major when the cross write applies, else from stateT
                    FF_TRACED(KN_COL, l, launch_line_phase(true, h->tune_ch[1][l], h->tune_wpb[1][l], h->tune_stg[1][l], census ? 1 : 0, d, n, l, t, upto, scr,
                                                        D.maxW[l], D.maxH[l], 0, work(1, l), st));
                    if (!line_cross_write(h->tune_wpb[1][l], D.maxH[l]))
                        FF_TRACED(KN_TRANS, l, launch_transpose_state(d, n, l, 0, D.maxW[l], D.maxH[l], st));
                }
                if (last) {
                    FF_HIP(h, copy_state(l));
                    return FF_OK;
                }
            }
        }
        if (subpix) {
            // sub-pixel refinement at level 0 on quarter-pixel flows (the
            // debug stops name it as level `levels`); the first row pass
            // scales the flows to quarter pixels as it loads them, unless a
            // stop asks for that state itself
            const bool stop_sub = run_k == 0 && stop.active && stop.st.kind == FF_STAGE_STATE && stop.st.level == L;
            if (stop_sub && stop.st.step == 0) {
                FF_TRACED(KN_QUARTER, 0, launch_to_quarter(d, n, D.maxPx[0], st));
                FF_HIP(h, copy_state(0));
                return FF_OK;
            }
            // fixed schedule, (1, 8) rows and (1, 4) columns: the fastest of
            // the generic-pass shapes measured on the 1242x375 batch
            SearchConst scs = scr;
            scs.radius = p.sub_radius;
            scs.trials = 0;
            while ((p.sub_radius >> scs.trials) > 0) ++scs.trials;
            scs.rng_level = L;
            for (int t = 0; t < p.sub_iters; ++t) {
                const bool last = stop_sub && stop.st.iter == t;
                const int upto = last ? stop.st.step : 7;
                FF_TRACED(KN_SUB_ROW, 0, launch_line_phase(false, 1, 8, 0, 2, d, n, 0, t, std::min(upto, 3), scs, D.maxH[0],
                                                           D.maxW[0], t == 0 ? 1 : 0, LineWork{nullptr, 0}, st));
                if (upto >= 4) {
                    FF_TRACED(KN_SUB_COL, 0, launch_line_phase(true, 1, 4, 0, 2, d, n, 0, t, upto, scs, D.maxW[0], D.maxH[0], 0,
                                                               LineWork{nullptr, 0}, st));
                    if (!line_cross_write(4, D.maxH[0]))
                        FF_TRACED(KN_TRANS, 0, launch_transpose_state(d, n, 0, 0, D.maxW[0], D.maxH[0], st));
                }
                if (last) {
                    FF_HIP(h, copy_state(0));
                    return FF_OK;
                }
            }
        }
    }
    if (stop.active) return fail(h, FF_ERR_INVALID, "debug stage names a point the schedule does not reach");
    // quarter-pixel flows: consistency target rounded to whole pixels, the
    // error and its threshold in 1/16 px^2
    const int shift = subpix ? 2 : 0, eps2 = sc.eps2 << (2 * shift);
    if (second)
        FF_TRACED(KN_FB, 0, launch_fb2(d, n, eps2, shift, D.maxPx[0], st));
    else
        FF_TRACED(KN_FB, 0, launch_fb(d, n, eps2, shift, D.maxPx[0], st));
    if (p.flags & FF_SPARSIFY)
        FF_TRACED(KN_SPARSE, 0, launch_sparse(d, n, eps2, p.sparse_min, D.maxW[0], D.maxH[0], st));
    return FF_OK;
}

constexpr size_t kMaxGraphs = 16;

// Replay the captured launch sequence for this geometry.  A geometry seen
// for the first time is launched directly; the second time it is captured
// on the handle's private stream.  The per-pair table is device memory
// uploaded before the replay, so one graph serves every batch of the same
// geometry whatever its buffers.
ff_status launch_graph(ff_ctx* h, const PairDev* d, const Dims& D, hipStream_t st)
{
    std::vector<long long> key;
    key.push_back(D.n);
    key.push_back((long long)(uintptr_t)d);
    key.push_back(D.maxQ);
    for (int l = 0; l < h->prm.levels; ++l) {
        key.push_back(D.maxW[l]);
        key.push_back(D.maxH[l]);
        key.push_back(D.maxPx[l]);
        key.push_back(D.nitems[0][l]);
        key.push_back(D.nitems[1][l]);
    }
    for (size_t i = 0; i < h->graphs.size(); ++i) {
        if (h->graphs[i].key != key) continue;
        ff_ctx::GraphEntry e = h->graphs[i];
        h->graphs.erase(h->graphs.begin() + (long)i);
        h->graphs.push_back(e);                        // most recently used last
        FF_HIP(h, hipGraphLaunch(e.exec, st));
        return FF_OK;
    }
    auto it = std::find(h->seen.begin(), h->seen.end(), key);
    if (it == h->seen.end()) {
        if (h->seen.size() >= 64) h->seen.erase(h->seen.begin());
        h->seen.push_back(key);
        return enqueue(h, d, D, st, Stop{}, nullptr, nullptr);
    }
    h->seen.erase(it);
    if (!h->cap_stream) FF_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    FF_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    ff_status s = enqueue(h, d, D, h->cap_stream, Stop{}, nullptr, nullptr);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &g);
    if (s != FF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (ec != hipSuccess) return hip_fail(h, ec, "hipStreamEndCapture");
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(h, ei, "hipGraphInstantiate");
    }
    if (h->graphs.size() >= kMaxGraphs) {
        (void)hipGraphExecDestroy(h->graphs.front().exec);
        (void)hipGraphDestroy(h->graphs.front().graph);
        h->graphs.erase(h->graphs.begin());
    }
    ff_ctx::GraphEntry e;
    e.key = key;
    e.graph = g;
    e.exec = ex;
    h->graphs.push_back(e);
    FF_HIP(h, hipGraphLaunch(ex, st));
    return FF_OK;
}

// The line phases' work lists of a batch of uneven pairs: for each phase and
// level, every (pair-direction, line block) that holds lines of its pair,
// pair-direction-major, as pair-direction << 16 | block -- so a launch covers
// each pair at its own size instead of the batch's largest (the blocks past a
// smaller pair's size would only start and exit).  The lists depend on the
// schedule's lines per block, so they are rebuilt when it changes.  Appended
// to the table blob at 16-byte aligned offsets.
// Only batches of at least kWorkListMinPairs pairs get them: the lists' sizes
// are part of the captured graph's geometry, so small cohorts of varying
// composition (a serving loop) would rarely replay a graph and keep paying
// for captures -- measured on the served stream at 0.9x capacity: p50 / p99
// latency 9-10 / 15 ms with lists on every uneven cohort, 4.6 / 7.5-9.8 ms
// without them, at the same throughput.
constexpr int kWorkListMinPairs = 32;

void build_work_lists(const ff_ctx* h, const PairPlan* plans, int n, Dims& D, std::vector<char>& blob)
{
    for (int ph = 0; ph < 2; ++ph)
        for (int l = 0; l < h->prm.levels; ++l) {
            const int wpb = h->tune_wpb[ph][l];
            size_t off = (blob.size() + 15) & ~(size_t)15;
            size_t cnt = 0;
            for (int i = 0; i < n; ++i) cnt += 2 * (size_t)(((ph ? plans[i].W[l] : plans[i].H[l]) + wpb - 1) / wpb);
            blob.resize(off + cnt * sizeof(uint32_t));
            uint32_t* it = (uint32_t*)(blob.data() + off);
            for (int i = 0; i < n; ++i) {
                const uint32_t nb = (uint32_t)(((ph ? plans[i].W[l] : plans[i].H[l]) + wpb - 1) / wpb);
                for (uint32_t d = 0; d < 2; ++d)
                    for (uint32_t b = 0; b < nb; ++b) *it++ = ((uint32_t)(2 * i) + d) << 16 | b;
            }
            D.nitems[ph][l] = (int)cnt;
            D.item_off[ph][l] = off;
        }
}

// Validate, size the workspace, upload the pair table, then enqueue the
// search (graph replay unless tracing or stopping at an intermediate).
ff_status run(ff_ctx* h, const ff_pair* pairs, int n, hipStream_t st, const Stop& stop)
{
    if (n < 1 || n > 32767) return fail(h, FF_ERR_INVALID, "batch size must be in 1..32767");
    const ff_params& p = h->prm;
    // the same pair array as the previous call, on the same arena: its
    // validation, plan and device table still hold (the table was uploaded
    // by that call and nothing has replaced it since)
    if (!stop.active && h->last_valid && h->arena && h->arena == h->last_arena && h->last_tune_gen == h->tune_gen &&
        (size_t)n == h->last_pairs.size() && std::memcmp(pairs, h->last_pairs.data(), (size_t)n * sizeof(ff_pair)) == 0) {
        FF_HIP(h, hipSetDevice(h->device));
        if (h->run_any && st != h->run_stream) FF_HIP(h, hipStreamWaitEvent(st, h->run_done, 0));
        const Dims& D = h->last_dims;
        ff_status s = (!h->prof_on && h->use_graphs) ? launch_graph(h, h->d_table, D, st)
                                                    : enqueue(h, h->d_table, D, st, Stop{}, nullptr, nullptr);
        if (s != FF_OK) return s;
        FF_HIP(h, hipGetLastError());
        FF_HIP(h, hipEventRecord(h->run_done, st));
        h->run_stream = st;
        h->run_any = true;
        return FF_OK;
    }
    h->last_pairs.clear();
    std::vector<PairPlan> plans(n);
    size_t need = 0;
    for (int i = 0; i < n; ++i) {
        ff_status s = validate_pair(h, pairs[i]);
        if (s != FF_OK) return s;
        plans[i] = plan_pair(p, pairs[i].width, pairs[i].height);
        need += plans[i].bytes;
    }
    FF_HIP(h, hipSetDevice(h->device));
    ff_status s = ensure_arena(h, need);
    if (s != FF_OK) return s;
    // the previous call may still run on another stream: this call reuses
    // its arena and device table, so it starts after it
    if (h->run_any && st != h->run_stream) FF_HIP(h, hipStreamWaitEvent(st, h->run_done, 0));
    std::vector<PairDev> tab(n);
    build_table(p, (char*)h->arena, pairs, n, tab.data(), plans.data());

    Dims D;
    D.n = n;
    bool uneven = false;
    for (int i = 0; i < n; ++i) {
        for (int l = 0; l < p.levels; ++l) {
            D.maxW[l] = std::max(D.maxW[l], plans[i].W[l]);
            D.maxH[l] = std::max(D.maxH[l], plans[i].H[l]);
            D.maxPx[l] = std::max(D.maxPx[l], plans[i].W[l] * plans[i].H[l]);
        }
        D.maxQ = std::max(D.maxQ, plans[i].nsx * plans[i].nsy);
        uneven |= plans[i].W[0] != plans[0].W[0] || plans[i].H[0] != plans[0].H[0];
    }
    // the device table: the pair entries, then for a batch of uneven pairs
    // the line phases' work lists, one per phase and level
    std::vector<char> blob((size_t)n * sizeof(PairDev));
    std::memcpy(blob.data(), tab.data(), blob.size());
    if (uneven && n >= kWorkListMinPairs) build_work_lists(h, plans.data(), n, D, blob);
    s = upload_table(h, blob, st);
    if (s != FF_OK) return s;
    if (!stop.active && !h->prof_on && h->use_graphs)
        s = launch_graph(h, h->d_table, D, st);
    else
        s = enqueue(h, h->d_table, D, st, stop, &tab[0], &plans[0]);
    if (s != FF_OK) return s;
    FF_HIP(h, hipGetLastError());
    FF_HIP(h, hipEventRecord(h->run_done, st));
    h->run_stream = st;
    h->run_any = true;
    if (!stop.active) {
        h->last_dims = D;
        h->last_valid = true;
        h->last_tune_gen = h->tune_gen;
        h->last_pairs.assign(pairs, pairs + n);
        h->last_arena = h->arena;
    }
    return FF_OK;
}

// The allocation-free form of ff_match_pair: the pair's workspace and its
// device table live in the library's static per-device scratch array (set up
// by ff_create), the launches are enqueued directly (no graph capture, no
// tracing events), and nothing is allocated -- neither device nor pinned
// memory (the staging ring holds 16 pairs from creation).  Calls on one
// device are ordered through the scratch's event: each waits on the stream
// for the previous call's work, so calls from different streams or handles
// never overlap on the array.
ff_status run_noalloc(ff_ctx* h, const ff_pair* pair, hipStream_t st)
{
    const ff_params& p = h->prm;
    ff_status s = validate_pair(h, *pair);
    if (s != FF_OK) return s;
    const PairPlan plan = plan_pair(p, pair->width, pair->height);
    const size_t head = align_up(sizeof(PairDev));
    const size_t cap = noalloc_scratch_bytes();
    if (head + plan.bytes > cap) {
        char buf[200];
        snprintf(buf, sizeof buf, "pair needs %zu bytes of workspace; the allocation-free entry point holds at most %zu",
                 head + plan.bytes, cap);
        return fail(h, FF_ERR_BUDGET, buf);
    }
    FF_HIP(h, hipSetDevice(h->device));
    void* base = nullptr;
    hipEvent_t done = nullptr;
    if (!noalloc_lookup(h->device, &base, &done))
        return fail(h, FF_ERR_HIP, "the allocation-free scratch of this device was not set up (ff_create)");
    PairDev tab;
    build_table(p, (char*)base + head, pair, 1, &tab, &plan);
    Dims D;
    D.n = 1;
    for (int l = 0; l < p.levels; ++l) {
        D.maxW[l] = plan.W[l];
        D.maxH[l] = plan.H[l];
        D.maxPx[l] = plan.W[l] * plan.H[l];
    }
    D.maxQ = plan.nsx * plan.nsy;
    noalloc_lock(h->device);
    s = FF_OK;
    do {
        hipError_t e = hipStreamWaitEvent(st, done, 0);
        // the table goes through the handle's pinned staging ring (slot k is
        // refilled only after the copy that last read it has finished)
        const int k = (int)(h->staging_next++ % ff_ctx::kStaging);
        if (e == hipSuccess) e = hipEventSynchronize(h->table_ev[k]);
        if (e == hipSuccess) {
            std::memcpy(h->h_table[k], &tab, sizeof(PairDev));
            e = hipMemcpyAsync(base, h->h_table[k], sizeof(PairDev), hipMemcpyHostToDevice, st);
        }
        if (e == hipSuccess) e = hipEventRecord(h->table_ev[k], st);
        if (e != hipSuccess) {
            s = hip_fail(h, e, "allocation-free table upload");
            break;
        }
        const bool prof = h->prof_on;
        h->prof_on = false;
        s = enqueue(h, (const PairDev*)base, D, st, Stop{}, &tab, &plan);
        h->prof_on = prof;
        if (s != FF_OK) break;
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventRecord(done, st);
        if (e != hipSuccess) s = hip_fail(h, e, "allocation-free launch");
    } while (0);
    noalloc_unlock(h->device);
    return s;
}

struct Timed {
    int kernel, level;
    double ms;
};

// Synchronise the traced launches' events and turn them into durations.
ff_status collect_profile(ff_ctx* h, std::vector<Timed>& out)
{
    for (const ff_ctx::ProfRec& r : h->prof) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(h->ev_pool[r.ev + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, h->ev_pool[r.ev], h->ev_pool[r.ev + 1]);
        if (e != hipSuccess) {
            h->prof.clear();
            h->ev_used = 0;
            return hip_fail(h, e, "event timing");
        }
        out.push_back(Timed{r.kernel, r.level, (double)t});
    }
    h->prof.clear();
    h->ev_used = 0;
    return FF_OK;
}

void drop_graphs(ff_ctx* h)
{
    for (auto& e : h->graphs) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
    }
    h->graphs.clear();
    h->seen.clear();
}

// Time every (chunks per window, lines per block) candidate on this batch
// and keep, per phase and level, the fastest.  Each candidate runs twice;
// the second run is timed.  The search result is the same for every
// candidate, so tuning never changes an output.
ff_status autotune(ff_ctx* h, const ff_pair* pairs, int n, hipStream_t st)
{
    static const int kCand[][3] = {{1, 2, 0}, {1, 4, 0}, {1, 8, 0}, {2, 2, 0}, {2, 4, 0}, {2, 8, 0},
                                   {4, 2, 0}, {4, 4, 0}, {4, 8, 0}, {8, 2, 0}, {8, 4, 0}, {8, 8, 0},
                                   {1, 2, 2}, {1, 4, 2}, {1, 8, 2}, {2, 2, 2}, {2, 4, 2}, {2, 8, 2},
                                   {1, 4, 1}, {1, 8, 1}, {1, 16, 1}, {2, 8, 1}};
    const int L = h->prm.levels;
    double best[2][kMaxLevels];
    int bc[2][kMaxLevels][3];
    for (int ph = 0; ph < 2; ++ph)
        for (int l = 0; l < L; ++l) {
            best[ph][l] = 1e30;
            bc[ph][l][0] = h->tune_ch[ph][l];
            bc[ph][l][1] = h->tune_wpb[ph][l];
            bc[ph][l][2] = h->tune_stg[ph][l];
        }
    const bool was_on = h->prof_on;
    // on failure the handle goes back to the schedule it had
    auto restore = [&](ff_status s) {
        for (int ph = 0; ph < 2; ++ph)
            for (int l = 0; l < L; ++l) {
                h->tune_ch[ph][l] = bc[ph][l][0];
                h->tune_wpb[ph][l] = bc[ph][l][1];
                h->tune_stg[ph][l] = bc[ph][l][2];
            }
        ++h->tune_gen;
        h->prof_on = was_on;
        drop_graphs(h);
        return s;
    };
    int orig[2][kMaxLevels][3];
    std::memcpy(orig, bc, sizeof orig);
    std::vector<Timed> discard;
    (void)collect_profile(h, discard);
    for (const auto& c : kCand) {
        if (c[2] == 1 && (h->prm.flags & FF_COST_CENSUS)) continue;   // staged: descriptor cost only
        drop_graphs(h);
        ++h->tune_gen;
        for (int ph = 0; ph < 2; ++ph)
            for (int l = 0; l < L; ++l) {
                h->tune_ch[ph][l] = c[0];
                h->tune_wpb[ph][l] = c[1];
                h->tune_stg[ph][l] = c[2];
            }
        for (int rep = 0; rep < 2; ++rep) {
            h->prof_on = rep == 1;
            ff_status s = run(h, pairs, n, st, Stop{});
            h->prof_on = false;
            if (s != FF_OK) {
                std::memcpy(bc, orig, sizeof orig);
                return restore(s);
            }
        }
        std::vector<Timed> recs;
        ff_status s = collect_profile(h, recs);
        if (s != FF_OK) {
            std::memcpy(bc, orig, sizeof orig);
            return restore(s);
        }
        double t[2][kMaxLevels] = {{0}};
        for (const Timed& r : recs) {
            if (r.kernel == KN_ROW) t[0][r.level] += r.ms;
            if (r.kernel == KN_COL) t[1][r.level] += r.ms;
        }
        for (int ph = 0; ph < 2; ++ph)
            for (int l = 0; l < L; ++l)
                if (t[ph][l] < best[ph][l]) {
                    best[ph][l] = t[ph][l];
                    for (int k = 0; k < 3; ++k) bc[ph][l][k] = c[k];
                }
    }
    return restore(FF_OK);                              // with bc now the fastest candidates
}

void free_ctx(ff_ctx* h);

// A handle on `device`; `root` (or the new handle itself) holds the
// allocation fault injection, which starts from FF_FAULT_ALLOC_AFTER when
// that is set.  On failure returns null and *st names why (FF_ERR_OOM when a
// pinned allocation failed), having released everything it made.
ff_ctx* make_ctx(const ff_params& p, int device, ff_ctx* root, ff_status* st)
{
    *st = FF_ERR_HIP;
    ff_ctx* h = new ff_ctx;
    h->prm = p;
    h->device = device;
    if (root) {
        h->fault_root = root;
    } else if (const char* f = std::getenv("FF_FAULT_ALLOC_AFTER")) {
        h->fault_after = std::atoll(f);
    }
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return nullptr;
    }
    for (int k = 0; k < ff_ctx::kStaging; ++k) {
        if (hipEventCreateWithFlags(&h->table_ev[k], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(h->table_ev[j]);
            delete h;
            return nullptr;
        }
    }
    // the staging ring starts with room for 16 pairs per slot, so a
    // single-pair call never allocates pinned memory
    if (hipEventCreateWithFlags(&h->run_done, hipEventDisableTiming) != hipSuccess) {
        free_ctx(h);
        return nullptr;
    }
    for (int k = 0; k < ff_ctx::kStaging; ++k) {
        if (pinned_malloc(h, (void**)&h->h_table[k], 16 * sizeof(PairDev)) != hipSuccess) {
            (void)hipGetLastError();
            h->h_table[k] = nullptr;
            free_ctx(h);
            *st = FF_ERR_OOM;
            return nullptr;
        }
        h->h_table_cap[k] = 16 * sizeof(PairDev);
    }
    const char* g = std::getenv("FF_GRAPHS");
    h->use_graphs = !(g && g[0] == '0');
    *st = FF_OK;
    return h;
}

void free_serve(ff_ctx* h)
{
    ServeState* sv = h->serve;
    if (!sv) return;
    for (ServeLane& l : sv->lanes) {
        if (l.stream) (void)hipStreamSynchronize(l.stream);
        if (l.done) (void)hipEventDestroy(l.done);
        if (l.stream) (void)hipStreamDestroy(l.stream);
        if (l.exec) free_ctx(l.exec);
    }
    for (const ServeReq& r : sv->pending) (void)hipEventDestroy(r.ready);
    for (hipEvent_t e : sv->ev_pool) (void)hipEventDestroy(e);
    delete sv;
    h->serve = nullptr;
}

void free_ctx(ff_ctx* h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    free_serve(h);
    (void)hipDeviceSynchronize();
    if (h->arena) (void)hipFree(h->arena);
    if (h->d_table) (void)hipFree(h->d_table);
    for (int k = 0; k < ff_ctx::kStaging; ++k) {
        if (h->h_table[k]) (void)hipHostFree(h->h_table[k]);
        if (h->table_ev[k]) (void)hipEventDestroy(h->table_ev[k]);
    }
    for (auto& e : h->graphs) {
        (void)hipGraphExecDestroy(e.exec);
        (void)hipGraphDestroy(e.graph);
    }
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->run_done) (void)hipEventDestroy(h->run_done);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

size_t serve_bytes(const ff_ctx* h)
{
    return h->serve ? h->serve->lanes.size() * h->serve->lane_bytes : 0;
}

ff_status serve_configure(ff_ctx* h, int lanes, size_t lane_bytes)
{
    if (lanes < 1 || lanes > 16) return fail(h, FF_ERR_INVALID, "lanes must be in 1..16");
    if (lane_bytes < (1u << 20)) return fail(h, FF_ERR_INVALID, "lane_bytes must be at least 1 MiB");
    if (h->prm.hbm_budget && (uint64_t)lanes * lane_bytes > h->prm.hbm_budget)
        return fail(h, FF_ERR_BUDGET, "lanes x lane_bytes exceeds the HBM budget");
    if (h->serve) {
        for (const ServeLane& l : h->serve->lanes)
            if (l.busy) return fail(h, FF_ERR_BUSY, "serving engine has work in flight");
        if (!h->serve->pending.empty()) return fail(h, FF_ERR_BUSY, "serving engine has queued requests");
        free_serve(h);
    }
    FF_HIP(h, hipSetDevice(h->device));
    // one budget per handle: when the handle's own arena and the lanes do not
    // fit together, the arena is released (ff_match_* regrows it within what
    // the lanes leave)
    if (h->prm.hbm_budget && h->arena && (uint64_t)lanes * lane_bytes + h->arena_bytes > h->prm.hbm_budget) {
        FF_HIP(h, hipDeviceSynchronize());
        FF_HIP(h, hipFree(h->arena));
        h->arena = nullptr;
        h->arena_bytes = 0;
        h->last.clear();
        h->last_pairs.clear();
    }
    ServeState* sv = new ServeState;
    h->serve = sv;
    sv->lane_bytes = lane_bytes;
    sv->max_cohort = 32767;
    sv->lanes.resize(lanes);
    ff_params sub = h->prm;
    sub.hbm_budget = 0;                       // the parent handle enforces the budget
    for (ServeLane& l : sv->lanes) {
        ff_status cs = FF_OK;
        l.exec = make_ctx(sub, h->device, h->fault_root, &cs);
        if (!l.exec) {
            free_serve(h);
            return fail(h, cs, "lane context creation failed");
        }
        if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess) {
            free_serve(h);
            return fail(h, FF_ERR_HIP, "lane stream/event creation failed");
        }
        ff_status st = ensure_arena(l.exec, lane_bytes, true);
        if (st != FF_OK) {
            std::string msg = l.exec->err;
            free_serve(h);
            return fail(h, st, "lane arena: " + msg);
        }
    }
    return FF_OK;
}

// Retire finished cohorts, then start new cohorts on idle lanes.
ff_status serve_pump(ff_ctx* h)
{
    ServeState* sv = h->serve;
    for (ServeLane& l : sv->lanes) {
        if (!l.busy) continue;
        const hipError_t q = hipEventQuery(l.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return hip_fail(h, q, "lane completion");
        for (uint64_t t : l.tags) sv->done.push_back(t);
        l.tags.clear();
        l.busy = false;
    }
    for (ServeLane& l : sv->lanes) {
        if (l.busy || sv->pending.empty()) continue;
        std::vector<ServeReq> taken;
        size_t bytes = 0;
        while (!sv->pending.empty() && (int)taken.size() < sv->max_cohort &&
               bytes + sv->pending.front().bytes <= sv->lane_bytes) {
            taken.push_back(sv->pending.front());
            sv->pending.pop_front();
            bytes += taken.back().bytes;
        }
        if (taken.empty()) break;
        // a cohort that cannot start goes back to the head of the queue, in
        // order, with its requests' ready events: nothing submitted is lost,
        // and a later ff_poll tries again (ff_poll reports this one's error)
        auto requeue = [&](ff_status s, const std::string& msg) {
            for (size_t i = taken.size(); i-- > 0;) sv->pending.push_front(taken[i]);
            return fail(h, s, msg);
        };
        std::vector<ff_pair> cohort;
        for (const ServeReq& r : taken) {
            const hipError_t e = hipStreamWaitEvent(l.stream, r.ready, 0);
            if (e != hipSuccess) return requeue(FF_ERR_HIP, std::string("cohort wait: ") + hipGetErrorString(e));
            cohort.push_back(r.pair);
        }
        ff_status st = run(l.exec, cohort.data(), (int)cohort.size(), l.stream, Stop{});
        if (st != FF_OK) return requeue(st, "cohort launch: " + l.exec->err);
        const hipError_t e = hipEventRecord(l.done, l.stream);
        if (e != hipSuccess) return requeue(FF_ERR_HIP, std::string("cohort completion event: ") + hipGetErrorString(e));
        for (const ServeReq& r : taken) {
            sv->ev_pool.push_back(r.ready);
            l.tags.push_back(r.tag);
        }
        l.busy = true;
    }
    return FF_OK;
}

}  // namespace

extern "C" {

ff_status ff_create(const ff_params* params, int device, ff_handle* out)
{
    if (!params || !out) return FF_ERR_INVALID;
    *out = nullptr;
    ff_ctx tmp;
    ff_status s = validate_params(&tmp, *params);
    if (s != FF_OK) return s;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return FF_ERR_INVALID;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FF_ERR_HIP;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FF_ERR_UNSUPPORTED;
    ff_status cs = FF_OK;
    ff_ctx* h = make_ctx(*params, device, nullptr, &cs);
    if (!h) return cs;
    // the allocation-free entry point's scratch on this device (once per
    // device; a failure here surfaces only on that entry point)
    (void)noalloc_setup(device);
    *out = h;
    return FF_OK;
}

ff_status ff_match_pair_noalloc(ff_handle h, const ff_pair* pair, void* stream)
{
    if (!h) return FF_ERR_INVALID;
    if (!pair) return fail(h, FF_ERR_INVALID, "pair is NULL");
    return run_noalloc(h, pair, (hipStream_t)stream);
}

ff_status ff_match_pair(ff_handle h, const ff_pair* pair, void* stream)
{
    if (!h) return FF_ERR_INVALID;
    if (!pair) return fail(h, FF_ERR_INVALID, "pair is NULL");
    return run(h, pair, 1, (hipStream_t)stream, Stop{});
}

ff_status ff_match_batch(ff_handle h, const ff_pair* pairs, int32_t n, void* stream)
{
    if (!h) return FF_ERR_INVALID;
    if (!pairs || n < 1) return fail(h, FF_ERR_INVALID, "pairs is NULL or n < 1");
    return run(h, pairs, n, (hipStream_t)stream, Stop{});
}

ff_status ff_debug_stage(ff_handle h, const ff_pair* pair, const ff_stage* which, void* dst, void* stream)
{
    if (!h) return FF_ERR_INVALID;
    if (!pair || !which || !dst) return fail(h, FF_ERR_INVALID, "pair, which and dst are required");
    const ff_stage& w = *which;
    const bool sub_stage = (h->prm.flags & FF_SUBPIXEL) && w.kind == FF_STAGE_STATE && w.level == h->prm.levels;
    if (w.kind < FF_STAGE_GRAY || w.kind > FF_STAGE_CENSUS || w.image < 0 || w.image > 1 || w.dir < 0 ||
        w.dir > 1 || w.level < 0 || (w.level >= h->prm.levels && !sub_stage) || w.step < 0 || w.step > 7 ||
        w.iter < 0 || (w.kind == FF_STAGE_STATE && w.step > 0 && w.iter >= (sub_stage ? h->prm.sub_iters : h->prm.iters)))
        return fail(h, FF_ERR_INVALID, "bad debug stage");
    if (w.kind == FF_STAGE_CENSUS && !(h->prm.flags & FF_COST_CENSUS))
        return fail(h, FF_ERR_INVALID, "Census strings exist only with FF_COST_CENSUS");
    Stop s;
    s.active = true;
    s.st = w;
    s.dst = dst;
    return run(h, pair, 1, (hipStream_t)stream, s);
}

ff_status ff_debug_fault_alloc(ff_handle h, int64_t after)
{
    if (!h) return FF_ERR_INVALID;
    if (h->fault_root != h) return fail(h, FF_ERR_INVALID, "not a root handle");
    h->fault_after = after < 0 ? -1 : after;
    h->allocs = 0;
    return FF_OK;
}

uint64_t ff_workspace_bytes(ff_handle h, const ff_pair* pairs, int32_t n)
{
    if (!h || !pairs || n < 1) return 0;
    uint64_t b = 0;
    for (int i = 0; i < n; ++i) b += plan_pair(h->prm, pairs[i].width, pairs[i].height).bytes;
    return b;
}

ff_status ff_profile_enable(ff_handle h, int32_t on)
{
    if (!h) return FF_ERR_INVALID;
    h->prof_on = on != 0;
    return FF_OK;
}

int32_t ff_profile_read(ff_handle h, ff_profile_entry* out, int32_t max)
{
    if (!h || (!out && max > 0) || max < 0) return -1;
    std::vector<Timed> recs;
    if (collect_profile(h, recs) != FF_OK) return -1;
    int32_t launches[KN_COUNT] = {0};
    double ms[KN_COUNT] = {0};
    for (const Timed& r : recs) {
        launches[r.kernel] += 1;
        ms[r.kernel] += r.ms;
    }
    int32_t k = 0;
    for (int i = 0; i < KN_COUNT; ++i) {
        if (!launches[i]) continue;
        if (k < max) {
            std::memset(out[k].name, 0, sizeof out[k].name);
            std::strncpy(out[k].name, kKernelNames[i], sizeof out[k].name - 1);
            out[k].launches = launches[i];
            out[k].total_ms = ms[i];
        }
        ++k;
    }
    return std::min(k, max);
}

ff_status ff_autotune(ff_handle h, const ff_pair* pairs, int32_t n, void* stream)
{
    if (!h) return FF_ERR_INVALID;
    if (!pairs || n < 1) return fail(h, FF_ERR_INVALID, "pairs is NULL or n < 1");
    return autotune(h, pairs, n, (hipStream_t)stream);
}

int32_t ff_tune_get(ff_handle h, int32_t* cfg, int32_t max)
{
    const int L = h ? h->prm.levels : 0;
    if (!h || max < 6 * L || !cfg) return -1;
    for (int ph = 0; ph < 2; ++ph)
        for (int l = 0; l < L; ++l) {
            cfg[(ph * L + l) * 3 + 0] = h->tune_ch[ph][l];
            cfg[(ph * L + l) * 3 + 1] = h->tune_wpb[ph][l];
            cfg[(ph * L + l) * 3 + 2] = h->tune_stg[ph][l];
        }
    return 6 * L;
}

ff_status ff_tune_set(ff_handle h, const int32_t* cfg, int32_t n)
{
    if (!h) return FF_ERR_INVALID;
    const int L = h->prm.levels;
    if (!cfg || n != 6 * L) return fail(h, FF_ERR_INVALID, "tuning vector must hold 6 * levels entries");
    for (int i = 0; i < n; i += 3) {
        const int ch = cfg[i], wpb = cfg[i + 1], stg = cfg[i + 2];
        const bool plain = stg == 0 && (ch == 1 || ch == 2 || ch == 4 || ch == 8) && (wpb == 2 || wpb == 4 || wpb == 8);
        const bool staged = stg == 1 && ((ch == 1 && (wpb == 4 || wpb == 8 || wpb == 16)) || (ch == 2 && wpb == 8));
        const bool lockstep = stg == 2 && (ch == 1 || ch == 2) && (wpb == 2 || wpb == 4 || wpb == 8);
        if (!plain && !staged && !lockstep) return fail(h, FF_ERR_INVALID, "unsupported (chunks, lines, mode) triple");
        if (staged && (h->prm.flags & FF_COST_CENSUS))
            return fail(h, FF_ERR_INVALID, "staged schedules need the descriptor cost");
    }
    for (int ph = 0; ph < 2; ++ph)
        for (int l = 0; l < L; ++l) {
            h->tune_ch[ph][l] = cfg[(ph * L + l) * 3 + 0];
            h->tune_wpb[ph][l] = cfg[(ph * L + l) * 3 + 1];
            h->tune_stg[ph][l] = cfg[(ph * L + l) * 3 + 2];
        }
    ++h->tune_gen;
    drop_graphs(h);
    return FF_OK;
}

void ff_destroy(ff_handle h)
{
    free_ctx(h);
}

ff_status ff_serve_config(ff_handle h, int32_t lanes, uint64_t lane_bytes)
{
    if (!h) return FF_ERR_INVALID;
    return serve_configure(h, lanes, (size_t)lane_bytes);
}

ff_status ff_submit(ff_handle h, const ff_pair* pair, uint64_t tag, void* stream)
{
    if (!h) return FF_ERR_INVALID;
    if (!pair) return fail(h, FF_ERR_INVALID, "pair is NULL");
    if (!h->serve) {
        const size_t lb = h->prm.hbm_budget ? (size_t)(h->prm.hbm_budget / 4) : ((size_t)4 << 30);
        ff_status s = serve_configure(h, 4, lb);
        if (s != FF_OK) return s;
    }
    ff_status s = validate_pair(h, *pair);
    if (s != FF_OK) return s;
    ServeState* sv = h->serve;
    const size_t bytes = plan_pair(h->prm, pair->width, pair->height).bytes;
    if (bytes > sv->lane_bytes) return fail(h, FF_ERR_BUDGET, "pair does not fit one serving lane's arena");
    hipEvent_t ready;
    if (!sv->ev_pool.empty()) {
        ready = sv->ev_pool.back();
        sv->ev_pool.pop_back();
    } else {
        FF_HIP(h, hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    }
    const hipError_t e = hipEventRecord(ready, (hipStream_t)stream);
    if (e != hipSuccess) {
        sv->ev_pool.push_back(ready);
        return hip_fail(h, e, "hipEventRecord(ready)");
    }
    sv->pending.push_back(ServeReq{*pair, tag, bytes, ready});
    // the pair is queued: a cohort that cannot start now stays queued and
    // the next ff_poll tries again (and reports the error if it persists)
    (void)serve_pump(h);
    return FF_OK;
}

int32_t ff_poll(ff_handle h, uint64_t* tags_done, int32_t max)
{
    if (!h || max < 0 || (max > 0 && !tags_done)) return -1;
    if (!h->serve) return 0;
    if (serve_pump(h) != FF_OK) return -1;
    ServeState* sv = h->serve;
    int32_t k = 0;
    while (k < max && !sv->done.empty()) {
        tags_done[k++] = sv->done.front();
        sv->done.pop_front();
    }
    return k;
}

int32_t ff_serve_inflight(ff_handle h)
{
    if (!h) return -1;
    if (!h->serve) return 0;
    int32_t n = (int32_t)h->serve->pending.size();
    for (const ServeLane& l : h->serve->lanes) n += (int32_t)l.tags.size();
    return n;
}

const char* ff_last_error(ff_handle h)
{
    if (!h) return g_static_err;
    return h->err.c_str();
}

}  // extern "C"
