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
void launch_init(const PairDev*, int, int, int, int, int, hipStream_t);
void launch_row_phase(const PairDev*, int, int, int, int, const SearchConst&, int, hipStream_t);
void launch_col_phase(const PairDev*, int, int, int, int, const SearchConst&, int, hipStream_t);
void launch_transpose_state(const PairDev*, int, int, int, int, int, hipStream_t);
void launch_fb(const PairDev*, int, int, int, hipStream_t);
void launch_copy_desc_signed(const uint8_t*, int8_t*, size_t, hipStream_t);
void launch_keys_to_index(const unsigned long long*, int32_t*, int, hipStream_t);
}  // namespace ff

using namespace ff;

struct ff_ctx {
    ff_params prm{};
    int device = 0;
    std::string err;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    PairDev* d_table = nullptr;      // device copy of the per-pair table
    size_t d_table_cap = 0;          // entries
    PairDev* h_table = nullptr;      // pinned staging for the upload
    size_t h_table_cap = 0;
    hipEvent_t table_ev = nullptr;   // last upload from h_table finished
    std::vector<PairDev> last;       // what d_table holds now
    // tracing: event pairs around every launch while enabled
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<int, size_t>> prof;   // (kernel id, first event index)
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
        const size_t n = (size_t)pl.W[l] * pl.H[l];
        b += 2 * align_up(n);            // gray planes
        b += 4 * align_up(n * 16);       // descriptors, row- and column-major
        b += 4 * align_up(n * 8);        // state, row- and column-major
    }
    const int c = p.levels - 1;
    pl.nsx = (pl.W[c] + p.seed_stride - 1) / p.seed_stride;
    pl.nsy = (pl.H[c] + p.seed_stride - 1) / p.seed_stride;
    b += 2 * align_up((size_t)pl.W[c] * pl.H[c] * 64);
    b += 2 * align_up((size_t)pl.nsx * pl.nsy * 8);
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
    if (p.flags != 0) return fail(h, FF_ERR_INVALID, "flags must be 0");
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
    if (((uintptr_t)q.flow_fwd & 3) || ((uintptr_t)q.flow_bwd & 3) || ((uintptr_t)q.cost_fwd & 3) ||
        ((uintptr_t)q.cost_bwd & 3))
        return fail(h, FF_ERR_INVALID, "flow and cost outputs must be 4-byte aligned");
    return FF_OK;
}

ff_status ensure_arena(ff_ctx* h, size_t need)
{
    if (h->prm.hbm_budget && need > h->prm.hbm_budget) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace of %zu bytes exceeds the budget of %llu bytes", need,
                 (unsigned long long)h->prm.hbm_budget);
        return fail(h, FF_ERR_BUDGET, buf);
    }
    if (need <= h->arena_bytes) return FF_OK;
    if (h->arena) {
        FF_HIP(h, hipDeviceSynchronize());
        FF_HIP(h, hipFree(h->arena));
        h->arena = nullptr;
        h->arena_bytes = 0;
        h->last.clear();
    }
    const size_t want = need + need / 8;     // head-room against regrowth
    hipError_t e = hipMalloc(&h->arena, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        e = hipMalloc(&h->arena, need);
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

// Fill the per-pair table: carve each pair's buffers out of the arena.
void build_table(ff_ctx* h, const ff_pair* pairs, int n, std::vector<PairDev>& tab,
                 std::vector<PairPlan>& plans)
{
    const ff_params& p = h->prm;
    tab.assign(n, PairDev{});
    char* base = (char*)h->arena;
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
            for (int k = 0; k < 2; ++k) L.gray[k] = (uint8_t*)take(np);
            for (int k = 0; k < 2; ++k) L.desc[k] = (uint8_t*)take(np * 16);
            for (int k = 0; k < 2; ++k) L.descT[k] = (uint8_t*)take(np * 16);
            for (int k = 0; k < 2; ++k) L.state[k] = (int2*)take(np * 8);
            for (int k = 0; k < 2; ++k) L.stateT[k] = (int2*)take(np * 8);
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
    }
}

ff_status upload_table(ff_ctx* h, const std::vector<PairDev>& tab, hipStream_t st)
{
    const size_t n = tab.size();
    if (h->last.size() == n && std::memcmp(h->last.data(), tab.data(), n * sizeof(PairDev)) == 0)
        return FF_OK;                                  // device table already current
    if (n > h->d_table_cap) {
        if (h->d_table) {
            FF_HIP(h, hipDeviceSynchronize());
            FF_HIP(h, hipFree(h->d_table));
            h->d_table = nullptr;
        }
        const size_t cap = std::max<size_t>(n, 16);
        FF_HIP(h, hipMalloc((void**)&h->d_table, cap * sizeof(PairDev)));
        h->d_table_cap = cap;
    }
    if (n > h->h_table_cap) {
        if (h->h_table) {
            FF_HIP(h, hipEventSynchronize(h->table_ev));
            FF_HIP(h, hipHostFree(h->h_table));
            h->h_table = nullptr;
        }
        const size_t cap = std::max<size_t>(n, 16);
        FF_HIP(h, hipHostMalloc((void**)&h->h_table, cap * sizeof(PairDev), hipHostMallocDefault));
        h->h_table_cap = cap;
    }
    FF_HIP(h, hipEventSynchronize(h->table_ev));      // previous upload done reading h_table
    std::memcpy(h->h_table, tab.data(), n * sizeof(PairDev));
    FF_HIP(h, hipMemcpyAsync(h->d_table, h->h_table, n * sizeof(PairDev), hipMemcpyHostToDevice, st));
    FF_HIP(h, hipEventRecord(h->table_ev, st));
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
    return sc;
}

const char* const kKernelNames[] = {"gray", "down2", "desc", "seed_records", "seed_nn",
                                    "init", "row_phase", "col_phase", "transpose", "fb"};
enum { KN_GRAY, KN_DOWN2, KN_DESC, KN_SEED_REC, KN_SEED_NN, KN_INIT, KN_ROW, KN_COL, KN_TRANS, KN_FB, KN_COUNT };

// Record the opening event of a traced launch; returns the pair index or -1.
long prof_begin(ff_ctx* h, int kernel, hipStream_t st)
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
    h->prof.emplace_back(kernel, i);
    return (long)i;
}

void prof_end(ff_ctx* h, long i, hipStream_t st)
{
    if (i >= 0) (void)hipEventRecord(h->ev_pool[(size_t)i + 1], st);
}

#define FF_TRACED(kernel, call)                 \
    do {                                        \
        const long pi_ = prof_begin(h, kernel, st); \
        call;                                   \
        prof_end(h, pi_, st);                   \
    } while (0)

// Enqueue the whole search (or, for a debug stop, the part up to it).
ff_status run(ff_ctx* h, const ff_pair* pairs, int n, hipStream_t st, const Stop& stop)
{
    if (n < 1 || n > 32767) return fail(h, FF_ERR_INVALID, "batch size must be in 1..32767");
    const ff_params& p = h->prm;
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
    std::vector<PairDev> tab;
    build_table(h, pairs, n, tab, plans);
    s = upload_table(h, tab, st);
    if (s != FF_OK) return s;
    const PairDev* d = h->d_table;

    int maxW[kMaxLevels] = {0}, maxH[kMaxLevels] = {0}, maxPx[kMaxLevels] = {0};
    int maxQ = 0;
    for (int i = 0; i < n; ++i) {
        for (int l = 0; l < p.levels; ++l) {
            maxW[l] = std::max(maxW[l], plans[i].W[l]);
            maxH[l] = std::max(maxH[l], plans[i].H[l]);
            maxPx[l] = std::max(maxPx[l], plans[i].W[l] * plans[i].H[l]);
        }
        maxQ = std::max(maxQ, plans[i].nsx * plans[i].nsy);
    }
    const int L = p.levels, c = L - 1;
    const SearchConst sc = search_const(p);

    FF_TRACED(KN_GRAY, launch_gray(d, n, maxPx[0], st));
    if (stop.active && stop.st.kind == FF_STAGE_GRAY) {
        FF_HIP(h, hipMemcpyAsync(stop.dst, tab[0].lv[0].gray[stop.st.image], (size_t)plans[0].W[0] * plans[0].H[0],
                                 hipMemcpyDeviceToDevice, st));
        return FF_OK;
    }
    for (int l = 1; l < L; ++l) FF_TRACED(KN_DOWN2, launch_down2(d, n, l, maxPx[l], st));
    if (stop.active && stop.st.kind == FF_STAGE_PYRAMID) {
        const int l = stop.st.level;
        FF_HIP(h, hipMemcpyAsync(stop.dst, tab[0].lv[l].gray[stop.st.image], (size_t)plans[0].W[l] * plans[0].H[l],
                                 hipMemcpyDeviceToDevice, st));
        return FF_OK;
    }
    for (int l = 0; l < L; ++l) FF_TRACED(KN_DESC, launch_desc(d, n, l, maxW[l], maxH[l], st));
    if (stop.active && stop.st.kind == FF_STAGE_DESC) {
        const int l = stop.st.level;
        launch_copy_desc_signed(tab[0].lv[l].desc[stop.st.image], (int8_t*)stop.dst,
                                (size_t)plans[0].W[l] * plans[0].H[l] * 16, st);
        return FF_OK;
    }
    FF_TRACED(KN_SEED_REC, launch_seed_records(d, n, c, maxPx[c], st));
    FF_TRACED(KN_SEED_NN, launch_seed_nn(d, n, c, p.seed_stride, maxQ, maxPx[c], st));
    if (stop.active && stop.st.kind == FF_STAGE_SEEDS) {
        launch_keys_to_index(tab[0].keys[stop.st.dir], (int32_t*)stop.dst, plans[0].nsx * plans[0].nsy, st);
        return FF_OK;
    }
    for (int l = c; l >= 0; --l) {
        FF_TRACED(KN_INIT, launch_init(d, n, l, l == c ? 1 : 0, p.seed_stride, maxPx[l], st));
        const bool stop_here = stop.active && stop.st.kind == FF_STAGE_STATE && stop.st.level == l;
        if (stop_here && stop.st.step == 0) {
            FF_HIP(h, hipMemcpyAsync(stop.dst, tab[0].lv[l].state[stop.st.dir], (size_t)plans[0].W[l] * plans[0].H[l] * 8,
                                     hipMemcpyDeviceToDevice, st));
            return FF_OK;
        }
        for (int t = 0; t < p.iters; ++t) {
            const bool last = stop_here && stop.st.iter == t;
            const int upto = last ? stop.st.step : 7;
            FF_TRACED(KN_ROW, launch_row_phase(d, n, l, t, std::min(upto, 3), sc, maxH[l], st));
            if (upto >= 4) {
                FF_TRACED(KN_TRANS, launch_transpose_state(d, n, l, 1, maxW[l], maxH[l], st));
                FF_TRACED(KN_COL, launch_col_phase(d, n, l, t, upto, sc, maxW[l], st));
                FF_TRACED(KN_TRANS, launch_transpose_state(d, n, l, 0, maxW[l], maxH[l], st));
            }
            if (last) {
                FF_HIP(h, hipMemcpyAsync(stop.dst, tab[0].lv[l].state[stop.st.dir],
                                         (size_t)plans[0].W[l] * plans[0].H[l] * 8, hipMemcpyDeviceToDevice, st));
                return FF_OK;
            }
        }
    }
    if (stop.active) return fail(h, FF_ERR_INVALID, "debug stage names a point the schedule does not reach");
    FF_TRACED(KN_FB, launch_fb(d, n, sc.eps2, maxPx[0], st));
    FF_HIP(h, hipGetLastError());
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
    ff_ctx* h = new ff_ctx;
    h->prm = *params;
    h->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipEventCreateWithFlags(&h->table_ev, hipEventDisableTiming) != hipSuccess) {
        delete h;
        return FF_ERR_HIP;
    }
    *out = h;
    return FF_OK;
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
    if (w.kind < FF_STAGE_GRAY || w.kind > FF_STAGE_STATE || w.image < 0 || w.image > 1 || w.dir < 0 ||
        w.dir > 1 || w.level < 0 || w.level >= h->prm.levels || w.step < 0 || w.step > 7 || w.iter < 0 ||
        (w.kind == FF_STAGE_STATE && w.step > 0 && w.iter >= h->prm.iters))
        return fail(h, FF_ERR_INVALID, "bad debug stage");
    Stop s;
    s.active = true;
    s.st = w;
    s.dst = dst;
    return run(h, pair, 1, (hipStream_t)stream, s);
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
    int32_t launches[KN_COUNT] = {0};
    double ms[KN_COUNT] = {0};
    for (const auto& r : h->prof) {
        float t = 0.f;
        if (hipEventSynchronize(h->ev_pool[r.second + 1]) != hipSuccess ||
            hipEventElapsedTime(&t, h->ev_pool[r.second], h->ev_pool[r.second + 1]) != hipSuccess) {
            (void)hipGetLastError();
            h->prof.clear();
            h->ev_used = 0;
            fail(h, FF_ERR_HIP, "event timing failed");
            return -1;
        }
        launches[r.first] += 1;
        ms[r.first] += t;
    }
    h->prof.clear();
    h->ev_used = 0;
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

void ff_destroy(ff_handle h)
{
    if (!h) return;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    if (h->arena) (void)hipFree(h->arena);
    if (h->d_table) (void)hipFree(h->d_table);
    if (h->h_table) (void)hipHostFree(h->h_table);
    if (h->table_ev) (void)hipEventDestroy(h->table_ev);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    delete h;
}

const char* ff_last_error(ff_handle h)
{
    if (!h) return g_static_err;
    return h->err.c_str();
}

}  // extern "C"
