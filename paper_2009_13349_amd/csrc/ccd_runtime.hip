// Host runtime and C ABI of the MI355X CCD library (see include/ccd.h).
//
// A batch runs as a fixed sequence of kernels on the caller's stream:
//   reset counters -> [root pass: level 0 of every query, survivors grouped
//   by kind] -> lane engine ->
//   group engine (wide queries handed on by the lane engine) ->
//   block engine (queries whose frontier outgrew a group arena).
// All scratch lives in one context, sized within the context's memory budget
// and reused across batches (grow-only).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ccd.h"
#include "ccd_host.h"
#include "ccd_internal.h"

namespace ccd {
template <bool P>
__global__ void k_lane(BatchArgs a, LaneCfg c);
template <int W, int OCC, bool LDS>
__global__ void k_group(BatchArgs a, GroupCfg g);
__global__ void k_root(BatchArgs a, int64_t* order);
__global__ void k_min_toi_init(unsigned long long* out);
__global__ void k_gather(int64_t n, const double* v0, const double* v1, const int32_t* ids,
                         int64_t nv, double* pos);
__global__ void k_scene_gamma_init(unsigned long long* g);
__global__ void k_scene_gamma(const double* v0, const double* v1, int64_t nv, unsigned long long* g);
__global__ void k_min_toi(const double* toi, int64_t n, unsigned long long* out);
__global__ void k_reset(unsigned long long* counters);
__global__ void k_order_records(const unsigned long long* counters, const uint8_t* levels,
                                int64_t cap, int32_t count_idx, int64_t* perm);
}  // namespace ccd

using namespace ccd;

namespace {

constexpr double kCoordLimitHost = 1e300;

thread_local char g_last_error[256] = "";

// Records a failed HIP call (text available through ccd_last_error) and
// returns false; clears HIP's sticky error state.
bool hip_ok(hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    std::snprintf(g_last_error, sizeof(g_last_error), "%s: %s", what, hipGetErrorString(e));
    (void)hipGetLastError();
    return false;
}

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

bool grow(DevBuf& b, size_t bytes) {
    if (bytes <= b.bytes) return true;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (bytes == 0) return true;
    if (!hip_ok(hipMalloc(&b.p, bytes), "hipMalloc")) return false;
    b.bytes = bytes;
    return true;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

}  // namespace

struct ccd_context {
    int device = 0;
    int num_cu = 256;
    size_t lds_per_block = 65536;  // device limit of LDS per workgroup
    size_t budget = 0;
    int engine = CCD_ENGINE_PERSISTENT;
    ccd_tuning tune{};
    DevBuf counters, order, rec_a, group_arena, rec_b, pool, block_arena;
    DevBuf io;      // staging for host-pointer batches
    DevBuf gather;  // structure-of-arrays coordinates of an indexed batch
    bool timing = false;
    hipEvent_t ev[5] = {};
    bool have_events = false;
    // hipGraph of the launch sequence, replayed while its parameters are unchanged
    bool use_graphs = true;  // (serving contexts launch eagerly: their arguments change per launch)
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    unsigned char graph_key[512] = {};
    size_t graph_key_len = 0;
    uint64_t graph_builds = 0, graph_replays = 0;
    bool last_timed = false;
    bool last_valid = false;
};

namespace {

int set_device(int dev) {
    return hip_ok(hipSetDevice(dev), "hipSetDevice") ? CCD_OK : CCD_EDEVICE;
}

void default_tuning(ccd_tuning& t, int num_cu) {
    t.lane_waves_per_cu = 8;
    t.lane_capacity = 16;
    t.lane_budget = 256;
    t.group_waves = 1;
    t.group_count = num_cu * 12;
    t.group_capacity = 1 << 16;
    t.block_count = 2 * num_cu;
    t.group_occupancy = 3;
    t.block_capacity = 0;             // 2 m_I + 2, within the budget
    t.handoff_words = int64_t(1) << 33;  // 64 GiB: in practice what the budget leaves
    t.group_lds_words = 0;            // off: measured slower on the simulation-shaped workload
    t.block_lds_words = 2048;         // 32 KiB per eight-wave block
}

void clamp_tuning(ccd_tuning& t) {
    t.lane_waves_per_cu = std::min(32, std::max(1, t.lane_waves_per_cu));
    t.lane_capacity = std::min(32, std::max(8, t.lane_capacity));
    t.lane_budget = std::max<int64_t>(1, t.lane_budget);
    if (t.group_waves >= 8) t.group_waves = 8;
    else if (t.group_waves >= 4) t.group_waves = 4;
    else if (t.group_waves >= 2) t.group_waves = 2;
    else t.group_waves = 1;
    t.group_count = std::min(1 << 16, std::max(1, t.group_count));
    t.group_capacity = std::min<int64_t>(int64_t(1) << 28, std::max<int64_t>(256, t.group_capacity));
    t.block_count = std::min(1 << 12, std::max(1, t.block_count));
    t.group_occupancy = std::min(4, std::max(1, t.group_occupancy));
    t.block_capacity = t.block_capacity <= 0 ? 0 : std::max<int64_t>(256, t.block_capacity);
    t.handoff_words = std::min<int64_t>(int64_t(1) << 34, std::max<int64_t>(0, t.handoff_words));
    t.group_lds_words = std::min(16384, std::max(0, t.group_lds_words)) & ~63;
    t.block_lds_words = std::min(16384, std::max(0, t.block_lds_words)) & ~63;
}

// 0 < t_max <= 1 (false for NaN), no unknown flags.
bool params_ok(const ccd_params& p) {
    return p.t_max > 0.0 && p.t_max <= 1.0 && p.reserved == 0 &&
           (p.flags & ~CCD_FLAG_LITERAL) == 0;
}

// Host copy of the device-side query validation (same rule, same arithmetic).
bool host_query_valid(const double X[24], int kind, double delta, int64_t max_iter, double min_sep) {
    if (kind != CCD_KIND_VF && kind != CCD_KIND_EE) return false;
    for (int i = 0; i < 24; ++i)
        if (!(std::fabs(X[i]) <= kCoordLimitHost)) return false;
    if (!(delta > 0.0) || !(delta <= 1.7976931348623157e308)) return false;
    if (max_iter < 1) return false;
    double gmin = 0.0;
    for (int c = 0; c < 3; ++c) {
        double g = 1.0;
        for (int k = 0; k < 8; ++k) g = std::max(g, std::fabs(X[3 * k + c]));
        gmin = (c == 0) ? g : std::min(gmin, g);
    }
    if (!(min_sep >= 0.0) || !(min_sep < gmin)) return false;
    return true;
}

struct Plan {
    int64_t n;
    int lane_slots;
    int lane_grid;       // blocks of kLaneBlock threads
    size_t lane_lds;     // dynamic LDS bytes per lane-engine block
    int64_t rec_a_words, rec_a_cap;
    int64_t rec_b_words, rec_b_cap;
    int64_t pool_words;  // group -> block hand-off pool
    int group_count;
    int64_t group_cap;
    int block_count;
    int64_t block_cap;
    int block_waves;     // 4 when there are at least two block engines per CU, else 8
};

// Saturating size arithmetic: a result that does not fit size_t becomes
// SIZE_MAX, which no budget admits.
size_t smul(size_t a, size_t b) {
    size_t r;
    return __builtin_mul_overflow(a, b, &r) ? SIZE_MAX : r;
}
size_t sadd(size_t a, size_t b) {
    size_t r;
    return __builtin_add_overflow(a, b, &r) ? SIZE_MAX : r;
}

constexpr size_t kArenaBytesPerWord = 6 * 8;  // two buffers of up to three words per box

// Sizes the scratch of a launch of n queries whose largest m_I is max_iter_max
// within the context's budget.  The block engine's arena would need 2 m_I + 2
// words per buffer for every query to finish there (a level of a query that
// has not returned has fewer than 2 m_I boxes); it is clamped to a quarter of
// the budget (and to the tuning's block_capacity), and a query whose level
// outgrows it ends with the flagged overflow return.
int plan_for(const ccd_tuning& t, int num_cu, size_t budget, int64_t n, int64_t max_iter_max,
             bool persistent, Plan& P) {
    std::memset(&P, 0, sizeof(P));  // padding too: plans are compared bytewise (graph reuse)
    P.n = n;
    const int K = t.lane_capacity;
    if (persistent) {
        const int64_t threads = (int64_t)num_cu * t.lane_waves_per_cu * 64;
        P.lane_grid = (int)((threads + kLaneBlock - 1) / kLaneBlock);
    } else {
        P.lane_grid = (int)((n + kLaneBlock - 1) / kLaneBlock);
    }
    P.lane_slots = P.lane_grid * (kLaneBlock / 64);
    P.lane_lds = (size_t)2 * K * kLaneBlock * 8;
    P.rec_a_words = kRecordHeaderWords + (int64_t)K;
    P.rec_a_cap = n;
    P.rec_b_words = kRecordHeaderWords + 1;
    P.rec_b_cap = n;
    P.group_cap = std::max<int64_t>(t.group_capacity, K);
    P.group_count = t.group_count;
    P.block_count = t.block_count;

    const size_t fixed = sadd(sadd(sadd(64 * 8, smul((size_t)n, 9)),                        // counters, order + record levels
                                   smul(smul((size_t)P.rec_a_cap, (size_t)P.rec_a_words), 8)),  // records A
                              smul(smul((size_t)P.rec_b_cap, (size_t)P.rec_b_words), 8));       // records B
    const size_t per_group = smul((size_t)P.group_cap, kArenaBytesPerWord);
    // the block engine takes the group engine's hand-offs, so its arena is at
    // least a group arena
    const size_t min_block = per_group;
    if (sadd(sadd(fixed, per_group), min_block) > budget) {
        set_last_error("scratch plan: device memory budget too small for the batch");
        return CCD_ENOMEM;
    }
    size_t left = budget - fixed;  // >= per_group + min_block
    // block arena capacity: min(2 m_I + 2, tuning, a quarter of what is left),
    // never below a group arena's
    uint64_t want = max_iter_max >= (INT64_MAX - 2) / 2 ? (uint64_t)INT64_MAX
                                                        : (uint64_t)(2 * max_iter_max + 2);
    if (t.block_capacity > 0) want = std::min<uint64_t>(want, (uint64_t)t.block_capacity);
    const uint64_t quarter = (uint64_t)(left / 4 / kArenaBytesPerWord);
    want = std::min<uint64_t>(want, quarter);
    P.block_cap = (int64_t)std::max<uint64_t>(want, (uint64_t)P.group_cap);
    const size_t per_block = smul((size_t)P.block_cap, kArenaBytesPerWord);
    // one arena of each engine always (per_block <= left / 4, or = per_group
    // <= left / 2: both fit)
    left -= per_group + per_block;
    // hand-off pool, first share: the tuning's size, at most an eighth of what
    // is left
    P.pool_words = std::min<int64_t>(t.handoff_words, (int64_t)(left / 8 / 8));
    left -= (size_t)P.pool_words * 8;
    // the group engine carries the bulk of the work: further groups get up to
    // 3/4 of what is left; further blocks the rest
    const size_t more_groups = (left / 4 * 3) / per_group;
    P.group_count = (int)std::min<size_t>((size_t)std::max(P.group_count, 1), 1 + more_groups);
    left -= (size_t)(P.group_count - 1) * per_group;
    const size_t blocks_fit = 1 + left / per_block;
    P.block_count = (int)std::min<size_t>((size_t)P.block_count, blocks_fit);
    left -= (size_t)(P.block_count - 1) * per_block;
    // two four-wave engines per CU check more wide queries at once than one
    // eight-wave engine (each keeps two waves per SIMD at its register use);
    // with fewer engines than that, each gets eight waves
    P.block_waves = P.block_count >= 2 * num_cu ? 4 : 8;
    // the pool takes what remains, up to the tuning's size: every hand-off
    // beyond it restarts its query at level 0 (the same result, more work).
    // Rounded down to 128 MiB steps, so that batches of other sizes (whose
    // records take more or less of the budget) mostly plan the same pool and
    // the context's grow-only buffer is not reallocated for a few bytes.
    P.pool_words += std::min<int64_t>(t.handoff_words - P.pool_words, (int64_t)(left / 8));
    constexpr int64_t kPoolStep = int64_t(1) << 24;
    if (P.pool_words > kPoolStep && P.pool_words < t.handoff_words) P.pool_words &= ~(kPoolStep - 1);
    return CCD_OK;
}

int make_plan(ccd_context* ctx, int64_t n, int64_t max_iter_max, bool persistent, Plan& P) {
    return plan_for(ctx->tune, ctx->num_cu, ctx->budget, n, max_iter_max, persistent, P);
}

size_t plan_bytes(const Plan& P) {
    return 64 * 8 + (size_t)P.n * 9 + (size_t)P.rec_a_cap * P.rec_a_words * 8 +
           (size_t)P.rec_b_cap * P.rec_b_words * 8 + (size_t)P.pool_words * 8 +
           (size_t)P.group_count * P.group_cap * kArenaBytesPerWord +
           (size_t)P.block_count * P.block_cap * kArenaBytesPerWord;
}

int ensure_scratch(ccd_context* ctx, const Plan& P) {
    bool ok = grow(ctx->counters, 64 * 8) && grow(ctx->order, (size_t)P.n * 9) &&
              grow(ctx->rec_a, (size_t)P.rec_a_cap * P.rec_a_words * 8) &&
              grow(ctx->rec_b, (size_t)P.rec_b_cap * P.rec_b_words * 8) &&
              grow(ctx->pool, (size_t)P.pool_words * 8) &&
              grow(ctx->group_arena, (size_t)P.group_count * P.group_cap * kArenaBytesPerWord) &&
              grow(ctx->block_arena, (size_t)P.block_count * P.block_cap * kArenaBytesPerWord);
    return ok ? CCD_OK : CCD_ENOMEM;
}

// Device scratch of one launch (the context's buffers, or the carved static
// array of the allocation-free entry point).
struct Scratch {
    unsigned long long* counters;
    int64_t* order;
    uint64_t* rec_a;
    uint64_t* rec_b;
    uint64_t* pool;
    uint64_t* group_arena;
    uint64_t* block_arena;
};

Scratch context_scratch(ccd_context* ctx) {
    return Scratch{(unsigned long long*)ctx->counters.p, (int64_t*)ctx->order.p,
                   (uint64_t*)ctx->rec_a.p, (uint64_t*)ctx->rec_b.p, (uint64_t*)ctx->pool.p,
                   (uint64_t*)ctx->group_arena.p, (uint64_t*)ctx->block_arena.p};
}

// Words of a level kept in LDS by a group-engine kernel: the tuning's value,
// limited by what the workgroup may hold next to the kernel's static LDS (two
// buffers of 8-byte words), a multiple of 64.  Kernels that would use more
// than 64 KiB get the runtime's permission once.
int64_t group_lds_words(const void* fn, int64_t want, size_t lds_per_block) {
    static std::mutex mu;
    static std::vector<std::pair<const void*, size_t>> seen;  // kernel -> static LDS bytes
    size_t stat = 32768;
    {
        std::lock_guard<std::mutex> lk(mu);
        bool found = false;
        for (auto& e : seen)
            if (e.first == fn) { stat = e.second; found = true; }
        if (!found) {
            hipFuncAttributes at;
            if (hipFuncGetAttributes(&at, fn) == hipSuccess) stat = at.sharedSizeBytes;
            (void)hipGetLastError();
            seen.emplace_back(fn, stat);
        }
    }
    const size_t room = lds_per_block > stat ? lds_per_block - stat : 0;
    int64_t w = std::min<int64_t>(want, (int64_t)(room / 16)) & ~int64_t(63);
    if (w < 0) w = 0;
    if (w > 0 && 16 * (size_t)w + stat > 65536)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(16 * w));
    (void)hipGetLastError();
    return w;
}

// Issues the batch's kernel sequence on stream s (events ev[0..4] between the
// kernels when timed).
void enqueue(const ccd_tuning& tune, const Plan& P, const Scratch& X, BatchArgs a, hipStream_t s,
             bool persistent, bool timed, hipEvent_t* ev, size_t lds_per_block) {
    const int K = tune.lane_capacity;
    a.counters = X.counters;
    a.order = nullptr;
    if (timed) (void)hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, a.counters);
    if (persistent) {
        // level 0 of every query; the survivors, grouped by kind, go on
        hipLaunchKernelGGL(k_root, dim3((unsigned)((P.n + 511) / 512)), dim3(512), 0, s, a, X.order);
        a.order = X.order;
    }
    if (timed) (void)hipEventRecord(ev[1], s);
    LaneCfg lc;
    lc.capacity = K;
    lc.persistent = persistent ? 1 : 0;
    lc.survivors = persistent ? 1 : 0;
    lc.pad = 0;
    lc.budget = persistent ? (uint64_t)tune.lane_budget : ~0ull;
    lc.records = X.rec_a;
    lc.record_words = P.rec_a_words;
    lc.record_cap = P.rec_a_cap;
    lc.record_levels = (uint8_t*)(X.order + P.n);  // the order buffer's tail: n bytes
    if (persistent)
        hipLaunchKernelGGL(k_lane<true>, dim3(P.lane_grid), dim3(kLaneBlock), P.lane_lds, s, a, lc);
    else
        hipLaunchKernelGGL(k_lane<false>, dim3(P.lane_grid), dim3(kLaneBlock), P.lane_lds, s, a, lc);
    if (timed) (void)hipEventRecord(ev[2], s);

    // the lane engine's records, heavy-looking queries first (the order
    // buffer, n entries, is free once the lane engine has run)
    hipLaunchKernelGGL(k_order_records, dim3(1), dim3(1024), 0, s, (const unsigned long long*)X.counters,
                       (const uint8_t*)(X.order + P.n), P.rec_a_cap, (int32_t)kCntRecA, X.order);
    GroupCfg g;
    g.capacity = P.group_cap;
    g.arena = X.group_arena;
    g.in_records = X.rec_a;
    g.in_record_words = P.rec_a_words;
    g.in_record_cap = P.rec_a_cap;
    g.in_pool = nullptr;
    g.in_perm = X.order;
    g.in_count_idx = kCntRecA;
    g.in_take_idx = kCntRecATake;
    g.out_records = X.rec_b;
    g.out_record_words = P.rec_b_words;
    g.out_record_cap = P.rec_b_cap;
    g.out_pool = X.pool;
    g.out_pool_words = P.pool_words;
    g.out_count_idx = kCntRecB;
    g.tier = 1;
    // about two such hand-offs per block engine: more would queue there
    g.tail_records = 2 * (int64_t)P.block_count;
    {
        const void* fn;
        int threads = 64;
        // levels staged in LDS: the eight-wave and the three-waves-per-SIMD
        // single-wave kernels have a variant for it
        const bool lds = tune.group_lds_words > 0 &&
                         (tune.group_waves == 8 || (tune.group_waves == 1 && tune.group_occupancy == 3));
        switch (tune.group_waves) {
            case 8:
                fn = lds ? (const void*)&k_group<8, 1, true> : (const void*)&k_group<8, 1, false>;
                threads = 512;
                break;
            case 4: fn = (const void*)&k_group<4, 1, false>; threads = 256; break;
            case 2: fn = (const void*)&k_group<2, 1, false>; threads = 128; break;
            default:
                switch (tune.group_occupancy) {
                    case 4: fn = (const void*)&k_group<1, 4, false>; break;
                    case 3:
                        fn = lds ? (const void*)&k_group<1, 3, true> : (const void*)&k_group<1, 3, false>;
                        break;
                    case 2: fn = (const void*)&k_group<1, 2, false>; break;
                    default: fn = (const void*)&k_group<1, 1, false>;
                }
        }
        g.lds_words = lds ? std::min<int64_t>(group_lds_words(fn, tune.group_lds_words, lds_per_block),
                                              P.group_cap)
                          : 0;
        void* args[] = {&a, &g};
        (void)hipLaunchKernel(fn, dim3(P.group_count), dim3(threads), args,
                              (size_t)16 * g.lds_words, s);
    }
    if (timed) (void)hipEventRecord(ev[3], s);

    GroupCfg b;
    b.capacity = P.block_cap;
    b.arena = X.block_arena;
    b.in_records = X.rec_b;
    b.in_record_words = P.rec_b_words;
    b.in_record_cap = P.rec_b_cap;
    b.in_pool = X.pool;
    b.in_perm = nullptr;
    b.in_count_idx = kCntRecB;
    b.in_take_idx = kCntRecBTake;
    b.out_records = nullptr;
    b.out_record_words = 0;
    b.out_record_cap = 0;
    b.out_pool = nullptr;
    b.out_pool_words = 0;
    b.out_count_idx = 0;
    b.tier = 2;
    b.tail_records = 0;
    if (P.block_waves == 4) {
        b.lds_words = 0;
        hipLaunchKernelGGL((k_group<4, 1, false>), dim3(P.block_count), dim3(256), 0, s, a, b);
    } else if (tune.block_lds_words > 0) {
        b.lds_words = std::min<int64_t>(
            group_lds_words((const void*)&k_group<8, 1, true>, tune.block_lds_words, lds_per_block),
            P.block_cap);
        hipLaunchKernelGGL((k_group<8, 1, true>), dim3(P.block_count), dim3(512),
                           (size_t)16 * b.lds_words, s, a, b);
    } else {
        b.lds_words = 0;
        hipLaunchKernelGGL((k_group<8, 1, false>), dim3(P.block_count), dim3(512), 0, s, a, b);
    }
    if (timed) (void)hipEventRecord(ev[4], s);
}

// Everything the launch sequence depends on; a graph is reused while this is
// byte-for-byte unchanged.
struct LaunchKey {
    BatchArgs a;
    Plan P;
    ccd_tuning tune;
    void* bufs[7];
    int32_t persistent, timed;
};

void drop_graph(ccd_context* ctx) {
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->graph_exec = nullptr;
    ctx->graph = nullptr;
    ctx->graph_key_len = 0;
}

int launch(ccd_context* ctx, const Plan& P, BatchArgs a, hipStream_t s, bool persistent) {
    const bool timed = ctx->timing && ctx->have_events;
    ctx->last_timed = timed;
    ctx->last_valid = true;
    // per-kernel timing needs events between the kernels: launch eagerly then
    if (ctx->use_graphs && ctx->cap_stream && !timed) {
        LaunchKey key;
        std::memset(&key, 0, sizeof(key));
        key.a = a;
        key.P = P;
        key.tune = ctx->tune;
        void* bufs[7] = {ctx->counters.p, ctx->order.p, ctx->rec_a.p, ctx->group_arena.p,
                         ctx->rec_b.p, ctx->pool.p, ctx->block_arena.p};
        std::memcpy(key.bufs, bufs, sizeof(bufs));
        key.persistent = persistent;
        key.timed = timed;
        static_assert(sizeof(LaunchKey) <= sizeof(ctx->graph_key), "graph key size");
        const bool same = ctx->graph_exec && ctx->graph_key_len == sizeof(key) &&
                          std::memcmp(ctx->graph_key, &key, sizeof(key)) == 0;
        if (!same) {
            drop_graph(ctx);
            bool ok = hip_ok(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal),
                             "hipStreamBeginCapture");
            if (ok) {
                enqueue(ctx->tune, P, context_scratch(ctx), a, ctx->cap_stream, persistent, timed,
                        ctx->ev, ctx->lds_per_block);
                hipGraph_t g = nullptr;
                ok = hip_ok(hipStreamEndCapture(ctx->cap_stream, &g), "hipStreamEndCapture");
                if (ok) {
                    ctx->graph = g;
                    ok = hip_ok(hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0),
                                "hipGraphInstantiate");
                }
            }
            if (!ok) {
                drop_graph(ctx);
                return CCD_EDEVICE;
            }
            std::memcpy(ctx->graph_key, &key, sizeof(key));
            ctx->graph_key_len = sizeof(key);
            ctx->graph_builds += 1;
        } else {
            ctx->graph_replays += 1;
        }
        return hip_ok(hipGraphLaunch(ctx->graph_exec, s), "hipGraphLaunch") ? CCD_OK : CCD_EDEVICE;
    }
    enqueue(ctx->tune, P, context_scratch(ctx), a, s, persistent, timed, ctx->ev, ctx->lds_per_block);
    return hip_ok(hipGetLastError(), "kernel launch") ? CCD_OK : CCD_EDEVICE;
}

}  // namespace

namespace ccd {

// Plans scratch for a launch of a.n queries whose largest m_I is mi_max,
// grows the context's buffers and enqueues the kernel sequence on s.
int run_args(ccd_context* ctx, BatchArgs a, int64_t mi_max, hipStream_t s) {
    const bool persistent = ctx->engine == CCD_ENGINE_PERSISTENT;
    Plan P;
    int rc = make_plan(ctx, a.n, std::max<int64_t>(mi_max, 1), persistent, P);
    if (rc != CCD_OK) return rc;
    rc = ensure_scratch(ctx, P);
    if (rc != CCD_OK) return rc;
    return launch(ctx, P, a, s, persistent);
}

int reserve(ccd_context* ctx, int64_t n, int64_t mi_max) {
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    Plan P;
    int rc = make_plan(ctx, n, std::max<int64_t>(mi_max, 1), ctx->engine == CCD_ENGINE_PERSISTENT, P);
    if (rc != CCD_OK) return rc;
    rc = ensure_scratch(ctx, P);
    if (rc != CCD_OK) return rc;
    // a smaller batch leaves more of the budget to the engines and the pool:
    // hold their sizes at this plan's, so that no later batch of up to n
    // queries plans a larger buffer (reallocating it would stall the device)
    ctx->tune.group_count = P.group_count;
    ctx->tune.block_count = P.block_count;
    ctx->tune.handoff_words = P.pool_words;
    return CCD_OK;
}

bool host_valid(const double X[24], int kind, double delta, int64_t max_iter, double min_sep) {
    return host_query_valid(X, kind, delta, max_iter, min_sep);
}

bool record_hip(hipError_t e, const char* what) { return hip_ok(e, what); }

void set_last_error(const char* msg) { std::snprintf(g_last_error, sizeof(g_last_error), "%s", msg); }

}  // namespace ccd

namespace {

std::mutex g_default_mu;
ccd_context* g_default = nullptr;

int single(int kind, const double x0[4][3], const double x1[4][3], const ccd_params* p,
           ccd_result* out) {
    if (!x0 || !x1 || !p || !out) return CCD_EINVAL;
    std::lock_guard<std::mutex> lk(g_default_mu);
    if (!g_default) {
        int rc = ccd_context_create(0, (size_t)1 << 30, &g_default);
        if (rc != CCD_OK) return rc;
    }
    double pos[24];
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) {
            pos[3 * k + c] = x0[k][c];
            pos[3 * (k + 4) + c] = x1[k][c];
        }
    ccd_batch_desc d;
    std::memset(&d, 0, sizeof(d));
    d.n = 1;
    d.pos = pos;
    d.kind = nullptr;
    d.default_kind = (uint8_t)kind;
    d.params = *p;
    d.on_device = 0;
    double toi, tw;
    uint8_t hit, st;
    uint64_t nc;
    ccd_result_soa o = {&toi, &tw, &hit, &nc, &st};
    int rc = ccd_batch(g_default, &d, &o, nullptr);
    if (rc != CCD_OK) return rc;
    std::memset(out, 0, sizeof(*out));
    out->toi = toi;
    out->t_width = tw;
    out->n_checks = nc;
    out->hit = hit;
    out->status = st;
    return CCD_OK;
}

}  // namespace

extern "C" {

void ccd_params_default(ccd_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->delta = 1e-6;
    p->max_iter = 1000000;
    p->min_sep = 0.0;
    p->t_max = 1.0;
}

const char* ccd_last_error(void) { return g_last_error; }

const char* ccd_strerror(int code) {
    switch (code) {
        case CCD_OK: return "ok";
        case CCD_EINVAL: return "invalid argument";
        case CCD_ENOMEM: return "device memory budget exceeded";
        case CCD_EDEVICE: return "HIP device error";
        case CCD_EAGAIN: return "request does not fit now";
        case CCD_ETIMEDOUT: return "timed out";
        case CCD_ECANCELED: return "cancelled";
        default: return "unknown error";
    }
}

int ccd_context_create(int device, size_t mem_budget_bytes, ccd_context** out) {
    if (!out) return CCD_EINVAL;
    int ndev = 0;
    if (!hip_ok(hipGetDeviceCount(&ndev), "hipGetDeviceCount")) return CCD_EDEVICE;
    if (ndev <= device || device < 0) {
        std::snprintf(g_last_error, sizeof(g_last_error), "no HIP device %d", device);
        return CCD_EDEVICE;
    }
    if (set_device(device) != CCD_OK) return CCD_EDEVICE;
    ccd_context* c = new ccd_context();
    c->device = device;
    c->budget = mem_budget_bytes ? mem_budget_bytes : ((size_t)16 << 30);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) {
        c->num_cu = prop.multiProcessorCount;
        if (prop.sharedMemPerBlock >= 16384) c->lds_per_block = prop.sharedMemPerBlock;
    }
    default_tuning(c->tune, c->num_cu);
    c->have_events = true;
    for (int i = 0; i < 5; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) c->have_events = false;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        c->cap_stream = nullptr;
    (void)hipGetLastError();
    *out = c;
    return CCD_OK;
}

void ccd_context_destroy(ccd_context* c) {
    if (!c) return;
    (void)set_device(c->device);
    (void)hipDeviceSynchronize();
    for (DevBuf* b : {&c->counters, &c->order, &c->rec_a, &c->group_arena, &c->rec_b, &c->pool,
                      &c->block_arena, &c->io, &c->gather})
        release(*b);
    if (c->have_events)
        for (int i = 0; i < 5; ++i) (void)hipEventDestroy(c->ev[i]);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

int ccd_plan_scratch(const ccd_tuning* tuning, int num_cu, size_t mem_budget_bytes, int64_t n,
                     int64_t max_iter, int engine, ccd_scratch_plan* out) {
    if (!out || num_cu < 1 || n < 0 || max_iter < 1 ||
        (engine != CCD_ENGINE_PERSISTENT && engine != CCD_ENGINE_PLAIN)) {
        set_last_error("ccd_plan_scratch: bad argument");
        return CCD_EINVAL;
    }
    ccd_tuning t;
    default_tuning(t, num_cu);
    if (tuning) {
        ccd_tuning n2 = t;
        const ccd_tuning* u = tuning;
        if (u->lane_waves_per_cu) n2.lane_waves_per_cu = u->lane_waves_per_cu;
        if (u->lane_capacity) n2.lane_capacity = u->lane_capacity;
        if (u->lane_budget) n2.lane_budget = u->lane_budget;
        if (u->group_waves) n2.group_waves = u->group_waves;
        if (u->group_count) n2.group_count = u->group_count;
        if (u->group_capacity) n2.group_capacity = u->group_capacity;
        if (u->block_count) n2.block_count = u->block_count;
        if (u->group_occupancy) n2.group_occupancy = u->group_occupancy;
        if (u->block_capacity) n2.block_capacity = u->block_capacity < 0 ? 0 : u->block_capacity;
        if (u->handoff_words) n2.handoff_words = u->handoff_words < 0 ? 0 : u->handoff_words;
        if (u->group_lds_words) n2.group_lds_words = u->group_lds_words < 0 ? 0 : u->group_lds_words;
        if (u->block_lds_words) n2.block_lds_words = u->block_lds_words < 0 ? 0 : u->block_lds_words;
        clamp_tuning(n2);
        t = n2;
    }
    Plan P;
    const size_t budget = mem_budget_bytes ? mem_budget_bytes : ((size_t)16 << 30);
    const int rc = plan_for(t, num_cu, budget, n, max_iter, engine == CCD_ENGINE_PERSISTENT, P);
    if (rc != CCD_OK) return rc;
    std::memset(out, 0, sizeof(*out));
    out->bytes = plan_bytes(P);
    out->lane_lds_bytes = P.lane_lds;
    out->lane_blocks = P.lane_grid;
    out->group_count = P.group_count;
    out->group_capacity = P.group_cap;
    out->block_count = P.block_count;
    out->block_capacity = P.block_cap;
    out->handoff_words = P.pool_words;
    return CCD_OK;
}

int ccd_context_set_engine(ccd_context* c, int engine) {
    if (!c || (engine != CCD_ENGINE_PERSISTENT && engine != CCD_ENGINE_PLAIN)) return CCD_EINVAL;
    c->engine = engine;
    return CCD_OK;
}

int ccd_context_get_tuning(ccd_context* c, ccd_tuning* out) {
    if (!c || !out) return CCD_EINVAL;
    *out = c->tune;
    return CCD_OK;
}

int ccd_context_set_tuning(ccd_context* c, const ccd_tuning* t) {
    if (!c || !t) return CCD_EINVAL;
    ccd_tuning n = c->tune;
    if (t->lane_waves_per_cu) n.lane_waves_per_cu = t->lane_waves_per_cu;
    if (t->lane_capacity) n.lane_capacity = t->lane_capacity;
    if (t->lane_budget) n.lane_budget = t->lane_budget;
    if (t->group_waves) n.group_waves = t->group_waves;
    if (t->group_count) n.group_count = t->group_count;
    if (t->group_capacity) n.group_capacity = t->group_capacity;
    if (t->block_count) n.block_count = t->block_count;
    if (t->group_occupancy) n.group_occupancy = t->group_occupancy;
    if (t->block_capacity) n.block_capacity = t->block_capacity < 0 ? 0 : t->block_capacity;
    if (t->handoff_words) n.handoff_words = t->handoff_words < 0 ? 0 : t->handoff_words;
    if (t->group_lds_words) n.group_lds_words = t->group_lds_words < 0 ? 0 : t->group_lds_words;
    if (t->block_lds_words) n.block_lds_words = t->block_lds_words < 0 ? 0 : t->block_lds_words;
    clamp_tuning(n);
    c->tune = n;
    return CCD_OK;
}

int ccd_context_enable_graphs(ccd_context* c, int enable) {
    if (!c) return CCD_EINVAL;
    c->use_graphs = enable != 0;
    if (!c->use_graphs) drop_graph(c);
    return CCD_OK;
}

int ccd_context_graph_counts(ccd_context* c, uint64_t* builds, uint64_t* replays) {
    if (!c || !builds || !replays) return CCD_EINVAL;
    *builds = c->graph_builds;
    *replays = c->graph_replays;
    return CCD_OK;
}

int ccd_context_enable_timing(ccd_context* c, int enable) {
    if (!c) return CCD_EINVAL;
    c->timing = enable != 0;
    return CCD_OK;
}

int ccd_context_last_stats(ccd_context* c, ccd_stats* out) {
    if (!c || !out) return CCD_EINVAL;
    std::memset(out, 0, sizeof(*out));
    if (!c->last_valid) return CCD_OK;
    if (set_device(c->device) != CCD_OK) return CCD_EDEVICE;
    if (!hip_ok(hipDeviceSynchronize(), "hipDeviceSynchronize")) return CCD_EDEVICE;
    unsigned long long h[kCntEnd];
    if (!hip_ok(hipMemcpy(h, c->counters.p, sizeof(h), hipMemcpyDeviceToHost), "copy counters"))
        return CCD_EDEVICE;
    for (int t = 0; t < 3; ++t)
        for (int k = 0; k < 2; ++k) out->checks[t][k] = h[kCntChecks + 2 * t + k];
    out->promoted[0] = h[kCntRecA];
    out->promoted[1] = h[kCntRecB];
    for (int t = 0; t < 3; ++t) out->lane_slots[t] = h[kCntSlots + t];
    out->overflowed = h[kCntOverflow];
    out->restarted = h[kCntRestart];
    out->deep = h[kCntDeep];
    out->handoff_words = h[kCntPool];
    out->probes[0] = h[kCntProbe];
    out->probes[1] = h[kCntProbeHit];
    if (c->last_timed)
        for (int i = 0; i < 4; ++i)
            if (!hip_ok(hipEventElapsedTime(&out->kernel_ms[i], c->ev[i], c->ev[i + 1]),
                        "hipEventElapsedTime"))
                out->kernel_ms[i] = 0.0f;
    return CCD_OK;
}

int ccd_batch(ccd_context* ctx, const ccd_batch_desc* d, const ccd_result_soa* out, void* stream) {
    if (!ctx || !d || !out) {
        set_last_error("ccd_batch: null context, descriptor or outputs");
        return CCD_EINVAL;
    }
    if (d->n < 0 || !params_ok(d->params) || d->default_kind > 1) {
        set_last_error("ccd_batch: negative count, bad parameters (t_max, flags) or kind");
        return CCD_EINVAL;
    }
    if (d->n == 0) return CCD_OK;
    if (!d->pos || !out->toi || !out->t_width || !out->hit || !out->n_checks || !out->status) {
        set_last_error("ccd_batch: null input or output array");
        return CCD_EINVAL;
    }
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = d->n;

    // batch-level parameter checks that do not depend on the queries
    int64_t mi_max = d->params.max_iter;
    if (!d->max_iter_q && d->params.max_iter < 1) {
        set_last_error("ccd_batch: max_iter < 1");
        return CCD_EINVAL;
    }

    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.delta = d->params.delta;
    a.max_iter = d->params.max_iter;
    a.min_sep = d->params.min_sep;
    a.t_max = d->params.t_max;
    a.flags = d->params.flags;
    a.default_kind = d->default_kind;

    if (!d->on_device) {
        // validate everything on the host before touching the device
        for (int64_t q = 0; q < n; ++q) {
            double X[24];
            for (int r = 0; r < 24; ++r) X[r] = d->pos[r * n + q];
            const int kind = d->kind ? d->kind[q] : d->default_kind;
            const double dl = d->delta_q ? d->delta_q[q] : d->params.delta;
            const int64_t mi = d->max_iter_q ? d->max_iter_q[q] : d->params.max_iter;
            const double ms = d->min_sep_q ? d->min_sep_q[q] : d->params.min_sep;
            if (!host_query_valid(X, kind, dl, mi, ms)) {
                std::snprintf(g_last_error, sizeof(g_last_error),
                              "ccd_batch: query %lld is invalid (coordinates, kind, delta, "
                              "max_iter or min_sep)", (long long)q);
                return CCD_EINVAL;
            }
            if (d->max_iter_q) mi_max = std::max(mi_max, mi);
        }
        if (d->max_iter_q) {
            mi_max = 1;
            for (int64_t q = 0; q < n; ++q) mi_max = std::max(mi_max, d->max_iter_q[q]);
        }
        // stage inputs and outputs in device memory
        size_t off = 0;
        auto take = [&](size_t bytes) { size_t o = off; off += (bytes + 255) & ~(size_t)255; return o; };
        const size_t o_pos = take((size_t)24 * n * 8);
        const size_t o_kind = d->kind ? take((size_t)n) : 0;
        const size_t o_dq = d->delta_q ? take((size_t)n * 8) : 0;
        const size_t o_mq = d->max_iter_q ? take((size_t)n * 8) : 0;
        const size_t o_sq = d->min_sep_q ? take((size_t)n * 8) : 0;
        const size_t o_toi = take((size_t)n * 8), o_tw = take((size_t)n * 8);
        const size_t o_hit = take((size_t)n), o_nc = take((size_t)n * 8), o_st = take((size_t)n);
        if (!grow(ctx->io, off)) return CCD_ENOMEM;
        char* base = (char*)ctx->io.p;
        bool ok = hip_ok(hipMemcpyAsync(base + o_pos, d->pos, (size_t)24 * n * 8, hipMemcpyHostToDevice, s), "copy pos");
        if (ok && d->kind) ok = hip_ok(hipMemcpyAsync(base + o_kind, d->kind, n, hipMemcpyHostToDevice, s), "copy kind");
        if (ok && d->delta_q) ok = hip_ok(hipMemcpyAsync(base + o_dq, d->delta_q, n * 8, hipMemcpyHostToDevice, s), "copy delta");
        if (ok && d->max_iter_q) ok = hip_ok(hipMemcpyAsync(base + o_mq, d->max_iter_q, n * 8, hipMemcpyHostToDevice, s), "copy max_iter");
        if (ok && d->min_sep_q) ok = hip_ok(hipMemcpyAsync(base + o_sq, d->min_sep_q, n * 8, hipMemcpyHostToDevice, s), "copy min_sep");
        if (!ok) return CCD_EDEVICE;
        a.pos = (const double*)(base + o_pos);
        a.kind = d->kind ? (const uint8_t*)(base + o_kind) : nullptr;
        a.delta_q = d->delta_q ? (const double*)(base + o_dq) : nullptr;
        a.max_iter_q = d->max_iter_q ? (const int64_t*)(base + o_mq) : nullptr;
        a.min_sep_q = d->min_sep_q ? (const double*)(base + o_sq) : nullptr;
        a.toi = (double*)(base + o_toi);
        a.t_width = (double*)(base + o_tw);
        a.hit = (uint8_t*)(base + o_hit);
        a.n_checks = (uint64_t*)(base + o_nc);
        a.status = (uint8_t*)(base + o_st);
        int rc = ccd::run_args(ctx, a, mi_max, s);
        if (rc != CCD_OK) return rc;
        ok = hip_ok(hipMemcpyAsync(out->toi, a.toi, n * 8, hipMemcpyDeviceToHost, s), "copy toi") &&
             hip_ok(hipMemcpyAsync(out->t_width, a.t_width, n * 8, hipMemcpyDeviceToHost, s), "copy t_width") &&
             hip_ok(hipMemcpyAsync(out->hit, a.hit, n, hipMemcpyDeviceToHost, s), "copy hit") &&
             hip_ok(hipMemcpyAsync(out->n_checks, a.n_checks, n * 8, hipMemcpyDeviceToHost, s), "copy n_checks") &&
             hip_ok(hipMemcpyAsync(out->status, a.status, n, hipMemcpyDeviceToHost, s), "copy status") &&
             hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
        return ok ? CCD_OK : CCD_EDEVICE;
    }

    // device pointers: per-query m_I must be known on the host to size the
    // widest arena; read it back when it varies per query (synchronises)
    if (d->max_iter_q) {
        std::vector<int64_t> h(n);
        if (!hip_ok(hipMemcpyAsync(h.data(), d->max_iter_q, n * 8, hipMemcpyDeviceToHost, s), "copy max_iter") ||
            !hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize"))
            return CCD_EDEVICE;
        mi_max = 1;
        for (int64_t v : h) mi_max = std::max(mi_max, v);
    }
    a.pos = d->pos;
    a.kind = d->kind;
    a.delta_q = d->delta_q;
    a.max_iter_q = d->max_iter_q;
    a.min_sep_q = d->min_sep_q;
    a.toi = out->toi;
    a.t_width = out->t_width;
    a.hit = out->hit;
    a.n_checks = out->n_checks;
    a.status = out->status;
    return ccd::run_args(ctx, a, mi_max, s);
}

// ---------------------------------------------------------------------------
// Allocation-free batches.  The scratch of ccd_batch_noalloc is one static
// device array per GPU (the code object's copy on each device), of kNoAllocBytes.
// Host code never uses the array's name as an address: the device address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress, that
// device current) and kept in g_noalloc_ptr.

namespace {

constexpr size_t kNoAllocBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (current), or null on failure.
void* noalloc_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        void* p = nullptr;
        if (!hip_ok(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"))
            return nullptr;
        g_noalloc_ptr[device] = p;
    }
    return g_noalloc_ptr[device];
}

// Carves the plan's buffers out of [base, base + bytes) at 256-byte offsets;
// false if they do not fit.
bool carve(const Plan& P, void* base, size_t bytes, Scratch& X) {
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = sadd(off, (b + 255) & ~(size_t)255);
        return (unsigned char*)base + o;
    };
    X.counters = (unsigned long long*)take(64 * 8);
    X.order = (int64_t*)take((size_t)P.n * 9);  // order, then one level byte per record
    X.rec_a = (uint64_t*)take(smul(smul((size_t)P.rec_a_cap, (size_t)P.rec_a_words), 8));
    X.rec_b = (uint64_t*)take(smul(smul((size_t)P.rec_b_cap, (size_t)P.rec_b_words), 8));
    X.pool = (uint64_t*)take(smul((size_t)P.pool_words, 8));
    X.group_arena = (uint64_t*)take(smul((size_t)P.group_count * P.group_cap, kArenaBytesPerWord));
    X.block_arena = (uint64_t*)take(smul((size_t)P.block_count * P.block_cap, kArenaBytesPerWord));
    return off <= bytes;
}

}  // namespace

extern "C" int ccd_batch_noalloc(ccd_context* ctx, const ccd_batch_desc* d, const ccd_result_soa* out,
                                 void* stream) {
    if (!ctx || !d || !out) {
        set_last_error("ccd_batch_noalloc: null context, descriptor or outputs");
        return CCD_EINVAL;
    }
    if (!d->on_device) {
        set_last_error("ccd_batch_noalloc: inputs and outputs must be device memory");
        return CCD_EINVAL;
    }
    if (d->n < 0 || !params_ok(d->params) || d->default_kind > 1 ||
        (!d->max_iter_q && d->params.max_iter < 1)) {
        set_last_error("ccd_batch_noalloc: negative count, bad parameters or kind");
        return CCD_EINVAL;
    }
    if (d->n == 0) return CCD_OK;
    if (!d->pos || !out->toi || !out->t_width || !out->hit || !out->n_checks || !out->status) {
        set_last_error("ccd_batch_noalloc: null input or output array");
        return CCD_EINVAL;
    }
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    void* base = noalloc_scratch(ctx->device);
    if (!base) return CCD_EDEVICE;
    const bool persistent = ctx->engine == CCD_ENGINE_PERSISTENT;
    // per-query m_I are not read back (that would need a host buffer): the
    // block arena then takes what the plan allows
    const int64_t mi_max = d->max_iter_q ? INT64_MAX : d->params.max_iter;
    Plan P;
    // (the budget leaves room for the 256-byte alignment of the seven buffers)
    if (plan_for(ctx->tune, ctx->num_cu, kNoAllocBytes - 7 * 256, d->n, mi_max, persistent, P) !=
        CCD_OK) {
        std::snprintf(g_last_error, sizeof(g_last_error),
                      "ccd_batch_noalloc: %lld queries need more scratch than the %zu MiB "
                      "allocation-free array",
                      (long long)d->n, kNoAllocBytes >> 20);
        return CCD_ENOMEM;
    }
    Scratch X;
    if (!carve(P, base, kNoAllocBytes, X)) {
        set_last_error("ccd_batch_noalloc: scratch plan does not fit the static array");
        return CCD_ENOMEM;
    }
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = d->n;
    a.pos = d->pos;
    a.kind = d->kind;
    a.delta_q = d->delta_q;
    a.max_iter_q = d->max_iter_q;
    a.min_sep_q = d->min_sep_q;
    a.delta = d->params.delta;
    a.max_iter = d->params.max_iter;
    a.min_sep = d->params.min_sep;
    a.t_max = d->params.t_max;
    a.flags = d->params.flags;
    a.default_kind = d->default_kind;
    a.toi = out->toi;
    a.t_width = out->t_width;
    a.hit = out->hit;
    a.n_checks = out->n_checks;
    a.status = out->status;
    // eager launches (a caller may be capturing the stream); the context's
    // counters and graph are not touched, so ccd_context_last_stats does not
    // describe this call
    ctx->last_valid = false;
    enqueue(ctx->tune, P, X, a, (hipStream_t)stream, persistent, false, nullptr, ctx->lds_per_block);
    return hip_ok(hipGetLastError(), "ccd_batch_noalloc launch") ? CCD_OK : CCD_EDEVICE;
}

// ---------------------------------------------------------------------------
// Autotuner: coordinate descent over the launch/capacity knobs, each candidate
// timed with events around whole batches.  Results do not depend on tuning, so
// the search only trades speed.

namespace {

float time_batch(ccd_context* ctx, const ccd_batch_desc* d, const ccd_result_soa* out,
                 hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, int* rc) {
    *rc = ccd_batch(ctx, d, out, s);  // warm-up (also builds the graph)
    if (*rc != CCD_OK) return -1.0f;
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, s);
        *rc = ccd_batch(ctx, d, out, s);
        if (*rc != CCD_OK) return -1.0f;
        (void)hipEventRecord(e1, s);
        if (!hip_ok(hipEventSynchronize(e1), "hipEventSynchronize")) {
            *rc = CCD_EDEVICE;
            return -1.0f;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    return t[t.size() / 2];
}

}  // namespace

int ccd_autotune(ccd_context* ctx, const ccd_batch_desc* d, const ccd_result_soa* out,
                 void* stream, int max_trials, ccd_tuning* best_out, float* best_ms_out) {
    if (!ctx || !d || !out || !d->on_device) return CCD_EINVAL;
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (!hip_ok(hipEventCreate(&e0), "hipEventCreate")) return CCD_EDEVICE;
    if (!hip_ok(hipEventCreate(&e1), "hipEventCreate")) {
        (void)hipEventDestroy(e0);
        return CCD_EDEVICE;
    }
    const bool timing = ctx->timing;
    ctx->timing = false;
    const int cu = ctx->num_cu;
    const ccd_tuning start = ctx->tune;
    ccd_tuning best = ctx->tune;
    int rc = CCD_OK;
    int trials = 0;
    float best_ms = time_batch(ctx, d, out, s, e0, e1, 3, &rc);
    ++trials;
    // knob candidates; group_count follows the occupancy (4 SIMDs per CU)
    struct Knob { int id; std::vector<int64_t> vals; };
    const std::vector<Knob> knobs = {
        {0, {2, 3, 4}},            // group_occupancy (with group_count = 4 * cu * occ)
        {1, {32, 64, 128, 192, 256, 384, 512}},  // lane_budget
        {2, {8, 16, 32}},          // lane_capacity
        {3, {4, 8, 12}},           // lane_waves_per_cu
        {4, {1, 2, 4}},            // group_waves
        {5, {0, 256, 512}},        // group_lds_words
    };
    for (int pass = 0; pass < 2 && rc == CCD_OK; ++pass) {
        bool improved = false;
        for (const Knob& k : knobs) {
            for (int64_t v : k.vals) {
                if (max_trials > 0 && trials >= max_trials) break;
                ccd_tuning t = best;
                switch (k.id) {
                    case 0: t.group_occupancy = (int32_t)v; t.group_count = (int32_t)(4 * cu * v); break;
                    case 1: t.lane_budget = v; break;
                    case 2: t.lane_capacity = (int32_t)v; break;
                    case 3: t.lane_waves_per_cu = (int32_t)v; break;
                    case 4: t.group_waves = (int32_t)v;
                            t.group_count = (int32_t)(v == 1 ? 4 * cu * t.group_occupancy : 4 * cu * 2 / v);
                            break;
                    case 5: t.group_lds_words = (int32_t)v; break;
                }
                clamp_tuning(t);
                if (std::memcmp(&t, &best, sizeof(t)) == 0) continue;
                ctx->tune = t;
                const float ms = time_batch(ctx, d, out, s, e0, e1, 3, &rc);
                ++trials;
                if (rc != CCD_OK) break;
                if (ms > 0.0f && ms < best_ms * 0.98f) {
                    best_ms = ms;
                    best = t;
                    improved = true;
                }
            }
            if (rc != CCD_OK) break;
        }
        if (!improved) break;
    }
    // confirm against the starting point with more repetitions
    if (rc == CCD_OK && std::memcmp(&best, &start, sizeof(best)) != 0) {
        ctx->tune = start;
        const float ms_start = time_batch(ctx, d, out, s, e0, e1, 5, &rc);
        ctx->tune = best;
        const float ms_best = rc == CCD_OK ? time_batch(ctx, d, out, s, e0, e1, 5, &rc) : -1.0f;
        if (rc == CCD_OK && !(ms_best < ms_start)) {
            best = start;
            best_ms = ms_start;
        } else if (rc == CCD_OK) {
            best_ms = ms_best;
        }
    }
    ctx->tune = best;
    ctx->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != CCD_OK) return rc;
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return CCD_OK;
}

// Tuning cache: one line per (device, workload key):
//   <arch> <cus> <hip-version> <key> <the twelve ccd_tuning fields>
namespace {
void device_tag(ccd_context* ctx, char* arch, size_t n, int* hipver) {
    hipDeviceProp_t prop;
    std::snprintf(arch, n, "unknown");
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess)
        std::snprintf(arch, n, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
        if (*c == ' ' || *c == ':') *c = '_';
    *hipver = 0;
    (void)hipRuntimeGetVersion(hipver);
    (void)hipGetLastError();
}
}  // namespace

int ccd_tuning_cache_store(ccd_context* ctx, const char* path, const char* key) {
    if (!ctx || !path || !key || !*key || std::strpbrk(key, " \t\n")) return CCD_EINVAL;
    char arch[128];
    int ver;
    device_tag(ctx, arch, sizeof(arch), &ver);
    std::vector<std::string> keep;
    if (FILE* f = std::fopen(path, "r")) {
        char line[512];
        while (std::fgets(line, sizeof(line), f)) {
            char a[128], k[128];
            int c, v;
            if (std::sscanf(line, "%127s %d %d %127s", a, &c, &v, k) == 4 &&
                std::strcmp(a, arch) == 0 && c == ctx->num_cu && v == ver && std::strcmp(k, key) == 0)
                continue;
            keep.emplace_back(line);
        }
        std::fclose(f);
    }
    FILE* f = std::fopen(path, "w");
    if (!f) return CCD_EINVAL;
    for (const std::string& l : keep) std::fputs(l.c_str(), f);
    const ccd_tuning& t = ctx->tune;
    std::fprintf(f, "%s %d %d %s %d %d %lld %d %d %lld %d %d %lld %lld %d %d\n", arch, ctx->num_cu,
                 ver, key, t.lane_waves_per_cu, t.lane_capacity, (long long)t.lane_budget,
                 t.group_waves, t.group_count, (long long)t.group_capacity, t.block_count,
                 t.group_occupancy, (long long)t.block_capacity, (long long)t.handoff_words,
                 t.group_lds_words, t.block_lds_words);
    std::fclose(f);
    return CCD_OK;
}

int ccd_tuning_cache_load(ccd_context* ctx, const char* path, const char* key) {
    if (!ctx || !path || !key) return CCD_EINVAL;
    char arch[128];
    int ver;
    device_tag(ctx, arch, sizeof(arch), &ver);
    FILE* f = std::fopen(path, "r");
    if (!f) return CCD_EAGAIN;
    char line[512];
    int found = 0;
    ccd_tuning t = ctx->tune;
    while (std::fgets(line, sizeof(line), f)) {
        char a[128], k[128];
        int c, v;
        long long lb, gc, bc, hw;
        ccd_tuning r{};
        if (std::sscanf(line, "%127s %d %d %127s %d %d %lld %d %d %lld %d %d %lld %lld %d %d", a, &c,
                        &v, k, &r.lane_waves_per_cu, &r.lane_capacity, &lb, &r.group_waves,
                        &r.group_count, &gc, &r.block_count, &r.group_occupancy, &bc, &hw,
                        &r.group_lds_words, &r.block_lds_words) == 16 &&
            std::strcmp(a, arch) == 0 && c == ctx->num_cu && v == ver && std::strcmp(k, key) == 0) {
            r.lane_budget = lb;
            r.group_capacity = gc;
            r.block_capacity = bc;
            r.handoff_words = hw;
            t = r;
            found = 1;
        }
    }
    std::fclose(f);
    if (!found) return CCD_EAGAIN;
    clamp_tuning(t);
    ctx->tune = t;
    return CCD_OK;
}

int ccd_min_toi(ccd_context* ctx, const double* toi, int64_t n, double* out, void* stream) {
    if (!ctx || n < 0 || !out || (n > 0 && !toi)) {
        set_last_error("ccd_min_toi: null pointer or negative n");
        return CCD_EINVAL;
    }
    if (((uintptr_t)out & 7) != 0) {
        set_last_error("ccd_min_toi: out is not 8-byte aligned");
        return CCD_EINVAL;
    }
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* o = reinterpret_cast<unsigned long long*>(out);
    hipLaunchKernelGGL(k_min_toi_init, dim3(1), dim3(64), 0, s, o);
    if (n > 0) {
        const int64_t blocks = std::min<int64_t>((n + 255) / 256, (int64_t)ctx->num_cu * 2);
        hipLaunchKernelGGL(k_min_toi, dim3((unsigned)blocks), dim3(256), 0, s, toi, n, o);
    }
    if (!record_hip(hipGetLastError(), "ccd_min_toi launch")) return CCD_EDEVICE;
    return CCD_OK;
}

int ccd_scene_gamma(ccd_context* ctx, const double* v0, const double* v1, int64_t n_vertices,
                    double* gamma, void* stream) {
    if (!ctx || n_vertices < 0 || !gamma || (n_vertices > 0 && (!v0 || !v1))) {
        set_last_error("ccd_scene_gamma: null pointer or negative count");
        return CCD_EINVAL;
    }
    if (((uintptr_t)gamma & 7) != 0) {
        set_last_error("ccd_scene_gamma: gamma is not 8-byte aligned");
        return CCD_EINVAL;
    }
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* g = reinterpret_cast<unsigned long long*>(gamma);
    hipLaunchKernelGGL(k_scene_gamma_init, dim3(1), dim3(64), 0, s, g);
    if (n_vertices > 0) {
        const int64_t blocks = std::min<int64_t>((n_vertices + 255) / 256, (int64_t)ctx->num_cu * 2);
        hipLaunchKernelGGL(k_scene_gamma, dim3((unsigned)blocks), dim3(256), 0, s, v0, v1,
                           n_vertices, g);
    }
    if (!record_hip(hipGetLastError(), "ccd_scene_gamma launch")) return CCD_EDEVICE;
    return CCD_OK;
}

int ccd_batch_indexed(ccd_context* ctx, const ccd_indexed_desc* d, const ccd_result_soa* out,
                      void* stream) {
    if (!ctx || !d || !out) {
        set_last_error("ccd_batch_indexed: null context, descriptor or outputs");
        return CCD_EINVAL;
    }
    if (d->n < 0 || d->n_vertices < 0 || !params_ok(d->params) || d->default_kind > 1 ||
        d->params.max_iter < 1) {
        set_last_error("ccd_batch_indexed: negative count, bad parameters or kind");
        return CCD_EINVAL;
    }
    if (!d->on_device) {
        set_last_error("ccd_batch_indexed: inputs and outputs must be device memory");
        return CCD_EINVAL;
    }
    if (d->n == 0) return CCD_OK;
    if (!d->ids || (d->n_vertices > 0 && (!d->v0 || !d->v1)) || !out->toi || !out->t_width ||
        !out->hit || !out->n_checks || !out->status) {
        set_last_error("ccd_batch_indexed: null input or output array");
        return CCD_EINVAL;
    }
    if (set_device(ctx->device) != CCD_OK) return CCD_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = d->n;
    if ((size_t)24 * n * 8 > ctx->budget) return CCD_ENOMEM;
    if (!grow(ctx->gather, (size_t)24 * n * 8)) return CCD_ENOMEM;
    double* pos = (double*)ctx->gather.p;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, d->v0,
                       d->v1, d->ids, d->n_vertices, pos);
    if (!record_hip(hipGetLastError(), "ccd_batch_indexed gather")) return CCD_EDEVICE;
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.pos = pos;
    a.kind = d->kind;
    a.default_kind = d->default_kind;
    a.delta = d->params.delta;
    a.max_iter = d->params.max_iter;
    a.min_sep = d->params.min_sep;
    a.t_max = d->params.t_max;
    a.flags = d->params.flags;
    a.gamma = d->gamma;
    a.toi = out->toi;
    a.t_width = out->t_width;
    a.hit = out->hit;
    a.n_checks = out->n_checks;
    a.status = out->status;
    return ccd::run_args(ctx, a, d->params.max_iter, s);
}

int ccd_vf(const double x0[4][3], const double x1[4][3], const ccd_params* p, ccd_result* out) {
    return single(CCD_KIND_VF, x0, x1, p, out);
}

int ccd_ee(const double x0[4][3], const double x1[4][3], const ccd_params* p, ccd_result* out) {
    return single(CCD_KIND_EE, x0, x1, p, out);
}

}  // extern "C"
