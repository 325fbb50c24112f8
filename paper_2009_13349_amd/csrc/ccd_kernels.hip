// Kernels of the MI355X CCD library.
//
// The root finder is Alg. 2 of the paper, run level by level.  All boxes of a
// level are checked; the sequential algorithm's decisions (it pops boxes in
// (level, t_lo, u_lo, v_lo) order) are then recovered with reductions over the
// level, so no sort is needed:
//   * f = the smallest colliding key; "first colliding box" of Alg. 2;
//   * n at f is N + rank(f) + 1, rank = number of keys below f on the level;
//   * the m_I test of Alg. 2 can only fire on a level with N + |L| >= m_I; it
//     fires at f, or later iff N + rank(max colliding key) + 1 >= m_I;
//   * the remembered (carried) terminal box is the smallest t_lo among the
//     terminal colliding boxes other than f;
//   * the next level is the admitted children of the non-terminal colliding
//     boxes.
// Three engines share this level logic:
//   lane engine  - one lane owns one query, its frontier in a small per-lane
//                  arena; "plain" = one thread per query, "persistent" = lanes
//                  pull queries from a cursor and hand long ones on;
//   group engine - W wavefronts (one block) share one query whose frontier is
//                  too wide for a lane; used with W = 1 for wide queries and
//                  W = 8 with a 2 m_I-box arena for the widest.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ccd_device.hpp"
#include "ccd_internal.h"

namespace ccd {

struct Query {
    double X[24];
    double eps[3];
    double kappa[3];
    double delta;
    double min_sep;
    int64_t max_iter;
    int kind;
    bool literal;
};

struct State {
    uint64_t N;      // checks before this level
    double tpend;    // carried terminal box t_lo (+inf: none)
    double wpend;
    int32_t level;
    int32_t d[3];
    uint32_t cnt;    // boxes on this level
};

struct LevelInfo {
    double wt, wu, wv;
    int axis;
    bool dcap;  // the split axis is at the depth limit: every colliding box is terminal
};

struct Acc {
    uint64_t ft, fu, fv;  // smallest colliding key
    uint32_t fflags;      // bit0: have, bit1: terminal, bit2: small (width or inside)
    uint64_t mt, mu, mv;  // largest colliding key
    uint32_t mhave;
    uint64_t tm;          // smallest it among terminal colliding boxes
    uint32_t thave;
};

struct Outcome {
    bool finish;
    double toi, tw;
    uint64_t n;
    uint8_t st;
};

__device__ __forceinline__ void load_query(const BatchArgs& a, int64_t q, Query& Q, bool& valid) {
#pragma unroll
    for (int r = 0; r < 24; ++r) Q.X[r] = a.pos[(int64_t)r * a.n + q];
    Q.kind = a.kind ? (int)a.kind[q] : (int)a.default_kind;
    Q.delta = a.delta_q ? a.delta_q[q] : a.delta;
    Q.max_iter = a.max_iter_q ? a.max_iter_q[q] : a.max_iter;
    Q.min_sep = a.min_sep_q ? a.min_sep_q[q] : a.min_sep;
    Q.literal = (a.flags & kFlagLiteral) != 0;
    double gmin;
    filter_eps(Q.kind, Q.X, Q.min_sep, Q.eps, &gmin);
    valid = (Q.kind == kVF || Q.kind == kEE) && query_valid(Q.X, Q.delta, Q.max_iter, Q.min_sep, gmin);
}

__device__ __forceinline__ LevelInfo level_info(const double kappa[3], const int32_t d[3]) {
    LevelInfo L;
    L.wt = pow2neg(d[0]);
    L.wu = pow2neg(d[1]);
    L.wv = pow2neg(d[2]);
    L.axis = split_axis(kappa, L.wt, L.wu, L.wv);
    L.dcap = d[L.axis] >= kMaxDepth;
    return L;
}

__device__ __forceinline__ void acc_init(Acc& A) {
    A.ft = A.fu = A.fv = ~0ull;
    A.fflags = 0;
    A.mt = A.mu = A.mv = 0;
    A.mhave = 0;
    A.tm = ~0ull;
    A.thave = 0;
}

__device__ __forceinline__ void acc_add(Acc& A, uint64_t bt, uint64_t bu, uint64_t bv, bool term,
                                        bool small) {
    if (!(A.fflags & 1u) || key_less(bt, bu, bv, A.ft, A.fu, A.fv)) {
        A.ft = bt; A.fu = bu; A.fv = bv;
        A.fflags = 1u | (term ? 2u : 0u) | (small ? 4u : 0u);
    }
    if (!A.mhave || key_less(A.mt, A.mu, A.mv, bt, bu, bv)) {
        A.mt = bt; A.mu = bu; A.mv = bv;
        A.mhave = 1;
    }
    if (term && (!A.thave || bt < A.tm)) {
        A.tm = bt;
        A.thave = 1;
    }
}

// Merge of two partial accumulators of the same level (commutative).
__device__ __forceinline__ void acc_merge(Acc& A, const Acc& B) {
    if ((B.fflags & 1u) && (!(A.fflags & 1u) || key_less(B.ft, B.fu, B.fv, A.ft, A.fu, A.fv))) {
        A.ft = B.ft; A.fu = B.fu; A.fv = B.fv; A.fflags = B.fflags;
    }
    if (B.mhave && (!A.mhave || key_less(A.mt, A.mu, A.mv, B.mt, B.mu, B.mv))) {
        A.mt = B.mt; A.mu = B.mu; A.mv = B.mv; A.mhave = 1;
    }
    if (B.thave && (!A.thave || B.tm < A.tm)) {
        A.tm = B.tm;
        A.thave = 1;
    }
}

__device__ __forceinline__ bool need_rank(const Acc& A, const State& S, const Query& Q,
                                          const LevelInfo& L) {
    if (!(A.fflags & 1u)) return false;
    const double tf = (double)A.ft * L.wt;
    const bool carry_ret = !Q.literal && S.tpend <= tf;
    const bool cap_possible = S.N + S.cnt >= (uint64_t)Q.max_iter;
    return carry_ret || cap_possible || (A.fflags & 2u);
}

// The level's decision (Alg. 2 replayed over one level).  rf / rm: number of
// keys on the level below the smallest / largest colliding key (only read when
// need_rank() said so).
__device__ __forceinline__ Outcome decide(const Acc& A, const State& S, const Query& Q,
                                          const LevelInfo& L, uint64_t rf, uint64_t rm) {
    Outcome O;
    O.finish = true;
    const uint64_t mI = (uint64_t)Q.max_iter;
    if (!(A.fflags & 1u)) {
        // nothing collides: the queue empties after this level
        const uint64_t n = S.N + S.cnt;
        O.n = n < mI ? n : mI;
        if (!Q.literal && S.tpend < INFINITY) {
            O.toi = S.tpend; O.tw = S.wpend; O.st = kStCarry;
        } else {
            O.toi = INFINITY; O.tw = 0.0; O.st = 0;
        }
        return O;
    }
    const double tf = (double)A.ft * L.wt;
    const bool cap_possible = S.N + S.cnt >= mI;
    const uint64_t nf = S.N + rf + 1;
    if (!Q.literal && S.tpend <= tf) {
        O.toi = S.tpend; O.tw = S.wpend; O.n = nf < mI ? nf : mI; O.st = kStCarry;
        return O;
    }
    if (cap_possible && nf >= mI) {
        O.toi = tf; O.tw = L.wt; O.n = mI; O.st = kStCap;
        return O;
    }
    if (A.fflags & 2u) {
        O.toi = tf; O.tw = L.wt; O.n = nf; O.st = (A.fflags & 4u) ? 0 : kStDepth;
        return O;
    }
    if (cap_possible && S.N + rm + 1 >= mI) {
        O.toi = tf; O.tw = L.wt; O.n = mI; O.st = kStCap;
        return O;
    }
    O.finish = false;
    return O;
}

// Moves S to the next level (after decide() returned finish = false).
__device__ __forceinline__ void advance(State& S, const Acc& A, const Query& Q, const LevelInfo& L,
                                        uint32_t next_cnt) {
    if (!Q.literal && A.thave) {
        const double tm = (double)A.tm * L.wt;
        if (tm < S.tpend) {
            S.tpend = tm;
            S.wpend = L.wt;
        }
    }
    S.N += S.cnt;
    S.level += 1;
    S.d[L.axis] += 1;
    S.cnt = next_cnt;
}

__device__ __forceinline__ void write_result(const BatchArgs& a, int64_t q, const Outcome& O) {
    a.toi[q] = O.toi;
    a.t_width[q] = O.tw;
    a.hit[q] = (O.toi <= 1.0) ? 1 : 0;
    a.n_checks[q] = O.n;
    a.status[q] = O.st;
}

__device__ __forceinline__ void write_invalid(const BatchArgs& a, int64_t q) {
    a.toi[q] = __longlong_as_double(0x7ff8000000000000ll);
    a.t_width[q] = __longlong_as_double(0x7ff8000000000000ll);
    a.hit[q] = 0;
    a.n_checks[q] = 0;
    a.status[q] = kStInvalid;
}

template <int KIND>
__device__ __forceinline__ CheckResult check_key(const Query& Q, const LevelInfo& L, uint64_t bt,
                                                 uint64_t bu, uint64_t bv, bool root,
                                                 double kappa_out[3]) {
    const double t0 = (double)bt * L.wt, t1 = (double)(bt + 1) * L.wt;
    const double u0 = (double)bu * L.wu, u1 = (double)(bu + 1) * L.wu;
    const double v0 = (double)bv * L.wv, v1 = (double)(bv + 1) * L.wv;
    return box_check<KIND>(Q.X, t0, t1, u0, u1, v0, v1, Q.eps, Q.min_sep, Q.delta, root,
                           kappa_out);
}

__device__ __forceinline__ CheckResult check_any(const Query& Q, const LevelInfo& L, uint64_t bt,
                                                 uint64_t bu, uint64_t bv, bool root,
                                                 double kappa_out[3]) {
    if (Q.kind == kEE) return check_key<kEE>(Q, L, bt, bu, bv, root, kappa_out);
    return check_key<kVF>(Q, L, bt, bu, bv, root, kappa_out);
}

// Children of a non-terminal colliding box on the split axis; c1 may be
// rejected by the prism test of vertex-face queries.
__device__ __forceinline__ void children(const Query& Q, const State& S, const LevelInfo& L,
                                         uint64_t bt, uint64_t bu, uint64_t bv, uint64_t c[2][3],
                                         bool ok[2]) {
    int d[3] = {S.d[0], S.d[1], S.d[2]};
    d[L.axis] += 1;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        c[b][0] = bt; c[b][1] = bu; c[b][2] = bv;
        c[b][L.axis] = 2 * c[b][L.axis] + (uint64_t)b;
        ok[b] = (Q.kind == kEE) || vf_admit(c[b][1], d[1], c[b][2], d[2]);
    }
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Query order grouped by kind (VF from the front, EE from the back), so that
// the lanes of a wavefront mostly run the same corner formula.

__global__ void k_partition(BatchArgs a, int64_t* order) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool act = q < a.n;
    const int kind = act ? (a.kind ? (int)a.kind[q] : (int)a.default_kind) : 0;
    const bool ee = act && kind == kEE;
    const bool vf = act && !ee;
    const uint64_t mv = __ballot(vf), me = __ballot(ee);
    const int lane = __lane_id();
    unsigned long long bv = 0, be = 0;
    if (lane == 0) {
        if (mv) bv = atomicAdd(&a.counters[kCntOrderFront], (unsigned long long)__popcll(mv));
        if (me) be = atomicAdd(&a.counters[kCntOrderBack], (unsigned long long)__popcll(me));
    }
    bv = __shfl(bv, 0);
    be = __shfl(be, 0);
    if (vf) order[bv + __popcll(mv & lanemask_lt())] = q;
    if (ee) order[a.n - 1 - (int64_t)(be + __popcll(me & lanemask_lt()))] = q;
}

// Resets the counters at the start of a batch (a kernel, so that it can sit
// in a captured graph).
__global__ void k_reset(unsigned long long* counters) {
    const int i = threadIdx.x;
    if (i < kCntEnd) counters[i] = 0;
}

// ---------------------------------------------------------------------------
// Lane engine.

__device__ __forceinline__ int64_t arena_idx(int K, int b, int i, int j) {
    return ((int64_t)((b * K + i) * 3 + j)) * 64;
}

template <bool PERSISTENT>
__global__ __launch_bounds__(256) void k_lane(BatchArgs a, LaneCfg c) {
    const int lane = threadIdx.x & 63;
    const int64_t gtid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t slot = gtid >> 6;
    const int K = c.capacity;
    uint64_t* ar = c.arena + slot * (int64_t)(2 * K * 3 * 64) + lane;

    int64_t q = -1;
    bool fresh = false;
    bool exhausted = false;
    if (!PERSISTENT) {
        if (gtid < a.n) {
            q = a.order ? a.order[gtid] : gtid;
            fresh = true;
        }
        exhausted = true;
    }

    Query Q;
    State S;
    Acc A;
    LevelInfo L;
    uint32_t idx = 0, next_cnt = 0;
    int cur = 0;
    uint64_t nchk[2] = {0, 0};

    while (true) {
        if (PERSISTENT && !exhausted) {
            const bool need = q < 0;
            const uint64_t m = __ballot(need);
            if (m) {
                const int leader = __builtin_ctzll(m);
                unsigned long long base = 0;
                if (lane == leader)
                    base = atomicAdd(&a.counters[kCntCursor], (unsigned long long)__popcll(m));
                base = __shfl(base, leader);
                if (need) {
                    const uint64_t r = base + __popcll(m & lanemask_lt());
                    if (r < (uint64_t)a.n) {
                        q = a.order ? a.order[r] : (int64_t)r;
                        fresh = true;
                    }
                }
                if (base + __popcll(m) >= (uint64_t)a.n) exhausted = true;
            }
        }
        if (__ballot(q >= 0) == 0) break;
        if (q >= 0 && fresh) {
            fresh = false;
            bool valid;
            load_query(a, q, Q, valid);
            if (!valid) {
                write_invalid(a, q);
                q = -1;
            } else {
                S.N = 0;
                S.tpend = INFINITY;
                S.wpend = 0.0;
                S.level = 0;
                S.d[0] = S.d[1] = S.d[2] = 0;
                S.cnt = 1;
                idx = 0;
                next_cnt = 0;
                cur = 0;
                acc_init(A);
                L.wt = L.wu = L.wv = 1.0;
                L.axis = 0;
                L.dcap = false;
            }
        }
        if (q < 0) continue;

        // ---- one box check
        const bool root = S.level == 0;
        uint64_t bt = 0, bu = 0, bv = 0;
        if (!root) {
            bt = ar[arena_idx(K, cur, idx, 0)];
            bu = ar[arena_idx(K, cur, idx, 1)];
            bv = ar[arena_idx(K, cur, idx, 2)];
        }
        const CheckResult R = check_any(Q, L, bt, bu, bv, root, Q.kappa);
        if (root) L = level_info(Q.kappa, S.d);
        nchk[Q.kind] += 1;
        if (R.collide) {
            const bool term = R.small || L.dcap;
            acc_add(A, bt, bu, bv, term, R.small);
            if (!term) {
                uint64_t ch[2][3];
                bool ok[2];
                children(Q, S, L, bt, bu, bv, ch, ok);
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    if (!ok[b]) continue;
                    if (next_cnt < (uint32_t)K) {
                        ar[arena_idx(K, cur ^ 1, next_cnt, 0)] = ch[b][0];
                        ar[arena_idx(K, cur ^ 1, next_cnt, 1)] = ch[b][1];
                        ar[arena_idx(K, cur ^ 1, next_cnt, 2)] = ch[b][2];
                    }
                    next_cnt += 1;
                }
            }
        }
        idx += 1;
        if (idx < S.cnt) continue;

        // ---- end of the level: replay Alg. 2's decisions
        uint64_t rf = 0, rm = 0;
        if (!root && need_rank(A, S, Q, L)) {
            for (uint32_t i = 0; i < S.cnt; ++i) {
                const uint64_t kt = ar[arena_idx(K, cur, i, 0)];
                const uint64_t ku = ar[arena_idx(K, cur, i, 1)];
                const uint64_t kv = ar[arena_idx(K, cur, i, 2)];
                rf += key_less(kt, ku, kv, A.ft, A.fu, A.fv) ? 1 : 0;
                rm += key_less(kt, ku, kv, A.mt, A.mu, A.mv) ? 1 : 0;
            }
        }
        const Outcome O = decide(A, S, Q, L, rf, rm);
        if (O.finish) {
            write_result(a, q, O);
            q = -1;
            continue;
        }
        // hand the query on at the start of a level when the next level does not
        // fit the lane, or (persistent) when the query has used its budget
        const bool overflow = next_cnt > (uint32_t)K;
        bool promote = overflow;
        if (!overflow) {
            advance(S, A, Q, L, next_cnt);
            cur ^= 1;
            idx = 0;
            next_cnt = 0;
            acc_init(A);
            L = level_info(Q.kappa, S.d);
            promote = PERSISTENT && S.N + S.cnt > c.budget;
        }
        if (promote) {
            // overflow: re-run this level (still in buffer cur) in the group
            // engine; budget: the next level (now in buffer cur) continues there
            const unsigned long long r = atomicAdd(&a.counters[kCntRecA], 1ull);
            if ((int64_t)r < c.record_cap) {
                uint64_t* rec = c.records + (int64_t)r * c.record_words;
                Record h;
                h.q = q; h.N = S.N; h.tpend = S.tpend; h.wpend = S.wpend; h.level = S.level;
                h.d[0] = S.d[0]; h.d[1] = S.d[1]; h.d[2] = S.d[2]; h.cnt = S.cnt; h.pad = 0;
                *reinterpret_cast<Record*>(rec) = h;
                uint64_t* boxes = rec + kRecordHeaderWords;
                for (uint32_t i = 0; i < S.cnt; ++i) {
                    const bool lvl0 = S.level == 0;
                    boxes[i] = lvl0 ? 0 : ar[arena_idx(K, cur, i, 0)];
                    boxes[K + i] = lvl0 ? 0 : ar[arena_idx(K, cur, i, 1)];
                    boxes[2 * K + i] = lvl0 ? 0 : ar[arena_idx(K, cur, i, 2)];
                }
                q = -1;
            } else if (overflow) {
                // no record left for a level that does not fit: a capacity the
                // host guaranteed (one record per query) was exceeded
                atomicAdd(&a.counters[kCntError], 1ull);
                q = -1;
            }
            // else: budget hand-off without a free record; keep solving here
        }
    }
    // per-wave check counters
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        unsigned long long v = nchk[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0 && v) atomicAdd(&a.counters[kCntChecks + k], v);
    }
}

// ---------------------------------------------------------------------------
// Group engine: W wavefronts share one query.

__device__ __forceinline__ void shfl_acc(Acc& B, const Acc& A, int off) {
    B.ft = __shfl_xor(A.ft, off);
    B.fu = __shfl_xor(A.fu, off);
    B.fv = __shfl_xor(A.fv, off);
    B.fflags = __shfl_xor(A.fflags, off);
    B.mt = __shfl_xor(A.mt, off);
    B.mu = __shfl_xor(A.mu, off);
    B.mv = __shfl_xor(A.mv, off);
    B.mhave = __shfl_xor(A.mhave, off);
    B.tm = __shfl_xor(A.tm, off);
    B.thave = __shfl_xor(A.thave, off);
}

__device__ __forceinline__ void wave_reduce_acc(Acc& A) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Acc B;
        shfl_acc(B, A, off);
        acc_merge(A, B);
    }
}

template <int W>
struct GroupShared {
    Acc acc[W];
    unsigned long long sum[W][2];
    unsigned long long next_cnt;
    int64_t rec;
};

template <int W>
__global__ __launch_bounds__(64 * W) void k_group(BatchArgs a, GroupCfg g) {
    constexpr int T = 64 * W;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    __shared__ GroupShared<W> sh;
    const int64_t cap = g.capacity;
    uint64_t* base = g.arena + (int64_t)blockIdx.x * (6 * cap);
    int64_t in_count = (int64_t)__atomic_load_n(&a.counters[g.in_count_idx], __ATOMIC_RELAXED);
    if (in_count > g.in_record_cap) in_count = g.in_record_cap;
    const int64_t in_k = (g.in_record_words - kRecordHeaderWords) / 3;
    uint64_t nchk[2] = {0, 0};

    while (true) {
        if (tid == 0) sh.rec = (int64_t)atomicAdd(&a.counters[g.in_take_idx], 1ull);
        __syncthreads();
        const int64_t r = sh.rec;
        __syncthreads();
        if (r >= in_count) break;
        const uint64_t* rec = g.in_records + r * g.in_record_words;
        const Record h = *reinterpret_cast<const Record*>(rec);
        Query Q;
        bool valid;
        load_query(a, h.q, Q, valid);
        {
            LevelInfo L0;
            L0.wt = L0.wu = L0.wv = 1.0;
            L0.axis = 0;
            L0.dcap = false;
            check_any(Q, L0, 0, 0, 0, true, Q.kappa);
        }
        State S;
        S.N = h.N; S.tpend = h.tpend; S.wpend = h.wpend; S.level = h.level;
        S.d[0] = h.d[0]; S.d[1] = h.d[1]; S.d[2] = h.d[2]; S.cnt = h.cnt;
        const uint64_t* rb = rec + kRecordHeaderWords;
        for (int64_t i = tid; i < (int64_t)S.cnt; i += T) {
            base[i] = rb[i];
            base[cap + i] = rb[in_k + i];
            base[2 * cap + i] = rb[2 * in_k + i];
        }
        __syncthreads();
        int cur = 0;
        while (true) {
            const LevelInfo L = level_info(Q.kappa, S.d);
            const uint64_t* ct = base + cur * 3 * cap;
            uint64_t* nt = base + (cur ^ 1) * 3 * cap;
            Acc A;
            acc_init(A);
            unsigned long long next_w = 0;  // W == 1: running count of the next level
            if (W > 1) {
                if (tid == 0) sh.next_cnt = 0;
                __syncthreads();
            }
            for (int64_t b0 = 0; b0 < (int64_t)S.cnt; b0 += T) {
                const int64_t i = b0 + tid;
                const bool act = i < (int64_t)S.cnt;
                bool e0 = false, e1 = false;
                uint64_t ch[2][3];
                if (act) {
                    const uint64_t bt = ct[i], bu = ct[cap + i], bv = ct[2 * cap + i];
                    double dummy[3];
                    const CheckResult R = check_any(Q, L, bt, bu, bv, false, dummy);
                    if (R.collide) {
                        const bool term = R.small || L.dcap;
                        acc_add(A, bt, bu, bv, term, R.small);
                        if (!term) {
                            bool ok[2];
                            children(Q, S, L, bt, bu, bv, ch, ok);
                            e0 = ok[0];
                            e1 = ok[1];
                        }
                    }
                }
                const uint64_t m0 = __ballot(e0), m1 = __ballot(e1);
                const unsigned long long tot = __popcll(m0) + __popcll(m1);
                unsigned long long wbase;
                if (W == 1) {
                    wbase = next_w;
                    next_w += tot;
                } else {
                    unsigned long long t = 0;
                    if (lane == 0 && tot) t = atomicAdd(&sh.next_cnt, tot);
                    wbase = __shfl(t, 0);
                }
                const uint64_t lt = lanemask_lt();
                const int64_t p = (int64_t)wbase + __popcll(m0 & lt) + __popcll(m1 & lt);
                if (e0 && p < cap) {
                    nt[p] = ch[0][0]; nt[cap + p] = ch[0][1]; nt[2 * cap + p] = ch[0][2];
                }
                const int64_t p1 = p + (e0 ? 1 : 0);
                if (e1 && p1 < cap) {
                    nt[p1] = ch[1][0]; nt[cap + p1] = ch[1][1]; nt[2 * cap + p1] = ch[1][2];
                }
            }
            const uint64_t cnt_here = S.cnt;
            wave_reduce_acc(A);
            uint64_t next_cnt;
            if (W > 1) {
                if (lane == 0) sh.acc[wid] = A;
                __syncthreads();
                A = sh.acc[0];
                for (int w = 1; w < W; ++w) acc_merge(A, sh.acc[w]);
                next_cnt = sh.next_cnt;
                __syncthreads();
            } else {
                next_cnt = next_w;
            }
            uint64_t rf = 0, rm = 0;
            if (need_rank(A, S, Q, L)) {
                unsigned long long sf = 0, sm = 0;
                for (int64_t i = tid; i < (int64_t)S.cnt; i += T) {
                    const uint64_t kt = ct[i], ku = ct[cap + i], kv = ct[2 * cap + i];
                    sf += key_less(kt, ku, kv, A.ft, A.fu, A.fv) ? 1 : 0;
                    sm += key_less(kt, ku, kv, A.mt, A.mu, A.mv) ? 1 : 0;
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    sf += __shfl_xor(sf, off);
                    sm += __shfl_xor(sm, off);
                }
                if (W > 1) {
                    if (lane == 0) { sh.sum[wid][0] = sf; sh.sum[wid][1] = sm; }
                    __syncthreads();
                    sf = 0; sm = 0;
                    for (int w = 0; w < W; ++w) { sf += sh.sum[w][0]; sm += sh.sum[w][1]; }
                    __syncthreads();
                }
                rf = sf;
                rm = sm;
            }
            if (tid == 0) nchk[Q.kind] += cnt_here;
            const Outcome O = decide(A, S, Q, L, rf, rm);
            if (O.finish) {
                if (tid == 0) write_result(a, h.q, O);
                break;
            }
            if (next_cnt > (uint64_t)cap) {
                // the next level does not fit: restart the query in the next engine
                if (tid == 0) {
                    if (g.out_records) {
                        const unsigned long long o = atomicAdd(&a.counters[g.out_count_idx], 1ull);
                        if ((int64_t)o < g.out_record_cap) {
                            uint64_t* orec = g.out_records + (int64_t)o * g.out_record_words;
                            Record nh;
                            nh.q = h.q; nh.N = 0; nh.tpend = INFINITY; nh.wpend = 0.0; nh.level = 0;
                            nh.d[0] = nh.d[1] = nh.d[2] = 0; nh.cnt = 1; nh.pad = 0;
                            *reinterpret_cast<Record*>(orec) = nh;
                            const int64_t ok = (g.out_record_words - kRecordHeaderWords) / 3;
                            orec[kRecordHeaderWords] = 0;
                            orec[kRecordHeaderWords + ok] = 0;
                            orec[kRecordHeaderWords + 2 * ok] = 0;
                        } else {
                            atomicAdd(&a.counters[kCntError], 1ull);
                        }
                    } else {
                        atomicAdd(&a.counters[kCntError], 1ull);
                    }
                }
                break;
            }
            advance(S, A, Q, L, (uint32_t)next_cnt);
            cur ^= 1;
            __syncthreads();
        }
        __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (nchk[k]) atomicAdd(&a.counters[kCntChecks + 2 * g.tier + k], (unsigned long long)nchk[k]);
    }
}

// Explicit instantiations used by the runtime.
template __global__ void k_lane<false>(BatchArgs, LaneCfg);
template __global__ void k_lane<true>(BatchArgs, LaneCfg);
template __global__ void k_group<1>(BatchArgs, GroupCfg);
template __global__ void k_group<2>(BatchArgs, GroupCfg);
template __global__ void k_group<4>(BatchArgs, GroupCfg);
template __global__ void k_group<8>(BatchArgs, GroupCfg);

}  // namespace ccd
