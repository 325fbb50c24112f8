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
    double tmax;      // time interval [0, tmax]
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
    double wt, wu, wv;                  // box widths; wt in s = t / tmax
    double tmax;                        // time values are tmax * s
    int64_t bt_bits, bu_bits, bv_bits;  // bit patterns of 2^(52-d) per axis (see dyadic())
    double bt_val, bu_val, bv_val;      // 2^(52-d) per axis
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
    int64_t fpos;         // group engine: where child 0 of the smallest key went, or -1
};

struct Outcome {
    bool finish;
    double toi, tw;
    uint64_t n;
    uint8_t st;
};

// Where the global query index v of a launch lives: a plain batch, or one of
// the requests of a serving launch (binary search of the request table).
struct QView {
    const double* pos;
    int64_t n;  // queries of its batch / request
    int64_t q;  // index within it
    const uint8_t* kind;
    uint32_t default_kind;
    const double* delta_q;
    const int64_t* max_iter_q;
    const double* min_sep_q;
    double delta;
    int64_t max_iter;
    double min_sep;
    double t_max;
    uint32_t flags;
    double* toi;
    double* t_width;
    uint8_t* hit;
    uint64_t* n_checks;
    uint8_t* status;
};

__device__ __forceinline__ QView view(const BatchArgs& a, int64_t v) {
    QView w;
    if (!a.reqs) {
        w.pos = a.pos; w.n = a.n; w.q = v; w.kind = a.kind; w.default_kind = a.default_kind;
        w.delta_q = a.delta_q; w.max_iter_q = a.max_iter_q; w.min_sep_q = a.min_sep_q;
        w.delta = a.delta; w.max_iter = a.max_iter; w.min_sep = a.min_sep; w.t_max = a.t_max;
        w.flags = a.flags;
        w.toi = a.toi; w.t_width = a.t_width; w.hit = a.hit; w.n_checks = a.n_checks;
        w.status = a.status;
        return w;
    }
    int64_t lo = 0, hi = a.nreq - 1;  // last entry with base <= v
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (a.reqs[mid].base <= v) lo = mid;
        else hi = mid - 1;
    }
    const ReqEntry& r = a.reqs[lo];
    w.pos = r.pos; w.n = r.n; w.q = v - r.base; w.kind = r.kind; w.default_kind = r.default_kind;
    w.delta_q = nullptr; w.max_iter_q = nullptr; w.min_sep_q = nullptr;
    w.delta = r.delta; w.max_iter = r.max_iter; w.min_sep = r.min_sep; w.t_max = r.t_max;
    w.flags = r.flags;
    w.toi = r.toi; w.t_width = r.t_width; w.hit = r.hit; w.n_checks = r.n_checks;
    w.status = r.status;
    return w;
}

__device__ __forceinline__ int query_kind(const BatchArgs& a, int64_t v) {
    if (!a.reqs) return a.kind ? (int)a.kind[v] : (int)a.default_kind;
    const QView w = view(a, v);
    return w.kind ? (int)w.kind[w.q] : (int)w.default_kind;
}

__device__ __forceinline__ void load_query(const BatchArgs& a, int64_t v, Query& Q, bool& valid) {
    const QView w = view(a, v);
    const int64_t q = w.q;
#pragma unroll
    for (int r = 0; r < 24; ++r) Q.X[r] = w.pos[(int64_t)r * w.n + q];
    Q.kind = w.kind ? (int)w.kind[q] : (int)w.default_kind;
    Q.delta = w.delta_q ? w.delta_q[q] : w.delta;
    Q.max_iter = w.max_iter_q ? w.max_iter_q[q] : w.max_iter;
    Q.min_sep = w.min_sep_q ? w.min_sep_q[q] : w.min_sep;
    Q.literal = (w.flags & kFlagLiteral) != 0;
    Q.tmax = w.t_max;
    double gmin;
    bool gok = true;
    if (a.gamma) gok = filter_eps_scene(Q.kind, Q.X, Q.min_sep, a.gamma, Q.eps, &gmin);
    else filter_eps(Q.kind, Q.X, Q.min_sep, Q.eps, &gmin);
    valid = gok && (Q.kind == kVF || Q.kind == kEE) &&
            query_valid(Q.X, Q.delta, Q.max_iter, Q.min_sep, gmin);
}

// The split rule compares w(I_t) kappa_t with w(I_t) = tmax * 2^-dt (exact).
__device__ __forceinline__ LevelInfo level_info(const double kappa[3], const int32_t d[3],
                                                double tmax) {
    LevelInfo L;
    L.tmax = tmax;
    L.wt = pow2neg(d[0]);
    L.wu = pow2neg(d[1]);
    L.wv = pow2neg(d[2]);
    L.bt_bits = (int64_t)(1023 + 52 - d[0]) << 52;
    L.bu_bits = (int64_t)(1023 + 52 - d[1]) << 52;
    L.bv_bits = (int64_t)(1023 + 52 - d[2]) << 52;
    L.bt_val = __longlong_as_double(L.bt_bits);
    L.bu_val = __longlong_as_double(L.bu_bits);
    L.bv_val = __longlong_as_double(L.bv_bits);
    L.axis = split_axis(kappa, tmax * L.wt, L.wu, L.wv);
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
    A.fpos = -1;
}

// track_max: the largest colliding key is only needed on a level where the
// m_I stop can fire (N + |level| >= m_I), a level-uniform condition.
__device__ __forceinline__ void acc_add(Acc& A, uint64_t bt, uint64_t bu, uint64_t bv, bool term,
                                        bool small, bool track_max = true, int64_t pos0 = -1) {
    if (!(A.fflags & 1u) || key_less(bt, bu, bv, A.ft, A.fu, A.fv)) {
        A.ft = bt; A.fu = bu; A.fv = bv;
        A.fflags = 1u | (term ? 2u : 0u) | (small ? 4u : 0u);
        A.fpos = pos0;
    }
    if (track_max && (!A.mhave || key_less(A.mt, A.mu, A.mv, bt, bu, bv))) {
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
        A.ft = B.ft; A.fu = B.fu; A.fv = B.fv; A.fflags = B.fflags; A.fpos = B.fpos;
    }
    if (B.mhave && (!A.mhave || key_less(A.mt, A.mu, A.mv, B.mt, B.mu, B.mv))) {
        A.mt = B.mt; A.mu = B.mu; A.mv = B.mv; A.mhave = 1;
    }
    if (B.thave && (!A.thave || B.tm < A.tm)) {
        A.tm = B.tm;
        A.thave = 1;
    }
}

__device__ __forceinline__ bool need_rank(const Acc& A, const State& S, bool literal,
                                          int64_t max_iter, const LevelInfo& L) {
    if (!(A.fflags & 1u)) return false;
    const double tf = L.tmax * ((double)A.ft * L.wt);
    const bool carry_ret = !literal && S.tpend <= tf;
    const bool cap_possible = S.N + S.cnt >= (uint64_t)max_iter;
    return carry_ret || cap_possible || (A.fflags & 2u);
}

// The outcomes of a level that depend only on its first colliding box f (A
// holds f as (t, u, v) indices) and rf, the number of the level's keys below
// f: the carried box comes first, m_I is reached at f, or f is terminal.
__device__ __forceinline__ Outcome decide_first(const Acc& A, const State& S, bool literal,
                                                int64_t max_iter, const LevelInfo& L, uint64_t rf) {
    Outcome O;
    O.finish = true;
    const uint64_t mI = (uint64_t)max_iter;
    const double tf = L.tmax * ((double)A.ft * L.wt);
    const bool cap_possible = S.N + S.cnt >= mI;
    const uint64_t nf = S.N + rf + 1;
    if (!literal && S.tpend <= tf) {
        O.toi = S.tpend; O.tw = S.wpend; O.n = nf < mI ? nf : mI; O.st = kStCarry;
        return O;
    }
    if (cap_possible && nf >= mI) {
        O.toi = tf; O.tw = L.tmax * L.wt; O.n = mI; O.st = kStCap;
        return O;
    }
    if (A.fflags & 2u) {
        O.toi = tf; O.tw = L.tmax * L.wt; O.n = nf; O.st = (A.fflags & 4u) ? 0 : kStDepth;
        return O;
    }
    O.finish = false;
    return O;
}

// The level's decision (Alg. 2 replayed over one level).  rf / rm: number of
// keys on the level below the smallest / largest colliding key (only read when
// need_rank() said so).
__device__ __forceinline__ Outcome decide(const Acc& A, const State& S, bool literal,
                                          int64_t max_iter, const LevelInfo& L, uint64_t rf,
                                          uint64_t rm) {
    Outcome O;
    O.finish = true;
    const uint64_t mI = (uint64_t)max_iter;
    if (!(A.fflags & 1u)) {
        // nothing collides: the queue empties after this level
        const uint64_t n = S.N + S.cnt;
        O.n = n < mI ? n : mI;
        if (!literal && S.tpend < INFINITY) {
            O.toi = S.tpend; O.tw = S.wpend; O.st = kStCarry;
        } else {
            O.toi = INFINITY; O.tw = 0.0; O.st = 0;
        }
        return O;
    }
    O = decide_first(A, S, literal, max_iter, L, rf);
    if (O.finish) return O;
    const double tf = L.tmax * ((double)A.ft * L.wt);
    const bool cap_possible = S.N + S.cnt >= mI;
    O.finish = true;
    if (cap_possible && S.N + rm + 1 >= mI) {
        O.toi = tf; O.tw = L.tmax * L.wt; O.n = mI; O.st = kStCap;
        return O;
    }
    O.finish = false;
    return O;
}

// Moves S to the next level (after decide() returned finish = false).
__device__ __forceinline__ void advance(State& S, const Acc& A, bool literal, const LevelInfo& L,
                                        uint32_t next_cnt) {
    if (!literal && A.thave) {
        const double tm = L.tmax * ((double)A.tm * L.wt);
        if (tm < S.tpend) {
            S.tpend = tm;
            S.wpend = L.tmax * L.wt;
        }
    }
    S.N += S.cnt;
    S.level += 1;
    S.d[L.axis] += 1;
    S.cnt = next_cnt;
}

__device__ __forceinline__ void write_result(const BatchArgs& a, int64_t v, const Outcome& O) {
    const QView w = view(a, v);
    const int64_t q = w.q;
    w.toi[q] = O.toi;
    w.t_width[q] = O.tw;
    w.hit[q] = (O.toi <= 1.0) ? 1 : 0;
    w.n_checks[q] = O.n;
    w.status[q] = O.st;
}

__device__ __forceinline__ void write_invalid(const BatchArgs& a, int64_t v) {
    const QView w = view(a, v);
    const int64_t q = w.q;
    w.toi[q] = __longlong_as_double(0x7ff8000000000000ll);
    w.t_width[q] = __longlong_as_double(0x7ff8000000000000ll);
    w.hit[q] = 0;
    w.n_checks[q] = 0;
    w.status[q] = kStInvalid;
}

template <int KIND>
__device__ __forceinline__ CheckResult check_key(const Query& Q, const LevelInfo& L, uint64_t bt,
                                                 uint64_t bu, uint64_t bv, bool root,
                                                 double kappa_out[3]) {
    const double s0 = dyadic(bt, L.bt_bits, L.bt_val);
    const double u0 = dyadic(bu, L.bu_bits, L.bu_val);
    const double v0 = dyadic(bv, L.bv_bits, L.bv_val);
    return box_check<KIND>(Q.X, L.tmax * s0, L.tmax * (s0 + L.wt), u0, u0 + L.wu, v0, v0 + L.wv,
                           Q.eps, Q.min_sep,
                           Q.delta, root, kappa_out);
}

__device__ __forceinline__ CheckResult check_any(const Query& Q, const LevelInfo& L, uint64_t bt,
                                                 uint64_t bu, uint64_t bv, bool root,
                                                 double kappa_out[3]) {
    if (Q.kind == kEE) return check_key<kEE>(Q, L, bt, bu, bv, root, kappa_out);
    return check_key<kVF>(Q, L, bt, bu, bv, root, kappa_out);
}

// ---------------------------------------------------------------------------
// Group-engine box check: the query's coordinates sit in LDS as Xs[c*8 + k]
// (one query per block), axes are evaluated one after the other and the
// remaining axes are skipped once no active lane of the wavefront still
// collides (Sec. 5.2, efficient evaluation: per-axis early exit).  The
// values are the same as box_check()'s.
template <int KIND>
__device__ __forceinline__ CheckResult check_box_lds(const double* Xs, const double* Es,
                                                     double t0, double t1, double u0, double u1,
                                                     double v0, double v1, double min_sep,
                                                     double delta) {
    bool col = true, ins = true;
    double width = 0.0;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        if (__ballot(col) == 0) break;
        double xc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) xc[k] = Xs[c * 8 + k];
        double f[8];
        corner_values_axis<KIND>(xc, t0, t1, u0, u1, v0, v1, f);
        double m = f[0], M = f[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) {
            m = fmin(m, f[i]);
            M = fmax(M, f[i]);
        }
        const double e = Es[c];
        const double lo = m - min_sep;
        const double hi = M + min_sep;
        col = col && (lo <= e) && (hi >= -e);
        ins = ins && (lo >= -e) && (hi <= e);
        width = fmax(width, M - m);
    }
    CheckResult r;
    r.collide = col;
    r.small = (width < delta) || ins;
    return r;
}

// eq. kappas from the level-0 corners, with the coordinates in LDS.
template <int KIND>
__device__ __forceinline__ void kappa_lds(const double* Xs, double kappa[3]) {
    double kt = 0.0, ku = 0.0, kv = 0.0;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        double xc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) xc[k] = Xs[c * 8 + k];
        double f[8];
        corner_values_axis<KIND>(xc, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0, f);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int jt = j;
            const int ju = ((j >> 1) << 2) | (j & 1);
            const int jv = ((j >> 1) << 2) | ((j & 1) << 1);
            kt = fmax(kt, fabs(f[jt] - f[4 | jt]));
            ku = fmax(ku, fabs(f[ju] - f[2 | ju]));
            kv = fmax(kv, fabs(f[jv] - f[1 | jv]));
        }
    }
    kappa[0] = 3.0 * kt;
    kappa[1] = 3.0 * ku;
    kappa[2] = 3.0 * kv;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Set bits of two wavefront masks in the lanes below this one (mbcnt).
__device__ __forceinline__ int below_lane(uint64_t m0, uint64_t m1) {
    unsigned int c = __builtin_amdgcn_mbcnt_lo((unsigned int)m0, 0u);
    c = __builtin_amdgcn_mbcnt_hi((unsigned int)(m0 >> 32), c);
    c = __builtin_amdgcn_mbcnt_lo((unsigned int)m1, c);
    c = __builtin_amdgcn_mbcnt_hi((unsigned int)(m1 >> 32), c);
    return (int)c;
}

// Values that are equal in every lane (LDS broadcasts, butterfly reductions)
// made provably wave-uniform, so that they live in scalar registers and the
// branches on them are scalar branches.
__device__ __forceinline__ uint32_t uni32(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return (uint64_t)uni32((uint32_t)x) | ((uint64_t)uni32((uint32_t)(x >> 32)) << 32);
}
__device__ __forceinline__ int64_t uni64s(int64_t x) { return (int64_t)uni64((uint64_t)x); }
__device__ __forceinline__ double unif64(double x) {
    return __longlong_as_double((long long)uni64((uint64_t)__double_as_longlong(x)));
}
__device__ __forceinline__ void acc_uniform(Acc& A) {
    A.ft = uni64(A.ft); A.fu = uni64(A.fu); A.fv = uni64(A.fv); A.fflags = uni32(A.fflags);
    A.mt = uni64(A.mt); A.mu = uni64(A.mu); A.mv = uni64(A.mv); A.mhave = uni32(A.mhave);
    A.tm = uni64(A.tm); A.thave = uni32(A.thave);
    A.fpos = uni64s(A.fpos);
}

// ---------------------------------------------------------------------------
// Level 0 of every query, one thread per query (Alg. 2's first pop: the box
// [0,1]^3).  Invalid queries get their invalid result.  A query whose root box
// does not collide is finished after one check; so is one whose root box is
// terminal or whose m_I is 1 (n = 1, toi = 0).  The others are listed in
// `order` for the lane engine, vertex-face ones from the front and edge-edge
// ones from the back (counts in kCntOrderFront / kCntOrderBack), so that its
// wavefronts mostly run one corner formula; the lane engine checks their root
// box again (it needs the level-0 corners for kappa) and counts that check.
__global__ __launch_bounds__(512) void k_root(BatchArgs a, int64_t* order) {
    __shared__ unsigned int cnt[2];
    __shared__ unsigned long long base[2];
    __shared__ unsigned int fin[2];
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int lane = __lane_id();
    if (threadIdx.x < 2) { cnt[threadIdx.x] = 0; fin[threadIdx.x] = 0; }
    __syncthreads();
    bool keep = false, done = false;
    int kind = 0;
    if (q < a.n) {
        Query Q;
        bool valid;
        load_query(a, q, Q, valid);
        kind = Q.kind;
        if (!valid) {
            write_invalid(a, q);
        } else {
            double kap[3];
            // the root box [0, tmax] x [0,1]^2 (time values tmax * 0 and tmax * 1)
            const double t1 = Q.tmax * 1.0;
            const CheckResult R = Q.kind == kEE
                ? box_check<kEE>(Q.X, 0.0, t1, 0.0, 1.0, 0.0, 1.0, Q.eps, Q.min_sep, Q.delta, false, kap)
                : box_check<kVF>(Q.X, 0.0, t1, 0.0, 1.0, 0.0, 1.0, Q.eps, Q.min_sep, Q.delta, false, kap);
            // Alg. 2's decision on a one-box level 0
            State S;
            S.N = 0; S.tpend = INFINITY; S.wpend = 0.0; S.level = 0;
            S.d[0] = S.d[1] = S.d[2] = 0; S.cnt = 1;
            LevelInfo L;
            L.wt = L.wu = L.wv = 1.0;
            L.tmax = Q.tmax;
            Acc A;
            acc_init(A);
            if (R.collide) acc_add(A, 0, 0, 0, R.small, R.small);
            const Outcome O = decide(A, S, Q.literal, Q.max_iter, L, 0, 0);
            if (O.finish) {
                write_result(a, q, O);
                done = true;
            } else {
                keep = true;
            }
        }
    }
    const bool ee = keep && kind == kEE;
    const bool vf = keep && !ee;
    const uint64_t mv = __ballot(vf), me = __ballot(ee);
    const uint64_t dv = __ballot(done && kind != kEE), de = __ballot(done && kind == kEE);
    unsigned int ov = 0, oe = 0;
    if (lane == 0) {
        if (mv) ov = atomicAdd(&cnt[0], (unsigned int)__popcll(mv));
        if (me) oe = atomicAdd(&cnt[1], (unsigned int)__popcll(me));
        if (dv) atomicAdd(&fin[0], (unsigned int)__popcll(dv));
        if (de) atomicAdd(&fin[1], (unsigned int)__popcll(de));
    }
    ov = __shfl(ov, 0);
    oe = __shfl(oe, 0);
    __syncthreads();
    if (threadIdx.x < 2) {
        if (cnt[threadIdx.x])
            base[threadIdx.x] = atomicAdd(&a.counters[threadIdx.x == 0 ? kCntOrderFront : kCntOrderBack],
                                          (unsigned long long)cnt[threadIdx.x]);
        // one check per query finished here; the survivors' root checks are
        // counted once, by the lane engine
        if (fin[threadIdx.x])
            atomicAdd(&a.counters[kCntChecks + threadIdx.x], (unsigned long long)fin[threadIdx.x]);
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    if (vf) order[base[0] + ov + __popcll(mv & lt)] = q;
    if (ee) order[a.n - 1 - (int64_t)(base[1] + oe + __popcll(me & lt))] = q;
}

// Candidate pairs given as vertex ids over shared vertex arrays (the active-set
// and line-search drivers of Sec. 7 work on a mesh): the 8 points of query q
// are gathered into the structure-of-arrays layout pos[(3k+c)*n + q].  An id
// outside [0, nv) gives the query NaN coordinates, which makes it invalid.
__global__ void k_gather(int64_t n, const double* v0, const double* v1, const int32_t* ids,
                         int64_t nv, double* pos) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int64_t id = ids[4 * q + k];
        const bool ok = id >= 0 && id < nv;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pos[(int64_t)(3 * k + c) * n + q] = ok ? v0[3 * id + c] : nan;
            pos[(int64_t)(3 * (k + 4) + c) * n + q] = ok ? v1[3 * id + c] : nan;
        }
    }
}

// Scene-wide gamma per axis: max(1, max over the vertices at t = 0 and t = 1 of
// |x^c|), non-finite coordinates skipped (their queries are invalid anyway).
// Non-negative doubles order like their bit patterns: integer atomic max.
__global__ void k_scene_gamma_init(unsigned long long* g) {
    if (threadIdx.x < 3) g[threadIdx.x] = (unsigned long long)__double_as_longlong(1.0);
}

__global__ __launch_bounds__(256) void k_scene_gamma(const double* v0, const double* v1,
                                                     int64_t nv, unsigned long long* g) {
    double m[3] = {1.0, 1.0, 1.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nv; i += stride) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double a = fabs(v0[3 * i + c]), b = fabs(v1[3 * i + c]);
            if (a <= 1.7976931348623157e308) m[c] = fmax(m[c], a);
            if (b <= 1.7976931348623157e308) m[c] = fmax(m[c], b);
        }
    }
    __shared__ double wm[4][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m[c] = fmax(m[c], __shfl_xor(m[c], off));
        if (__lane_id() == 0) wm[threadIdx.x >> 6][c] = m[c];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int c = threadIdx.x;
        const double r = fmax(fmax(wm[0][c], wm[1][c]), fmax(wm[2][c], wm[3][c]));
        atomicMax(&g[c], (unsigned long long)__double_as_longlong(r));
    }
}

// Smallest toi of a batch: the line search bounds its step by the earliest time
// of impact (alpha = min over the candidates, Sec. 7).  toi values are +0..1,
// +inf or NaN (invalid queries, skipped); the bit patterns of non-negative
// doubles order like their values, so an integer atomic min gives the result.
__global__ void k_min_toi_init(unsigned long long* out) {
    if (threadIdx.x == 0) *out = (unsigned long long)__double_as_longlong(INFINITY);
}

__global__ __launch_bounds__(256) void k_min_toi(const double* toi, int64_t n,
                                                 unsigned long long* out) {
    double m = INFINITY;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const double v = toi[i];
        if (v < m) m = v;  // false for NaN
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
    // one atomic per block
    __shared__ double wmin[4];
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) wmin[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
        if (m < INFINITY) atomicMin(out, (unsigned long long)__double_as_longlong(m));
    }
}

// Resets the counters at the start of a batch (a kernel, so that it can sit
// in a captured graph).
__global__ void k_reset(unsigned long long* counters) {
    const int i = threadIdx.x;
    if (i < kCntEnd) counters[i] = 0;
}

// Orders the group engine's input records by the level at which the lane
// engine handed their query on, lowest first: a query whose level outgrew the
// lane frontier early branches widely and tends to need far more checks (on
// the simulation-shaped workload the rank correlation of that level with the
// query's check count is -0.85), and a single-wave group that takes such a
// query last holds the launch open long after the other groups are done.
// Any order gives the same results.  One workgroup: a counting sort over the
// 64 possible levels (the lane engine writes each record's level to a byte
// array beside the records); perm receives record indices.
__global__ __launch_bounds__(1024) void k_order_records(const unsigned long long* counters,
                                                        const uint8_t* levels, int64_t cap,
                                                        int32_t count_idx, int64_t* perm) {
    __shared__ unsigned long long hist[64];
    const int tid = threadIdx.x;
    int64_t count = (int64_t)counters[count_idx];
    if (count > cap) count = cap;
    if (tid < 64) hist[tid] = 0;
    __syncthreads();
    for (int64_t i = tid; i < count; i += 1024) atomicAdd(&hist[levels[i] & 63], 1ull);
    __syncthreads();
    if (tid == 0) {
        unsigned long long run = 0;
        for (int l = 0; l < 64; ++l) {
            const unsigned long long c = hist[l];
            hist[l] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int64_t i = tid; i < count; i += 1024) perm[atomicAdd(&hist[levels[i] & 63], 1ull)] = i;
}

// ---------------------------------------------------------------------------
// Packed keys.  A level whose total bisection depth D = dt + du + dv is at
// most 64 stores each box as one u64 key
//   key = (it << (du + dv)) | (iu << dv) | iv,
// whose numeric order is the lexicographic (t, u, v) order of Alg. 2.  Every
// level bisects one axis once, so D is the level number.  Deeper levels store
// the three indices in three arrays (group engine only).

__device__ __forceinline__ uint64_t shl64(uint64_t x, int s) { return s >= 64 ? 0ull : x << s; }
__device__ __forceinline__ uint64_t shr64(uint64_t x, int s) { return s >= 64 ? 0ull : x >> s; }
__device__ __forceinline__ uint64_t mask64(int d) { return d >= 64 ? ~0ull : ((1ull << d) - 1ull); }

struct KeyCodec {
    int st, su;        // shifts of the t and u fields
    uint64_t mu, mv;   // masks of the u and v fields
    __device__ __forceinline__ void init(int du, int dv) {
        st = du + dv;
        su = dv;
        mu = mask64(du);
        mv = mask64(dv);
    }
    __device__ __forceinline__ uint64_t encode(uint64_t t, uint64_t u, uint64_t v) const {
        return shl64(t, st) | shl64(u, su) | v;
    }
    __device__ __forceinline__ void decode(uint64_t k, uint64_t& t, uint64_t& u, uint64_t& v) const {
        t = shr64(k, st);
        u = shr64(k, su) & mu;
        v = k & mv;
    }
};

// Child b of a packed key whose split axis field starts at bit sx: the field
// gains one low bit (0: lower half, 1: upper half), the fields above it move
// up one bit.  Needs a level number below 64 (the child has depth sum <= 64).
__device__ __forceinline__ uint64_t child_key(uint64_t key, int sx, uint64_t b) {
    return shl64(key >> sx, sx + 1) | (b << sx) | (key & mask64(sx));
}

// Result of a query whose next level does not fit the scratch it was given:
// Alg. 2's return at the current level's first colliding box f, as at the m_I
// stop (its t_lo is a lower bound of every root the level's boxes hold, so the
// value stays conservative), flagged with the overflow status.  Only called
// after decide() kept the query going, so f exists and the carried box (if
// any) is later than t_lo(f).
__device__ __forceinline__ void write_overflow(const BatchArgs& a, int64_t v, const Acc& A,
                                               const State& S, const LevelInfo& L,
                                               int64_t max_iter) {
    Outcome O;
    O.finish = true;
    O.toi = L.tmax * ((double)A.ft * L.wt);
    O.tw = L.tmax * L.wt;
    const uint64_t n = S.N + S.cnt;
    O.n = n < (uint64_t)max_iter ? n : (uint64_t)max_iter;
    O.st = kStOverflow;
    write_result(a, v, O);
    atomicAdd(&a.counters[kCntOverflow], 1ull);
}

// ---------------------------------------------------------------------------
// Lane engine.  One lane owns one query.  Its frontier lives in LDS: two
// buffers (the level being checked and the next one) of `capacity` packed keys
// per lane, laid out [buffer][box][thread of the block], so that the 64 lanes
// of a wavefront touch 64 consecutive words (no bank conflict) whichever box
// each of them is at.  A query is handed on (a key-format Record) when its
// next level has more than `capacity` boxes or would need keys wider than 64
// bits (level 64), or (persistent) once it has used its check budget.

template <bool PERSISTENT>
__global__ __launch_bounds__(kLaneBlock) void k_lane(BatchArgs a, LaneCfg c) {
    extern __shared__ uint64_t lane_frontier[];
    const int lane = threadIdx.x & 63;
    const int64_t gtid = blockIdx.x * (int64_t)kLaneBlock + threadIdx.x;
    const int K = c.capacity;
    uint64_t* fr = lane_frontier + threadIdx.x;
    auto slot = [&](int b, uint32_t i) -> uint64_t& {
        return fr[((int64_t)b * K + (int64_t)i) * kLaneBlock];
    };

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
    KeyCodec kc;
    uint32_t idx = 0, next_cnt = 0;
    int cur = 0;
    uint64_t nchk[2] = {0, 0};
    uint64_t iters = 0;
    // persistent: the queries are the root pass's survivors, vertex-face at
    // order[0, nf) and edge-edge at order[n - ne, n), taken as one range
    uint64_t total = (uint64_t)a.n, nf = 0, ne = 0;
    if (PERSISTENT && c.survivors) {
        nf = uni64(a.counters[kCntOrderFront]);
        ne = uni64(a.counters[kCntOrderBack]);
        total = nf + ne;
    }

    while (true) {
        // idle lanes take new queries together, once a quarter of the wave is
        // idle: the queries' scattered coordinate loads then cost the wave one
        // memory latency for many lanes instead of one per finished query
        if (PERSISTENT && !exhausted) {
            const bool need = q < 0;
            const uint64_t m = __ballot(need);
            if (__popcll(m) >= 16) {
                const int leader = __builtin_ctzll(m);
                unsigned long long base = 0;
                if (lane == leader)
                    base = atomicAdd(&a.counters[kCntCursor], (unsigned long long)__popcll(m));
                base = uni64(__shfl(base, leader));
                if (need) {
                    const uint64_t r = base + __popcll(m & lanemask_lt());
                    if (r < total) {
                        const uint64_t o = (c.survivors && r >= nf) ? (uint64_t)a.n - ne + (r - nf) : r;
                        q = a.order ? a.order[o] : (int64_t)o;
                        fresh = true;
                    }
                }
                if (base + __popcll(m) >= total) exhausted = true;
            }
        }
        if (__ballot(q >= 0) == 0) break;
        iters += 1;
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
                Q.kappa[0] = Q.kappa[1] = Q.kappa[2] = 0.0;  // set at the level-0 check
                L = level_info(Q.kappa, S.d, Q.tmax);
                kc.init(0, 0);
            }
        }
        if (q < 0) continue;

        // ---- one box check (lanes whose level still has boxes)
        if (idx < S.cnt) {
            const bool root = S.level == 0;
            const uint64_t key = root ? 0ull : slot(cur, idx);
            uint64_t bt, bu, bv;
            kc.decode(key, bt, bu, bv);
            // kappa (eq. kappas) comes from the corners of [0,1]^3: the level-0 check
            // produces it when the time interval is the full one
            const bool fused = root && Q.tmax == 1.0;
            if (root && !fused) {
                if (Q.kind == kEE)
                    (void)box_check<kEE>(Q.X, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0, Q.eps, Q.min_sep, Q.delta,
                                         true, Q.kappa);
                else
                    (void)box_check<kVF>(Q.X, 0.0, 1.0, 0.0, 1.0, 0.0, 1.0, Q.eps, Q.min_sep, Q.delta,
                                         true, Q.kappa);
            }
            const CheckResult R = check_any(Q, L, bt, bu, bv, fused, Q.kappa);
            if (root) L = level_info(Q.kappa, S.d, Q.tmax);
            nchk[Q.kind] += 1;
            if (R.collide) {
                const bool term = R.small || L.dcap;
                acc_add(A, bt, bu, bv, term, R.small);
                if (!term) {
                    // both children on the split axis; child 0 keeps the box's
                    // (u_lo, v_lo), which passed the vertex-face prism test when
                    // the box was made, so only child 1 is tested
                    const int ax = L.axis;
                    const int sx = ax == 0 ? kc.st : (ax == 1 ? kc.su : 0);
                    const bool ok1 = Q.kind == kEE ||
                                     vf_admit(ax == 1 ? 2 * bu + 1 : bu, S.d[1] + (ax == 1 ? 1 : 0),
                                              ax == 2 ? 2 * bv + 1 : bv, S.d[2] + (ax == 2 ? 1 : 0));
                    const bool fits = S.level < 64;
                    if (fits && next_cnt < (uint32_t)K) slot(cur ^ 1, next_cnt) = child_key(key, sx, 0);
                    next_cnt += 1;
                    if (ok1) {
                        if (fits && next_cnt < (uint32_t)K) slot(cur ^ 1, next_cnt) = child_key(key, sx, 1);
                        next_cnt += 1;
                    }
                }
            }
            idx += 1;
        }
        // ---- end of a level: a lane whose level is checked waits until a quarter
        // of the wave's busy lanes do, and they run the level-end code together
        // (the wave then executes it once for all of them instead of at nearly
        // every step); the decisions themselves are per query, so this changes
        // only when a lane spends its idle steps
        {
            const uint64_t m_end = __ballot(idx >= S.cnt);
            const uint64_t m_act = __ballot(true);
            if (__popcll(m_end) * 4 < __popcll(m_act) || idx < S.cnt) continue;
        }

        // ---- end of the level: replay Alg. 2's decisions
        uint64_t rf = 0, rm = 0;
        if (S.level != 0 && need_rank(A, S, Q.literal, Q.max_iter, L)) {
            const uint64_t fk = kc.encode(A.ft, A.fu, A.fv);
            const uint64_t mk = kc.encode(A.mt, A.mu, A.mv);
            for (uint32_t i = 0; i < S.cnt; ++i) {
                const uint64_t k = slot(cur, i);
                rf += k < fk ? 1 : 0;
                rm += k < mk ? 1 : 0;
            }
        }
        const Outcome O = decide(A, S, Q.literal, Q.max_iter, L, rf, rm);
        if (O.finish) {
            write_result(a, q, O);
            q = -1;
            continue;
        }
        // hand the query on at the start of a level when the next level does not
        // fit the lane (too many boxes, or keys of more than 64 bits), or
        // (persistent) when the query has used its budget
        const bool deep = S.level >= 64;
        const bool overflow = next_cnt > (uint32_t)K || deep;
        bool promote = overflow;
        if (!overflow) {
            advance(S, A, Q.literal, L, next_cnt);
            cur ^= 1;
            idx = 0;
            next_cnt = 0;
            acc_init(A);
            L = level_info(Q.kappa, S.d, Q.tmax);
            kc.init(S.d[1], S.d[2]);
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
                h.d[0] = S.d[0]; h.d[1] = S.d[1]; h.d[2] = S.d[2]; h.cnt = S.cnt;
                h.fmt = kFmtKey;
                h.words = S.level == 0 ? 0 : S.cnt;
                *reinterpret_cast<Record*>(rec) = h;
                c.record_levels[r] = (uint8_t)(S.level < 63 ? S.level : 63);
                uint64_t* boxes = rec + kRecordHeaderWords;
                if (S.level != 0)
                    for (uint32_t i = 0; i < S.cnt; ++i) boxes[i] = slot(cur, i);
                if (deep) atomicAdd(&a.counters[kCntDeep], 1ull);
                q = -1;
            } else if (overflow) {
                // no record left for a level that does not fit (the host provides
                // one record per query, so this does not happen): flagged return
                write_overflow(a, q, A, S, L, Q.max_iter);
                q = -1;
            }
            // else: budget hand-off without a free record; keep solving here
        }
    }
    // per-wave check and lane-slot counters
    if (lane == 0 && iters) atomicAdd(&a.counters[kCntSlots + 0], (unsigned long long)iters * 64ull);
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
    B.fpos = __shfl_xor(A.fpos, off);
}

__device__ __forceinline__ void wave_reduce_acc(Acc& A) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        Acc B;
        shfl_acc(B, A, off);
        acc_merge(A, B);
    }
}


// Accumulator of a packed level: keys are single words.
struct KeyAcc {
    uint64_t f;      // smallest colliding key
    uint64_t m;      // largest colliding key (levels where m_I can stop)
    uint64_t tm;     // smallest it among terminal colliding boxes
    int64_t fpos;    // where child 0 of f went, or -1
    uint32_t ff;     // bit0: have, bit1: terminal, bit2: small
    uint32_t mh;
    uint32_t th;
};

__device__ __forceinline__ void keyacc_init(KeyAcc& K) {
    K.f = ~0ull; K.m = 0; K.tm = ~0ull; K.fpos = -1; K.ff = 0; K.mh = 0; K.th = 0;
}

__device__ __forceinline__ void keyacc_add(KeyAcc& K, uint64_t key, uint64_t bt, bool term,
                                           bool small, bool track_max, int64_t pos0) {
    if (!(K.ff & 1u) || key < K.f) {
        K.f = key;
        K.ff = 1u | (term ? 2u : 0u) | (small ? 4u : 0u);
        K.fpos = pos0;
    }
    if (track_max && (!K.mh || K.m < key)) {
        K.m = key;
        K.mh = 1;
    }
    if (term && (!K.th || bt < K.tm)) {
        K.tm = bt;
        K.th = 1;
    }
}

__device__ __forceinline__ void keyacc_merge(KeyAcc& K, const KeyAcc& B) {
    if ((B.ff & 1u) && (!(K.ff & 1u) || B.f < K.f)) { K.f = B.f; K.ff = B.ff; K.fpos = B.fpos; }
    if (B.mh && (!K.mh || K.m < B.m)) { K.m = B.m; K.mh = 1; }
    if (B.th && (!K.th || B.tm < K.tm)) { K.tm = B.tm; K.th = 1; }
}

// Lane l's value (l wave-uniform): two v_readlane, no LDS round trip.
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

// Wavefront minimum / maximum of a 64-bit value with DPP moves (no LDS round
// trips): within each row of 16 lanes a running prefix (row_shr 1, 2, 3, then
// 4 and 8 on the upper banks) leaves the row's result in its lane 15; the
// row broadcasts (lane 15 into rows 1 and 3, then lane 31 into rows 2 and 3)
// fold the rows, so that lane 63 holds the wave's result.  A lane whose DPP
// source is masked or outside its row receives the identity.
template <int CTRL, int ROWS, int BANKS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x, uint64_t ident) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)ident, (int)(uint32_t)x,
                                                              CTRL, ROWS, BANKS, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(ident >> 32),
                                                              (int)(uint32_t)(x >> 32), CTRL, ROWS,
                                                              BANKS, false);
    return ((uint64_t)hi << 32) | lo;
}

template <bool MAX>
__device__ __forceinline__ uint64_t wave_ext_u64(uint64_t x) {
    const uint64_t id = MAX ? 0ull : ~0ull;
    auto pick = [](uint64_t a, uint64_t b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
    const uint64_t x0 = x;
    x = pick(x, dpp_u64<0x111, 0xf, 0xf>(x0, id));  // row_shr:1
    x = pick(x, dpp_u64<0x112, 0xf, 0xf>(x0, id));  // row_shr:2
    x = pick(x, dpp_u64<0x113, 0xf, 0xf>(x0, id));  // row_shr:3
    x = pick(x, dpp_u64<0x114, 0xf, 0xe>(x, id));   // row_shr:4, banks 1-3
    x = pick(x, dpp_u64<0x118, 0xf, 0xc>(x, id));   // row_shr:8, banks 2-3
    x = pick(x, dpp_u64<0x142, 0xa, 0xf>(x, id));   // row_bcast:15, rows 1 and 3
    x = pick(x, dpp_u64<0x143, 0xc, 0xf>(x, id));   // row_bcast:31, rows 2 and 3
    return readlane64(x, 63);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) { return wave_ext_u64<false>(x); }
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) { return wave_ext_u64<true>(x); }

// Wavefront reduction; the result is made wave-uniform.  Keys of one level are
// distinct, so the smallest one is held by exactly one lane, which supplies its
// flags and position; the largest key and the smallest terminal time index are
// plain maximum / minimum reductions (lanes without one contribute the
// identity).
__device__ __forceinline__ void keyacc_reduce(KeyAcc& K) {
    const bool hf = (K.ff & 1u) != 0;
    const uint64_t g = wave_min_u64(hf ? K.f : ~0ull);
    const uint64_t hold = __ballot(hf && K.f == g);
    const int l = hold ? __builtin_ctzll(hold) : 0;
    const uint32_t ff = (uint32_t)__builtin_amdgcn_readlane((int)K.ff, l);
    const int64_t fpos = (int64_t)readlane64((uint64_t)K.fpos, l);
    const uint64_t mh = __ballot(K.mh != 0), th = __ballot(K.th != 0);
    // (most levels have neither: no m_I stop possible, no terminal box)
    const uint64_t m = mh ? wave_max_u64(K.mh ? K.m : 0ull) : 0ull;
    const uint64_t tm = th ? wave_min_u64(K.th ? K.tm : ~0ull) : ~0ull;
    K.f = hold ? g : ~0ull;
    K.ff = hold ? ff : 0u;
    K.fpos = hold ? fpos : -1;
    K.m = mh ? m : 0ull; K.mh = mh ? 1u : 0u;
    K.tm = th ? tm : ~0ull; K.th = th ? 1u : 0u;
}

// Pair words (kFmtPair): the flag bit marks a pair whose child 1 passed the prism test.
constexpr uint64_t kPairFlag = 1ull << 63;  // the pair's child 1 passed the prism test

// One buffer of a group arena.  Word i of a packed level (keys or pair words)
// is in LDS when i < nl and in HBM (at the same index) otherwise: the first nl
// words of every level never leave the CU.  Triple levels (three HBM arrays
// of cap words) use nl = 0.
// (The two pointers carry their address spaces so that the compiler keeps an
// LDS access and a global access apart instead of merging them into one flat
// access through a selected pointer.)
typedef __attribute__((address_space(3))) uint64_t lds_u64;
constexpr int kProbeChunks = 16;  // level probe: leading chunks scanned for a colliding box
typedef __attribute__((address_space(1))) uint64_t hbm_u64;

struct Buf {
    lds_u64* lds;
    hbm_u64* hbm;
    int64_t nl;
    __device__ __forceinline__ uint64_t get(int64_t i) const {
        uint64_t v;
        if (i < nl) v = lds[i];
        else v = hbm[i];
        return v;
    }
    __device__ __forceinline__ void put(int64_t i, uint64_t v) const {
        if (i < nl) lds[i] = v;
        else hbm[i] = v;
    }
};

template <int W>
struct GroupShared {
    double Xs[24];  // the query's coordinates, Xs[c*8 + k]
    double Es[3];   // eps per axis
    Acc acc[W];
    KeyAcc kacc[W];
    unsigned long long sum[W][3];
    unsigned long long next_cnt;  // W > 1: words of the next level
    unsigned long long next_box;  // W > 1: boxes of the next level
    int64_t rec;
    int64_t ho[2];      // hand-off: record index and pool offset (or -1)
    // head try / level probe: unchecked words below the first colliding key
    // (multi-wave groups: two chunks, for the streamed candidate check)
    uint64_t cand[W > 1 ? 128 * W : 64];
    unsigned int ncand; // cap-level probe: candidates gathered
};

// ---------------------------------------------------------------------------
// Sibling pairs.  Alg. 2 checks both children of every colliding box that is
// not terminal (the second one only if the vertex-face prism test admits it).
// The two children share the face of the split: 4 of their 8 corners and, on
// a u or v split, both t planes.  A level stored as pairs is checked a pair per
// lane with the shared corner values computed once; every corner value is the
// same sequence of binary64 operations as corner_values_axis() for that
// corner, so the results are those of checking the two boxes one by one.
//
// All three coordinates are evaluated: on the levels this runs on, a chunk of
// 128 boxes where every box already fails after one or two coordinates (the
// only case where stopping early saves time for a wavefront) practically never
// occurs, and the wave-wide test for it costs more than it saves.
//
// tv, uv, vv: the box's lower and upper ends per axis; on the split axis SPLIT
// three values lo < mid < hi (child 0 = [lo, mid], child 1 = [mid, hi]).
//
// Edge-edge corners: F = fl(ea_b - eb_e) with ea_b depending only on the u end
// b and eb_e only on the v end e (for a time plane).  Rounding is monotonic
// (x <= y implies fl(x) <= fl(y)), so over any set of corners that is a
// product of u ends and v ends, min F = fl(min ea - max eb) and max F =
// fl(max ea - min eb): the same values as the corner-by-corner minimum and
// maximum (up to the sign of a zero, which no comparison or width below can
// see), with fewer operations.  MS: the enlargement by d is applied only
// with d > 0 (x - 0 = x exactly).
template <int KIND, int SPLIT, bool MS>
__device__ __forceinline__ void check_pair_lds(const double* Xs, const double* Es,
                                               const double tv[3], const double uv[3],
                                               const double vv[3], double min_sep, double delta,
                                               bool act1, CheckResult& R0, CheckResult& R1) {
    constexpr int NA = SPLIT == 0 ? 3 : 2;
    constexpr int NB = SPLIT == 1 ? 3 : 2;
    constexpr int NE = SPLIT == 2 ? 3 : 2;
    bool col0 = true, ins0 = true, col1 = act1, ins1 = true;
    double wid0 = 0.0, wid1 = 0.0;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
        const double* xs = Xs + c * 8;
        // corner ranges per group: 0 = child 0 only, 1 = the shared face,
        // 2 = child 1 only (4 corners each); each group starts from its first
        double glo[3] = {0.0, 0.0, 0.0}, ghi[3] = {0.0, 0.0, 0.0};
        bool gset[3] = {false, false, false};
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const double ta = tv[a];
            const double sa = 1.0 - ta;
            double P[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) P[k] = sa * xs[k] + ta * xs[k + 4];
            double ea[NB], eb[NE];
            if (KIND == kEE) {
#pragma unroll
                for (int b = 0; b < NB; ++b) ea[b] = (1.0 - uv[b]) * P[0] + uv[b] * P[1];
#pragma unroll
                for (int e = 0; e < NE; ++e) eb[e] = (1.0 - vv[e]) * P[2] + vv[e] * P[3];
                double lo[3], hi[3];
                int ng;
                if (SPLIT == 0) {
                    const double mna = fmin(ea[0], ea[1]), mxa = fmax(ea[0], ea[1]);
                    const double mnb = fmin(eb[0], eb[1]), mxb = fmax(eb[0], eb[1]);
                    lo[0] = mna - mxb; hi[0] = mxa - mnb; ng = 1;
                } else if (SPLIT == 1) {
                    const double mnb = fmin(eb[0], eb[1]), mxb = fmax(eb[0], eb[1]);
#pragma unroll
                    for (int b = 0; b < NB; ++b) { lo[b] = ea[b] - mxb; hi[b] = ea[b] - mnb; }
                    ng = NB;
                } else {
                    const double mna = fmin(ea[0], ea[1]), mxa = fmax(ea[0], ea[1]);
#pragma unroll
                    for (int e = 0; e < NE; ++e) { lo[e] = mna - eb[e]; hi[e] = mxa - eb[e]; }
                    ng = NE;
                }
#pragma unroll
                for (int g = 0; g < 3; ++g) {
                    if (g >= ng) break;
                    const int sp = SPLIT == 0 ? a : g;
                    if (!gset[sp]) { glo[sp] = lo[g]; ghi[sp] = hi[g]; gset[sp] = true; }
                    else { glo[sp] = fmin(glo[sp], lo[g]); ghi[sp] = fmax(ghi[sp], hi[g]); }
                }
                continue;
            }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    double f;
                    if (KIND == kEE) {
                        f = ea[b] - eb[e];
                    } else {
                        const double w = (1.0 - uv[b]) - vv[e];
                        const double s12 = w * P[1] + uv[b] * P[2];
                        f = P[0] - (s12 + vv[e] * P[3]);
                    }
                    const int sp = SPLIT == 0 ? a : (SPLIT == 1 ? b : e);
                    if (!gset[sp]) {
                        glo[sp] = f;
                        ghi[sp] = f;
                        gset[sp] = true;
                    } else {
                        glo[sp] = fmin(glo[sp], f);
                        ghi[sp] = fmax(ghi[sp], f);
                    }
                }
        }
        const double lo0 = fmin(glo[0], glo[1]), hi0 = fmax(ghi[0], ghi[1]);
        const double lo1 = fmin(glo[1], glo[2]), hi1 = fmax(ghi[1], ghi[2]);
        const double eps = Es[c];
        {
            const double l = MS ? lo0 - min_sep : lo0, h = MS ? hi0 + min_sep : hi0;
            col0 = col0 && (l <= eps) && (h >= -eps);
            ins0 = ins0 && (l >= -eps) && (h <= eps);
            wid0 = fmax(wid0, hi0 - lo0);
        }
        {
            const double l = MS ? lo1 - min_sep : lo1, h = MS ? hi1 + min_sep : hi1;
            col1 = col1 && (l <= eps) && (h >= -eps);
            ins1 = ins1 && (l >= -eps) && (h <= eps);
            wid1 = fmax(wid1, hi1 - lo1);
        }
    }
    R0.collide = col0;
    R0.small = (wid0 < delta) || ins0;
    R1.collide = col1;
    R1.small = (wid1 < delta) || ins1;
}

// Child key b of a pair word's parent key (split field at bit sx of the
// current level's packed key).
__device__ __forceinline__ uint64_t pair_child(uint64_t word, int sx, uint64_t lowx, uint64_t b) {
    const uint64_t pk = word & ~kPairFlag;
    return ((((pk >> sx) << 1) | b) << sx) | (pk & lowx);
}

// Shift of an axis field in a packed key with depths (du, dv).
__device__ __forceinline__ int field_shift(int axis, const KeyCodec& kc) {
    return axis == 0 ? kc.st : (axis == 1 ? kc.su : 0);
}

// The boxes one lane holds in one chunk: one (Key / Triple input) or the two
// siblings of a pair word.
struct LaneBoxes {
    uint64_t key[2];          // packed keys (Key / Pair input)
    uint64_t it[2], iu[2], iv[2];
    double t0[2], u0[2], v0[2];
    bool act[2];
    CheckResult R[2];
};

// One level of one query, run by the whole block: check every box, accumulate,
// and store what the next level needs.  FIN: this level's storage format;
// SPLIT: for pair input, the axis the stored parents were split on; OP: store
// the next level as pairs (each colliding box that is not terminal becomes one
// word), else as triples (its admitted children).  S and L are wave-uniform.
// Returns the block-reduced, wave-uniform accumulator with keys as (t, u, v)
// indices, the next level's word and box counts, and in A.fpos where the word
// (pairs) or child 0 (triples) of the smallest colliding box went.
//
// Children: the split axis field of a box gains one low bit (0: lower half,
// 1: upper half).  In a packed key whose split field starts at bit sx this is
//   child_b = ((key >> sx) << (sx + 1)) | (b << sx) | (key & (2^sx - 1)).
// Child 0 shares the parent's (u_lo, v_lo), which passed the vertex-face prism
// test when the parent was made (the root trivially), so only child 1 of a u or
// v split is tested: u_lo + v_lo <= 1 with the new lower end, computed exactly
// in binary64 (all values are multiples of 2^-52 below 2).
//
// Head try (one wavefront, packed input): Alg. 2 ends a level at its first
// colliding box f when f is terminal, when the carried box comes first or when
// m_I is reached at f; the boxes after f are never checked.  The first time a
// chunk holds a colliding box for which one of these can hold, the running
// smallest colliding key g is reduced and the unchecked words holding a key
// below g (usually none or few: the level's smallest key is stored first) are
// checked from LDS.  f is then known exactly (every key below it has been
// checked), its rank comes from a count, and if decide_first() ends the query
// the pass returns early with that outcome; otherwise it goes on unchanged.
// The chunk loop leaves at that chunk and the head try runs outside it, then a
// second loop takes the remaining chunks: the rarely run head-try code is then
// not part of the hot loop (which spills less for it).
template <int W, int KIND, int FIN, int SPLIT, bool OP>
__device__ __forceinline__ void level_pass(GroupShared<W>& sh, const Buf& ct, const Buf& nt,
                                           int64_t cap, const State& S, int64_t words,
                                           const LevelInfo& L, double min_sep, double delta,
                                           bool cap_level, bool literal, int64_t max_iter, Acc& A,
                                           uint64_t& next_words, uint64_t& next_boxes,
                                           bool& early, Outcome& Oe, uint64_t& checked,
                                           unsigned long long* a_counters) {
    constexpr int T = 64 * W;
    constexpr bool kPacked = FIN != kFmtTriple;
    constexpr bool kPair = FIN == kFmtPair;
    constexpr bool kHead = (W == 1) && kPacked;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    KeyCodec kc;
    kc.init(S.d[1], S.d[2]);
    const int axis = L.axis;
    const int psx = kPair ? field_shift(SPLIT, kc) : 0;  // split field of the stored parents
    const uint64_t plowx = mask64(psx);
    // child 1's offset of u_lo and v_lo on this level's split axis (adding 0.0 is
    // exact, so one formula serves the three axes)
    const double du1 = axis == 1 ? 0.5 * L.wu : 0.0, dv1 = axis == 2 ? 0.5 * L.wv : 0.0;
    const double wsp = SPLIT == 0 ? L.wt : (SPLIT == 1 ? L.wu : L.wv);
    KeyAcc K;  // packed input
    if (kPacked) keyacc_init(K);
    else acc_init(A);
    early = false;
    bool tried = !kHead;
    const bool has_pend = !literal && S.tpend < INFINITY;  // a carried box exists
    uint64_t boxes_done = 0;
    unsigned long long next_w = 0, next_b = 0;  // W == 1: running sizes of the next level
    if (W > 1) {
        if (tid == 0) { sh.next_cnt = 0; sh.next_box = 0; }
        __syncthreads();
    }

    // the boxes of the word at index i (FIN's format) and their checks
    // (c0: the chunk's first word, wave-uniform; a chunk lies wholly in LDS or
    // wholly in HBM because the LDS part is a multiple of T words)
    auto load = [&](int64_t c0, uint64_t& p0, uint64_t& p1, uint64_t& p2) {
        const int64_t i = c0 + tid;
        if (kPacked) {
            if (c0 < ct.nl) p0 = ct.lds[i];
            else p0 = ct.hbm[i];
        } else {
            p0 = ct.hbm[i]; p1 = ct.hbm[cap + i]; p2 = ct.hbm[2 * cap + i];
        }
    };
    auto expand = [&](bool act, uint64_t p0, uint64_t p1, uint64_t p2, LaneBoxes& B) {
        B.act[0] = act;
        B.act[1] = false;
        if (kPair) {
            B.key[0] = pair_child(p0, psx, plowx, 0);
            B.key[1] = B.key[0] | (1ull << psx);
            B.act[1] = act && (p0 & kPairFlag);
            kc.decode(B.key[0], B.it[0], B.iu[0], B.iv[0]);
            B.it[1] = B.it[0] + (SPLIT == 0 ? 1 : 0);
            B.iu[1] = B.iu[0] + (SPLIT == 1 ? 1 : 0);
            B.iv[1] = B.iv[0] + (SPLIT == 2 ? 1 : 0);
        } else if (kPacked) {
            B.key[0] = p0;
            kc.decode(p0, B.it[0], B.iu[0], B.iv[0]);
        } else {
            B.it[0] = p0; B.iu[0] = p1; B.iv[0] = p2;
        }
        B.t0[0] = dyadic(B.it[0], L.bt_bits, L.bt_val);
        B.u0[0] = dyadic(B.iu[0], L.bu_bits, L.bu_val);
        B.v0[0] = dyadic(B.iv[0], L.bv_bits, L.bv_val);
        if (kPair) {
            B.t0[1] = SPLIT == 0 ? B.t0[0] + wsp : B.t0[0];
            B.u0[1] = SPLIT == 1 ? B.u0[0] + wsp : B.u0[0];
            B.v0[1] = SPLIT == 2 ? B.v0[0] + wsp : B.v0[0];
        }
    };
    auto check = [&](LaneBoxes& B) {
        B.R[0].collide = false; B.R[0].small = false;
        B.R[1].collide = false; B.R[1].small = false;
        if (!B.act[0]) return;
        if (kPair) {
            double tv[3], uv[3], vv[3];
            // time values tmax * s at s0, s0 + w, s0 + 2w (the sums are exact)
            tv[0] = L.tmax * B.t0[0];
            tv[1] = L.tmax * (B.t0[0] + L.wt);
            tv[2] = L.tmax * ((B.t0[0] + L.wt) + L.wt);
            uv[0] = B.u0[0]; uv[1] = uv[0] + L.wu; uv[2] = uv[1] + L.wu;
            vv[0] = B.v0[0]; vv[1] = vv[0] + L.wv; vv[2] = vv[1] + L.wv;
            if (min_sep > 0.0)
                check_pair_lds<KIND, SPLIT, true>(sh.Xs, sh.Es, tv, uv, vv, min_sep, delta, B.act[1],
                                                  B.R[0], B.R[1]);
            else
                check_pair_lds<KIND, SPLIT, false>(sh.Xs, sh.Es, tv, uv, vv, min_sep, delta, B.act[1],
                                                   B.R[0], B.R[1]);
        } else {
            B.R[0] = check_box_lds<KIND>(sh.Xs, sh.Es, L.tmax * B.t0[0], L.tmax * (B.t0[0] + L.wt), B.u0[0],
                                         B.u0[0] + L.wu, B.v0[0], B.v0[0] + L.wv, min_sep, delta);
        }
    };

    // Level probe of the multi-wave groups (which have no head try).  Alg. 2
    // ends a level at its first colliding box f (carried box first, m_I
    // reached at f, f terminal) or, on a level where m_I can stop the query
    // (N + |level| >= m_I), at the first colliding box whose rank is at least
    // m_I - N - 1, with t_lo(f) either way; only when neither happens does the
    // level go on to the next.  So f with its rank, and on such a level any
    // colliding box of large enough rank, decide the level without checking
    // the boxes in between.  The probe checks the level's chunks in storage
    // order (the first holds its smallest key) until one holds a colliding
    // box, and on an m_I level also the last chunk (keys of large rank).
    // When a checked colliding box could end the query (terminal, at or after
    // the carried box), or on an m_I level, it counts ranks with one pass over
    // the keys, checks the unprobed boxes below the smallest colliding probe
    // box (so that f is exact), and returns the decision if it is proven;
    // otherwise the level is checked in full as usual.  (Single-wave groups
    // stop the same levels with the head try below, and hand m_I levels of
    // more than four chunks to the block tier; measured, a probe there costs
    // more in register pressure than it saves.)
    if (kPacked && W > 1) {
        const uint64_t mI = (uint64_t)max_iter;
        KeyAcc P;
        keyacc_init(P);
        unsigned long long nprobe = 0;
        bool ends = cap_level;
        // the level's first chunks, in storage order, until one holds a
        // colliding box (at most kProbeChunks of them), then (m_I level) the
        // last chunk
        auto probe_chunk = [&](int64_t c) -> bool {
            uint64_t q0 = 0, q1 = 0, q2 = 0;
            const bool act = c + tid < words;
            if (act) load(c, q0, q1, q2);
            LaneBoxes B;
            expand(act, q0, q1, q2, B);
            check(B);
            nprobe += (B.act[0] ? 1 : 0) + (B.act[1] ? 1 : 0);
            bool col = false;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (!B.R[b].collide) continue;
                col = true;
                const bool tb = B.R[b].small || L.dcap;
                keyacc_add(P, B.key[b], B.it[b], tb, B.R[b].small, true, -1);
                ends = ends || tb || (!literal && S.tpend <= L.tmax * B.t0[b]);
            }
            return col;
        };
        int64_t cend = 0;  // chunks [0, cend) scanned
        for (int k = 0; k < kProbeChunks && cend < words; ++k) {
            const bool col = probe_chunk(cend);
            cend += T;
            if (__syncthreads_or(col ? 1 : 0)) break;
        }
        // m_I level: the last chunks, backwards, until one holds a colliding box
        // (at most kProbeChunks of them, none already scanned): [c1, words)
        int64_t c1 = words;
        if (cap_level) {
            int64_t c = ((words - 1) / T) * T;
            for (int k = 0; k < kProbeChunks && c >= cend; ++k, c -= T) {
                const bool col = probe_chunk(c);
                c1 = c;
                if (__syncthreads_or(col ? 1 : 0)) break;
            }
        }
        ends = __syncthreads_or(ends ? 1 : 0) != 0;
        auto block_keyacc = [&](KeyAcc& X) {
            keyacc_reduce(X);
            if (W > 1) {
                if (lane == 0) sh.kacc[wid] = X;
                __syncthreads();
                X = sh.kacc[0];
                for (int w = 1; w < W; ++w) keyacc_merge(X, sh.kacc[w]);
                __syncthreads();
                X.f = uni64(X.f); X.m = uni64(X.m); X.ff = uni32(X.ff); X.mh = uni32(X.mh);
            }
        };
        auto block_sum3 = [&](unsigned long long& x0, unsigned long long& x1, unsigned long long& x2) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                x0 += __shfl_xor(x0, off);
                x1 += __shfl_xor(x1, off);
                x2 += __shfl_xor(x2, off);
            }
            if (W > 1) {
                if (lane == 0) { sh.sum[wid][0] = x0; sh.sum[wid][1] = x1; sh.sum[wid][2] = x2; }
                __syncthreads();
                x0 = 0; x1 = 0; x2 = 0;
                for (int w = 0; w < W; ++w) { x0 += sh.sum[w][0]; x1 += sh.sum[w][1]; x2 += sh.sum[w][2]; }
                __syncthreads();
            }
            x0 = uni64(x0); x1 = uni64(x1); x2 = uni64(x2);
        };
        block_keyacc(P);
        if ((P.ff & 1u) && ends) {
            if (tid == 0) atomicAdd(&a_counters[kCntProbe], 1ull);
            const uint64_t gmin = P.f, gmax = P.m;
            // ranks of gmin and gmax; unprobed words that hold a key below gmin
            if (tid == 0) sh.ncand = 0;
            __syncthreads();
            unsigned long long rmin = 0, rmax = 0;
            for (int64_t j = tid; j < words; j += T) {
                const uint64_t wd = ct.get(j);
                const uint64_t k0 = kPair ? pair_child(wd, psx, plowx, 0) : wd;
                const bool two = kPair && (wd & kPairFlag);
                const uint64_t k1 = k0 | (1ull << psx);
                rmin += (k0 < gmin ? 1 : 0) + ((two && k1 < gmin) ? 1 : 0);
                rmax += (k0 < gmax ? 1 : 0) + ((two && k1 < gmax) ? 1 : 0);
                const bool probed = j < cend || j >= c1;
                if (!probed && k0 < gmin) {
                    const unsigned int at = atomicAdd(&sh.ncand, 1u);
                    if (at < (unsigned int)T) sh.cand[at] = wd;
                }
            }
            __syncthreads();
            const unsigned int ncand = uni32(sh.ncand);
            block_sum3(rmin, rmax, nprobe);
            // the candidates are checked one chunk's worth (T words) at a time:
            // at most T of them are in sh.cand already; more (up to a quarter
            // of the level's words, beyond which the full pass is cheaper) are
            // gathered again from the level in storage order, the gathering
            // stopping whenever a chunk's worth waits (sh.cand holds 2 T)
            const bool stream = ncand > (unsigned int)T;
            if (!stream || 4 * (uint64_t)ncand <= (uint64_t)words) {
                KeyAcc G;
                keyacc_init(G);
                unsigned long long ncheck = 0;
                int64_t sc = 0;  // streamed gathering: next storage chunk
                if (stream) {
                    __syncthreads();
                    if (tid == 0) sh.ncand = 0;
                    __syncthreads();
                }
                while (true) {
                    unsigned int n = ncand;
                    if (stream) {
                        while (sc < words) {
                            const int64_t j = sc + tid;
                            if (j < words && !(j < cend || j >= c1)) {
                                const uint64_t wd = ct.get(j);
                                const uint64_t k0 = kPair ? pair_child(wd, psx, plowx, 0) : wd;
                                if (k0 < gmin) sh.cand[atomicAdd(&sh.ncand, 1u)] = wd;
                            }
                            sc += T;
                            __syncthreads();
                            const unsigned int waiting = uni32(sh.ncand);
                            __syncthreads();  // every wave has read it before the next appends
                            if (waiting >= (unsigned int)T) break;
                        }
                        n = min(uni32(sh.ncand), (unsigned int)T);
                    }
                    if (n == 0) break;
                    const bool cact = tid < (int)n;
                    const uint64_t cw = cact ? sh.cand[tid] : 0;
                    LaneBoxes C;
                    expand(cact, cw, 0, 0, C);
                    check(C);
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        if (C.R[b].collide)
                            keyacc_add(G, C.key[b], C.it[b], C.R[b].small || L.dcap, C.R[b].small, false, -1);
                    ncheck += (C.act[0] ? 1 : 0) + (C.act[1] ? 1 : 0);
                    if (!stream) break;
                    // the waiting words beyond the checked chunk move to the front
                    const unsigned int m = uni32(sh.ncand);
                    const uint64_t rest = (unsigned int)tid + T < m ? sh.cand[T + tid] : 0;
                    __syncthreads();
                    if ((unsigned int)tid + T < m) sh.cand[tid] = rest;
                    if (tid == 0) sh.ncand = m > (unsigned int)T ? m - T : 0;
                    __syncthreads();
                }
                block_keyacc(G);
                uint64_t f = gmin;
                uint32_t ff = P.ff;
                unsigned long long rf = rmin;
                if ((G.ff & 1u) && G.f < gmin) {
                    // a candidate below gmin collides: it is f; its rank by a count
                    f = G.f;
                    ff = G.ff;
                    unsigned long long r = 0, z = 0;
                    for (int64_t j = tid; j < words; j += T) {
                        const uint64_t wd = ct.get(j);
                        const uint64_t k0 = kPair ? pair_child(wd, psx, plowx, 0) : wd;
                        const bool two = kPair && (wd & kPairFlag);
                        r += (k0 < f ? 1 : 0) + ((two && (k0 | (1ull << psx)) < f) ? 1 : 0);
                    }
                    block_sum3(r, z, ncheck);
                    rf = r;
                } else {
                    unsigned long long z0 = 0, z1 = 0;
                    block_sum3(z0, z1, ncheck);
                }
                Acc Fa;
                acc_init(Fa);
                kc.decode(f, Fa.ft, Fa.fu, Fa.fv);
                Fa.fflags = ff;
                Outcome O = decide_first(Fa, S, literal, max_iter, L, rf);
                if (!O.finish && cap_level && S.N + rmax + 1 >= mI) {
                    // a colliding box at rank >= m_I - N - 1: the m_I stop
                    O.finish = true;
                    O.toi = L.tmax * ((double)Fa.ft * L.wt);
                    O.tw = L.tmax * L.wt;
                    O.n = mI;
                    O.st = kStCap;
                }
                if (O.finish) {
                    if (tid == 0) atomicAdd(&a_counters[kCntProbeHit], 1ull);
                    early = true;
                    Oe = O;
                    checked = nprobe + ncheck;
                    return;
                }
            }
        }
    }

    uint64_t p0 = 0, p1 = 0, p2 = 0;  // software pipelining: the next chunk loads early
    if (tid < words) load(0, p0, p1, p2);
    // one chunk of T words: check, accumulate, store the next level; returns
    // whether a colliding box of it could end the query (head try)
    auto chunk = [&](int64_t b0) -> bool {
        const int64_t i = b0 + tid;
        const bool act = i < words;
        LaneBoxes B;
        expand(act, p0, p1, p2, B);
        if (i + T < words) load(b0 + T, p0, p1, p2);
        check(B);
        if (kHead) boxes_done += __popcll(__ballot(B.act[0])) + __popcll(__ballot(B.act[1]));
        bool col[2], term[2], e[2], adm[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            col[b] = B.R[b].collide;
            term[b] = B.R[b].small || L.dcap;
            e[b] = col[b] && !term[b];
            // vertex-face prism test of child 1; on a t split its (u_lo, v_lo) is
            // the box's own, which passed when the box was made
            // (every box of a level has u_lo + v_lo <= 1, so child 1 of a t
            // split is admitted without the test)
            adm[b] = KIND != kVF || axis == 0 || (B.u0[b] + du1) + (B.v0[b] + dv1) <= 1.0;
        }
        // positions of what this lane stores for the next level
        int64_t q[2];
        unsigned long long wtot, btot;
        uint64_t mk[4];
        if (OP) {
            mk[0] = __ballot(e[0]); mk[1] = __ballot(e[1]);
            mk[2] = __ballot(e[0] && adm[0]); mk[3] = __ballot(e[1] && adm[1]);
            wtot = __popcll(mk[0]) + __popcll(mk[1]);
            btot = wtot + __popcll(mk[2]) + __popcll(mk[3]);
        } else {
            mk[0] = __ballot(e[0]); mk[1] = __ballot(e[0] && adm[0]);
            mk[2] = __ballot(e[1]); mk[3] = __ballot(e[1] && adm[1]);
            wtot = __popcll(mk[0]) + __popcll(mk[1]) + __popcll(mk[2]) + __popcll(mk[3]);
            btot = wtot;
        }
        unsigned long long wbase;
        if (W == 1) {
            wbase = next_w;
            next_w += wtot;
            next_b += btot;
        } else {
            unsigned long long t = 0;
            if (lane == 0 && wtot) {
                t = atomicAdd(&sh.next_cnt, wtot);
                atomicAdd(&sh.next_box, btot);
            }
            wbase = readlane64(t, 0);
        }
        if (OP) {
            // one word per stored box; mk[2], mk[3] only count boxes
            q[0] = (int64_t)wbase + below_lane(mk[0], mk[1]);
            q[1] = q[0] + (e[0] ? 1 : 0);
        } else {
            // up to four child triples per lane, all counted by mk[0..3]
            q[0] = (int64_t)wbase + below_lane(mk[0], mk[1]) + below_lane(mk[2], mk[3]);
            q[1] = q[0] + (e[0] ? 1 : 0) + (e[0] && adm[0] ? 1 : 0);
        }
        if (kPacked) {
            // smallest colliding key, every level
            // a lane's second box has the larger key (sibling 1 of a pair): it can
            // only be the lane's smallest colliding key when the first misses
            {
                const int b = col[0] ? 0 : 1;
                const bool c = col[0] || col[1];
                const uint64_t key = b ? B.key[1] : B.key[0];
                const bool eb = b ? e[1] : e[0];
                const int64_t qb = b ? q[1] : q[0];
                const bool tb = b ? term[1] : term[0];
                const bool sb = b ? B.R[1].small : B.R[0].small;
                if (c && (!(K.ff & 1u) || key < K.f)) {
                    K.f = key;
                    K.ff = 1u | (tb ? 2u : 0u) | (sb ? 4u : 0u);
                    K.fpos = (eb && qb < cap) ? qb : -1;
                }
            }
            // largest colliding key: only on a level where m_I can stop
            if (cap_level) {
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    if (col[b] && (!K.mh || K.m < B.key[b])) { K.m = B.key[b]; K.mh = 1; }
            }
            // terminal colliding boxes (the carried box): rare before the last level
            if (__ballot((col[0] && term[0]) || (col[1] && term[1])) != 0) {
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    if (col[b] && term[b] && (!K.th || B.it[b] < K.tm)) { K.tm = B.it[b]; K.th = 1; }
            }
        } else {
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (!col[b]) continue;
                const int64_t pos = (e[b] && q[b] < cap) ? q[b] : -1;
                acc_add(A, B.it[b], B.iu[b], B.iv[b], term[b], B.R[b].small, cap_level, pos);
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            if (!e[b]) continue;
            if (OP) {
                if (q[b] < cap) nt.put(q[b], B.key[b] | (adm[b] ? kPairFlag : 0ull));
            } else {
                const uint64_t c0t = axis == 0 ? 2 * B.it[b] : B.it[b];
                const uint64_t c0u = axis == 1 ? 2 * B.iu[b] : B.iu[b];
                const uint64_t c0v = axis == 2 ? 2 * B.iv[b] : B.iv[b];
                const int64_t r0 = q[b];
                hbm_u64* nh = nt.hbm;
                if (r0 < cap) { nh[r0] = c0t; nh[cap + r0] = c0u; nh[2 * cap + r0] = c0v; }
                const int64_t r1 = r0 + 1;
                if (adm[b] && r1 < cap) {
                    nh[r1] = c0t | (axis == 0 ? 1 : 0);
                    nh[cap + r1] = c0u | (axis == 1 ? 1 : 0);
                    nh[2 * cap + r1] = c0v | (axis == 2 ? 1 : 0);
                }
            }
        }
        bool found = false;
        if (kHead && !tried) {
            bool ends = false;
#pragma unroll
            for (int b = 0; b < 2; ++b) ends = ends || (col[b] && (term[b] || cap_level));
            // the carried box can come first only when there is one
            if (has_pend) {
#pragma unroll
                for (int b = 0; b < 2; ++b) ends = ends || (col[b] && S.tpend <= L.tmax * B.t0[b]);
            }
            found = __ballot(ends) != 0;
        }
        return found;
    };
    int64_t b0 = 0;
    bool found = false;
    for (; b0 < words; b0 += T) {
        if (chunk(b0)) {
            found = true;
            b0 += T;
            break;
        }
    }
    if (kHead && found) {
        tried = true;
        const uint64_t lt = lanemask_lt();
        KeyAcc F = K;
        keyacc_reduce(F);
        const uint64_t g = F.f;
        const int64_t done = b0 < words ? b0 : words;
        // unchecked words holding a key below g, gathered in LDS
        uint32_t nc = 0;
        bool fits = true;
        for (int64_t j0 = done; j0 < words; j0 += T) {
            const int64_t j = j0 + lane;
            const uint64_t wd = j < words ? ct.get(j) : 0;
            const uint64_t k0 = kPair ? pair_child(wd, psx, plowx, 0) : wd;
            const bool below = j < words && k0 < g;
            const uint64_t m = __ballot(below);
            if (m) {
                const uint32_t c = (uint32_t)__popcll(m);
                if (nc + c > 64) { fits = false; break; }
                if (below) sh.cand[nc + __popcll(m & lt)] = wd;
                nc += c;
            }
        }
        if (fits) {
            __syncthreads();  // one wavefront: orders the LDS writes before the reads
            const bool cact = (uint32_t)lane < nc;
            const uint64_t cw = cact ? sh.cand[lane] : 0;
            LaneBoxes C;
            expand(cact, cw, 0, 0, C);
            check(C);
            KeyAcc G;
            keyacc_init(G);
#pragma unroll
            for (int b = 0; b < 2; ++b)
                if (C.R[b].collide)
                    keyacc_add(G, C.key[b], C.it[b], C.R[b].small || L.dcap, C.R[b].small,
                               false, -1);
            keyacc_reduce(G);
            keyacc_merge(F, G);
            const uint64_t f = F.f;  // the level's first colliding key
            // rank of f: keys below it among checked words and candidates
            unsigned long long r = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) r += (C.act[b] && C.key[b] < f) ? 1 : 0;
            for (int64_t j = lane; j < done; j += T) {
                const uint64_t wd = ct.get(j);
                if (kPair) {
                    const uint64_t k0 = pair_child(wd, psx, plowx, 0);
                    r += k0 < f ? 1 : 0;
                    r += ((wd & kPairFlag) && (k0 | (1ull << psx)) < f) ? 1 : 0;
                } else {
                    r += wd < f ? 1 : 0;
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off);
            const uint64_t rf = uni64(r);
            Acc Fa;
            acc_init(Fa);
            kc.decode(f, Fa.ft, Fa.fu, Fa.fv);
            Fa.fflags = F.ff;
            const Outcome O = decide_first(Fa, S, literal, max_iter, L, rf);
            if (O.finish) {
                early = true;
                Oe = O;
                checked = boxes_done + (uint64_t)(__popcll(__ballot(C.act[0])) +
                                                  __popcll(__ballot(C.act[1])));
                return;
            }
        }
        // the head try did not end the query: the level goes on
        for (; b0 < words; b0 += T) (void)chunk(b0);
    }
    checked = S.cnt;
    if (kPacked) {
        keyacc_reduce(K);
        if (W > 1) {
            if (lane == 0) sh.kacc[wid] = K;
            __syncthreads();
            K = sh.kacc[0];
            for (int w = 1; w < W; ++w) keyacc_merge(K, sh.kacc[w]);
            next_w = sh.next_cnt;
            next_b = sh.next_box;
            __syncthreads();
            K.f = uni64(K.f); K.m = uni64(K.m); K.tm = uni64(K.tm); K.fpos = uni64s(K.fpos);
            K.ff = uni32(K.ff); K.mh = uni32(K.mh); K.th = uni32(K.th);
        }
        acc_init(A);
        if (K.ff & 1u) kc.decode(K.f, A.ft, A.fu, A.fv);
        if (K.mh) kc.decode(K.m, A.mt, A.mu, A.mv);
        A.fflags = K.ff; A.mhave = K.mh; A.tm = K.tm; A.thave = K.th; A.fpos = K.fpos;
    } else {
        wave_reduce_acc(A);
        if (W > 1) {
            if (lane == 0) sh.acc[wid] = A;
            __syncthreads();
            A = sh.acc[0];
            for (int w = 1; w < W; ++w) acc_merge(A, sh.acc[w]);
            next_w = sh.next_cnt;
            next_b = sh.next_box;
            __syncthreads();
        }
        acc_uniform(A);
    }
    next_words = uni64(next_w);
    next_boxes = uni64(next_b);
}

// Number of boxes of the level below f and below m (keys as (t, u, v)).
template <int W, int FIN, int SPLIT>
__device__ __forceinline__ void rank_pass(GroupShared<W>& sh, const Buf& ct, int64_t cap,
                                          const State& S, int64_t words, const Acc& A,
                                          uint64_t& rf, uint64_t& rm) {
    constexpr int T = 64 * W;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    KeyCodec kc;
    kc.init(S.d[1], S.d[2]);
    const uint64_t fk = kc.encode(A.ft, A.fu, A.fv);
    const uint64_t mk = kc.encode(A.mt, A.mu, A.mv);
    const int psx = FIN == kFmtPair ? field_shift(SPLIT, kc) : 0;
    const uint64_t plowx = mask64(psx);
    unsigned long long sf = 0, sm = 0;
    for (int64_t i = tid; i < words; i += T) {
        if (FIN == kFmtPair) {
            const uint64_t wd = ct.get(i);
            const uint64_t k0 = pair_child(wd, psx, plowx, 0);
            const uint64_t k1 = k0 | (1ull << psx);
            const bool two = (wd & kPairFlag) != 0;
            sf += (k0 < fk ? 1 : 0) + ((two && k1 < fk) ? 1 : 0);
            sm += (k0 < mk ? 1 : 0) + ((two && k1 < mk) ? 1 : 0);
        } else if (FIN == kFmtKey) {
            const uint64_t k = ct.get(i);
            sf += k < fk ? 1 : 0;
            sm += k < mk ? 1 : 0;
        } else {
            const uint64_t kt = ct.hbm[i], ku = ct.hbm[cap + i], kv = ct.hbm[2 * cap + i];
            sf += key_less(kt, ku, kv, A.ft, A.fu, A.fv) ? 1 : 0;
            sm += key_less(kt, ku, kv, A.mt, A.mu, A.mv) ? 1 : 0;
        }
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
    rf = uni64(sf);
    rm = uni64(sm);
}

__device__ __forceinline__ int depth_sum(const int32_t d[3]) { return d[0] + d[1] + d[2]; }

// Dispatch of one level to the pass for its storage format, pair split axis
// and output format (all wave-uniform).
template <int W, int KIND>
__device__ __forceinline__ void run_level(GroupShared<W>& sh, const Buf& ct, const Buf& nt,
                                          int64_t cap, const State& S, int64_t words, int fmt,
                                          int pa, bool op, const LevelInfo& L, double min_sep,
                                          double delta, bool cap_level, bool literal,
                                          int64_t max_iter, Acc& A, uint64_t& nw, uint64_t& nb,
                                          bool& early, Outcome& Oe, uint64_t& checked,
                                          unsigned long long* counters) {
#define CCD_PASS(FIN, SP, OPV)                                                                    \
    level_pass<W, KIND, FIN, SP, OPV>(sh, ct, nt, cap, S, words, L, min_sep, delta, cap_level,    \
                                      literal, max_iter, A, nw, nb, early, Oe, checked, counters)
    if (fmt == kFmtPair) {
        if (op) {
            if (pa == 0) CCD_PASS(kFmtPair, 0, true);
            else if (pa == 1) CCD_PASS(kFmtPair, 1, true);
            else CCD_PASS(kFmtPair, 2, true);
        } else {
            if (pa == 0) CCD_PASS(kFmtPair, 0, false);
            else if (pa == 1) CCD_PASS(kFmtPair, 1, false);
            else CCD_PASS(kFmtPair, 2, false);
        }
    } else if (fmt == kFmtKey) {
        if (op) CCD_PASS(kFmtKey, 0, true);
        else CCD_PASS(kFmtKey, 0, false);
    } else {
        CCD_PASS(kFmtTriple, 0, false);
    }
#undef CCD_PASS
}

template <int W>
__device__ __forceinline__ void run_rank(GroupShared<W>& sh, const Buf& ct, int64_t cap,
                                         const State& S, int64_t words, int fmt, int pa,
                                         const Acc& A, uint64_t& rf, uint64_t& rm) {
    if (fmt == kFmtPair) {
        if (pa == 0) rank_pass<W, kFmtPair, 0>(sh, ct, cap, S, words, A, rf, rm);
        else if (pa == 1) rank_pass<W, kFmtPair, 1>(sh, ct, cap, S, words, A, rf, rm);
        else rank_pass<W, kFmtPair, 2>(sh, ct, cap, S, words, A, rf, rm);
    } else if (fmt == kFmtKey) {
        rank_pass<W, kFmtKey, 0>(sh, ct, cap, S, words, A, rf, rm);
    } else {
        rank_pass<W, kFmtTriple, 0>(sh, ct, cap, S, words, A, rf, rm);
    }
}

// The level loop of one query, run by the whole block.  The level's boxes are
// in buffer 0 of the block's arena when it starts, as packed keys when their
// depth sum allows it, else as triples.
// Hands a query on to the next engine at the start of its current level (in
// buffer ct, `words` words in format fmt): a record with the level's state,
// its words copied to the hand-off pool.  When the pool is full the record
// restarts the query at level 0 instead (same results, more work).  Returns
// false (nothing written) when there is no next engine or no record left.
template <int W>
__device__ __forceinline__ bool handoff(const BatchArgs& a, const GroupCfg& g, GroupShared<W>& sh,
                                        const State& S, int fmt, int pa, int64_t words, const Buf& ct,
                                        int64_t cap, int64_t q) {
    constexpr int T = 64 * W;
    const int tid = threadIdx.x;
    const int64_t nwords = (fmt == kFmtTriple ? 3 : 1) * words;
    if (tid == 0) {
        int64_t o = -1, p = -1;
        if (g.out_records) {
            const unsigned long long r = atomicAdd(&a.counters[g.out_count_idx], 1ull);
            if ((int64_t)r < g.out_record_cap) {
                o = (int64_t)r;
                const unsigned long long po = atomicAdd(&a.counters[kCntPool], (unsigned long long)nwords);
                if ((int64_t)po + nwords <= g.out_pool_words) p = (int64_t)po;
            }
        }
        sh.ho[0] = o;
        sh.ho[1] = p;
    }
    __syncthreads();
    const int64_t o = uni64s(sh.ho[0]), p = uni64s(sh.ho[1]);
    __syncthreads();  // (sh.ho is not read again before the next level's writes)
    if (o < 0) return false;
    uint64_t* orec = g.out_records + o * g.out_record_words;
    if (p >= 0) {
        uint64_t* dst = g.out_pool + p;
        for (int64_t i = tid; i < words; i += T) {
            if (fmt == kFmtTriple) {
                dst[i] = ct.hbm[i];
                dst[words + i] = ct.hbm[cap + i];
                dst[2 * words + i] = ct.hbm[2 * cap + i];
            } else {
                dst[i] = ct.get(i);
            }
        }
    }
    if (tid == 0) {
        Record nh;
        nh.q = q;
        if (p >= 0) {
            nh.N = S.N; nh.tpend = S.tpend; nh.wpend = S.wpend; nh.level = S.level;
            nh.d[0] = S.d[0]; nh.d[1] = S.d[1]; nh.d[2] = S.d[2]; nh.cnt = S.cnt;
            nh.fmt = (uint32_t)fmt | ((uint32_t)pa << 4);
            nh.words = (uint64_t)words;
            orec[kRecordHeaderWords] = (uint64_t)p;
        } else {
            nh.N = 0; nh.tpend = INFINITY; nh.wpend = 0.0; nh.level = 0;
            nh.d[0] = nh.d[1] = nh.d[2] = 0; nh.cnt = 1; nh.fmt = kFmtKey; nh.words = 0;
            orec[kRecordHeaderWords] = 0;
            atomicAdd(&a.counters[kCntRestart], 1ull);
        }
        *reinterpret_cast<Record*>(orec) = nh;
    }
    return true;
}

template <int W, int KIND>
__device__ __forceinline__ void group_query(const BatchArgs& a, const GroupCfg& g, GroupShared<W>& sh,
                                            uint64_t* base, uint64_t* lbase, int64_t nl,
                                            const Record& h, int fmt, int pa,
                                            int64_t words, const double kappa[3],
                                            double delta, double min_sep, double tmax,
                                            int64_t max_iter, bool literal, uint64_t& nchk,
                                            uint64_t& slots) {
    constexpr int T = 64 * W;
    const int tid = threadIdx.x;
    const int64_t cap = g.capacity;
    State S;
    S.N = h.N; S.tpend = h.tpend; S.wpend = h.wpend; S.level = h.level;
    S.d[0] = h.d[0]; S.d[1] = h.d[1]; S.d[2] = h.d[2]; S.cnt = h.cnt;
    int cur = 0;
    while (true) {
        LevelInfo L = level_info(kappa, S.d, tmax);
        // equal in every lane: keep the level's description in scalar registers
        L.axis = (int)uni32((uint32_t)L.axis);
        L.dcap = uni32(L.dcap ? 1u : 0u) != 0;
        L.wt = unif64(L.wt); L.wu = unif64(L.wu); L.wv = unif64(L.wv);
        // pairs need this level's keys packed with a spare top bit
        const bool op = fmt != kFmtTriple && depth_sum(S.d) <= 63;
        const Buf ct{(lds_u64*)(lbase + cur * nl), (hbm_u64*)(base + cur * 3 * cap),
                     fmt != kFmtTriple ? nl : 0};
        const Buf nt{(lds_u64*)(lbase + (cur ^ 1) * nl), (hbm_u64*)(base + (cur ^ 1) * 3 * cap),
                     op ? nl : 0};
        const bool cap_level = S.N + S.cnt >= (uint64_t)max_iter;
        // the next level could outgrow this arena (it has at most two words per
        // word of this one), or this is a level where m_I can stop the query and
        // it spans more than a few chunks (the next engine's level probe
        // decides such a level without checking it in full), or (single-wave
        // groups) every record of this engine has been taken, the level has
        // at least cap / 16 words and fewer than g.tail_records such
        // hand-offs have been made: the heavy queries that started last
        // would otherwise run their widest levels on one wave each while the
        // other groups sit idle, and the block engine checks them eight
        // waves at a time.  Hand the query on before checking this level, so
        // that the next engine checks it once.
        bool tail = false;
        if (W == 1 && g.out_records && 16 * words >= cap &&
            (int64_t)__atomic_load_n(&a.counters[kCntTail], __ATOMIC_RELAXED) < g.tail_records) {
            int64_t cnt = (int64_t)__atomic_load_n(&a.counters[g.in_count_idx], __ATOMIC_RELAXED);
            if (cnt > g.in_record_cap) cnt = g.in_record_cap;
            tail = (int64_t)__atomic_load_n(&a.counters[g.in_take_idx], __ATOMIC_RELAXED) >= cnt;
        }
        tail = uni32(tail ? 1u : 0u) != 0;
        if (tail && tid == 0) atomicAdd(&a.counters[kCntTail], 1ull);
        if (g.out_records && (2 * words > cap || (cap_level && words > 4 * T) || tail) &&
            handoff<W>(a, g, sh, S, fmt, pa, words, ct, cap, h.q))
            return;
        Acc A;
        uint64_t nw = 0, nb = 0, checked = 0;
        bool early;
        Outcome Oe;
        run_level<W, KIND>(sh, ct, nt, cap, S, words, fmt, pa, op, L, min_sep, delta, cap_level,
                           literal, max_iter, A, nw, nb, early, Oe, checked, a.counters);
        if (tid == 0) {
            nchk += checked;
            slots += (uint64_t)((words + T - 1) / T) * T * (fmt == kFmtPair ? 2 : 1);
        }
        if (early) {
            if (tid == 0) write_result(a, h.q, Oe);
            return;
        }
        uint64_t rf = 0, rm = 0;
        if (need_rank(A, S, literal, max_iter, L)) run_rank<W>(sh, ct, cap, S, words, fmt, pa, A, rf, rm);
        const Outcome O = decide(A, S, literal, max_iter, L, rf, rm);
        if (O.finish) {
            if (tid == 0) write_result(a, h.q, O);
            return;
        }
        if (nw > (uint64_t)cap) {
            // the next level does not fit: hand the query on (it checks this
            // level again), or end it with the flagged overflow return when
            // there is no next engine (or no record left)
            if (!handoff<W>(a, g, sh, S, fmt, pa, words, ct, cap, h.q) && tid == 0)
                write_overflow(a, h.q, A, S, L, max_iter);
            return;
        }
        // f is colliding and not terminal here, so its word (pairs) or child 0
        // (triples) is on the next level and holds that level's smallest key
        // (bisection preserves Alg. 2's order): store it first, where the head
        // try and the level probe look first (a level of one chunk is checked
        // whole in its first chunk anyway)
        if (A.fpos > 0 && nw > (uint64_t)T) {
            __syncthreads();
            if (tid == 0) {
                const int64_t p = A.fpos;
                if (op) {
                    const uint64_t x0 = nt.get(0), xp = nt.get(p);
                    nt.put(0, xp);
                    nt.put(p, x0);
                } else {
                    for (int w = 0; w < 3; ++w) {
                        const uint64_t x0 = nt.hbm[w * cap], xp = nt.hbm[w * cap + p];
                        nt.hbm[w * cap] = xp;
                        nt.hbm[w * cap + p] = x0;
                    }
                }
            }
        }
        advance(S, A, literal, L, (uint32_t)nb);
        fmt = op ? kFmtPair : kFmtTriple;
        pa = L.axis;
        words = (int64_t)nw;
        cur ^= 1;
        __syncthreads();
    }
}

// OCC: minimum resident waves per SIMD the register allocation must allow.
// LDS: the first g.lds_words words of every packed level stay in LDS (without
// it the limit is the constant 0 and the LDS paths compile away).
template <int W, int OCC, bool LDS>
__global__ __launch_bounds__(64 * W, OCC) void k_group(BatchArgs a, GroupCfg g) {
    constexpr int T = 64 * W;
    const int tid = threadIdx.x;
    __shared__ GroupShared<W> sh;
    extern __shared__ uint64_t group_lds[];  // two level buffers of g.lds_words words
    const int64_t cap = g.capacity;
    // (a multiple of T: chunks lie wholly in LDS or wholly in HBM)
    const int64_t nl = LDS ? (g.lds_words & ~(int64_t)(T - 1)) : 0;
    uint64_t* base = g.arena + (int64_t)blockIdx.x * (6 * cap);
    int64_t in_count = (int64_t)__atomic_load_n(&a.counters[g.in_count_idx], __ATOMIC_RELAXED);
    if (in_count > g.in_record_cap) in_count = g.in_record_cap;
    uint64_t nchk[2] = {0, 0};
    uint64_t slots = 0;
    while (true) {
        if (tid == 0) sh.rec = (int64_t)atomicAdd(&a.counters[g.in_take_idx], 1ull);
        __syncthreads();
        const int64_t r = uni64s(sh.rec);
        if (r >= in_count) break;
        const uint64_t* rec = g.in_records + (g.in_perm ? g.in_perm[r] : r) * g.in_record_words;
        // everything below is per query, hence wave-uniform (scalar registers)
        Record h = *reinterpret_cast<const Record*>(rec);
        h.q = uni64s(h.q);
        h.N = uni64(h.N);
        h.tpend = unif64(h.tpend);
        h.wpend = unif64(h.wpend);
        h.level = (int32_t)uni32((uint32_t)h.level);
        for (int k = 0; k < 3; ++k) h.d[k] = (int32_t)uni32((uint32_t)h.d[k]);
        h.cnt = uni32(h.cnt);
        const QView qv = view(a, h.q);
        const int64_t q = qv.q;
        const int kind = (int)uni32(qv.kind ? (uint32_t)qv.kind[q] : qv.default_kind);
        const double delta = unif64(qv.delta_q ? qv.delta_q[q] : qv.delta);
        const int64_t max_iter = uni64s(qv.max_iter_q ? qv.max_iter_q[q] : qv.max_iter);
        const double min_sep = unif64(qv.min_sep_q ? qv.min_sep_q[q] : qv.min_sep);
        const double tmax = unif64(qv.t_max);
        const bool literal = (uni32(qv.flags) & kFlagLiteral) != 0;
        if (tid < 24) {
            const int c = tid % 3, k = tid / 3;
            sh.Xs[c * 8 + k] = qv.pos[(int64_t)tid * qv.n + q];
        }
        h.fmt = uni32(h.fmt);
        h.words = uni64(h.words);
        // the record's level into buffer 0 of the arena: keys and pairs as they
        // are, triples packed into keys when the depth sum allows it; a level-0
        // record is the root box alone
        int fmt = (int)(h.fmt & 3u), pa = (int)((h.fmt >> 4) & 3u);
        int64_t words = (int64_t)h.words;
        const uint64_t* rb = g.in_pool ? g.in_pool + rec[kRecordHeaderWords] : rec + kRecordHeaderWords;
        const Buf b0{(lds_u64*)group_lds, (hbm_u64*)base, nl};  // buffer 0, packed formats
        if (h.level == 0 || words > cap || fmt > kFmtTriple) {
            // (words > cap and unknown formats cannot come from the engines
            // before this one; restarting from the root is always correct)
            h.N = 0; h.tpend = INFINITY; h.wpend = 0.0; h.level = 0;
            h.d[0] = h.d[1] = h.d[2] = 0; h.cnt = 1;
            fmt = kFmtKey; pa = 0; words = 1;
            if (tid == 0) b0.put(0, 0);
        } else if (fmt == kFmtTriple && depth_sum(h.d) <= 64) {
            KeyCodec kc;
            kc.init(h.d[1], h.d[2]);
            for (int64_t i = tid; i < words; i += T)
                b0.put(i, kc.encode(rb[i], rb[words + i], rb[2 * words + i]));
            fmt = kFmtKey;
        } else if (fmt == kFmtTriple) {
            for (int64_t i = tid; i < words; i += T) {
                base[i] = rb[i];
                base[cap + i] = rb[words + i];
                base[2 * cap + i] = rb[2 * words + i];
            }
        } else {
            for (int64_t i = tid; i < words; i += T) b0.put(i, rb[i]);
        }
        __syncthreads();
        if (tid < 3) {
            // gamma_c and eps_c (Sec. 5.2); min_sep > 0 selects the Sec. 6.1 constants
            const double K = filter_constant(kind, min_sep);
            double gm = 1.0;
            for (int k = 0; k < 8; ++k) gm = fmax(gm, fabs(sh.Xs[tid * 8 + k]));
            if (a.gamma) gm = a.gamma[tid];  // scene-wide filter (checked at level 0)
            sh.Es[tid] = ((K * gm) * gm) * gm;
        }
        double kappa[3];
        if (kind == kEE) kappa_lds<kEE>(sh.Xs, kappa);
        else kappa_lds<kVF>(sh.Xs, kappa);
        for (int k = 0; k < 3; ++k) kappa[k] = unif64(kappa[k]);
        __syncthreads();
        if (kind == kEE)
            group_query<W, kEE>(a, g, sh, base, group_lds, nl, h, fmt, pa, words, kappa, delta,
                                min_sep, tmax, max_iter, literal, nchk[1], slots);
        else
            group_query<W, kVF>(a, g, sh, base, group_lds, nl, h, fmt, pa, words, kappa, delta,
                                min_sep, tmax, max_iter, literal, nchk[0], slots);
        __syncthreads();
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (nchk[k]) atomicAdd(&a.counters[kCntChecks + 2 * g.tier + k], (unsigned long long)nchk[k]);
        if (slots) atomicAdd(&a.counters[kCntSlots + g.tier], (unsigned long long)slots);
    }
}

// Explicit instantiations used by the runtime.
template __global__ void k_lane<false>(BatchArgs, LaneCfg);
template __global__ void k_lane<true>(BatchArgs, LaneCfg);
template __global__ void k_group<1, 1, false>(BatchArgs, GroupCfg);
template __global__ void k_group<1, 2, false>(BatchArgs, GroupCfg);
template __global__ void k_group<1, 3, false>(BatchArgs, GroupCfg);
template __global__ void k_group<1, 4, false>(BatchArgs, GroupCfg);
template __global__ void k_group<2, 1, false>(BatchArgs, GroupCfg);
template __global__ void k_group<4, 1, false>(BatchArgs, GroupCfg);
template __global__ void k_group<8, 1, false>(BatchArgs, GroupCfg);
template __global__ void k_group<1, 3, true>(BatchArgs, GroupCfg);
template __global__ void k_group<8, 1, true>(BatchArgs, GroupCfg);

}  // namespace ccd
