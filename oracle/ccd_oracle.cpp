// CPU oracle for the inclusion-based CCD root finder (Wang et al., "A Large Scale
// Benchmark and an Inclusion-Based Algorithm for Continuous Collision Detection",
// ACM TOG 40(5), 2021).
//
// TEST INFRASTRUCTURE ONLY. This file is the plain, slow, single-threaded
// reference that the GPU library is checked against. Only the test-suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it. It shares
// no source with the HIP library.
//
// Build: g++ -std=c++17 -O2 -ffp-contract=off -fPIC -shared (no fast-math): every
// arithmetic operation below is one IEEE-754 binary64 operation, rounded to
// nearest-even, in exactly the order written.
//
// Structure follows the paper:
//   * linear trajectories p(t) = (1-t) p0 + t p1                  (Sec. 3, Preliminaries)
//   * F_vf and F_ee                                               (Sec. 3, eqs. F-vf, F-ee)
//   * box inclusion B_F(I): AABB of F at the 8 corners of I        (Sec. 5.2, eq. box)
//   * floating-point filter eps = K * gamma^3                      (Sec. 5.2, eq. ccd-error)
//   * minimum-separation filter and enlarged box                   (Sec. 6.1, eq. msccd-error)
//   * kappa_t, kappa_u, kappa_v and the split rule                 (Sec. 5.2, eq. kappas; Alg. 2 SPLIT)
//   * SOLVE with a priority queue ordered by (level, t)            (Alg. 2)
//
// Readings where the paper is silent or ambiguous (each one also appears in the
// design notes of the repository):
//   * kappa is computed once per query from the level-0 corners (eq. kappas uses
//     u_i, v_j in {0,1}); hence every box of a level has the same widths.
//   * gamma_c is the max over the 8 input points of |x^c|, floored at 1.
//   * ties in ORDER are broken by u_lo then v_lo (ORDER compares only t).
//   * "carry" (default): a colliding box that meets the termination test but is
//     not the first colliding box of its level is remembered (t_pend) instead of
//     dropped; it is returned once no earlier candidate remains. The literal
//     mode drops it, exactly as Alg. 2 is printed.
//   * the m_I test sits where Alg. 2 puts it: inside the colliding branch.
//   * a split never goes below 2^-52 on an axis: a colliding box whose split axis
//     is already at depth 52 is treated as terminal, so every endpoint and every
//     complement 1-t, 1-u, (1-u)-v stays exact (1-t only while t_max = 1).
//   * n_checks is reported saturated at m_I.
//   * shortened time interval (Sec. 7.2, line search: only the initial I changes):
//     I_t = [0, t_max], 0 < t_max <= 1, bisected in the normalized coordinate
//     s = t / t_max; a box's time endpoints are fl(t_max * s) and its width is
//     w(I_t) = t_max * w(I_s) (exact).  kappa keeps eq. kappas (corners at
//     t = 0 and t = 1: a per-unit slope).  ORDER compares s, which orders like t.
//   * scene-wide filter (Sec. 7: eps from the maximum over all the vertices of
//     the scene): an optional gamma per axis replaces the query's own; it must
//     be at least the query's gamma (else the filter's bound does not cover the
//     query, which is then invalid), and d < min_c gamma_c uses it.
#include <cmath>
#include <cstdint>
#include <queue>
#include <vector>

extern "C" {

// One result of SOLVE. box/level/depth describe the box whose t_lo was returned
// (debug output used by the tests' accuracy checks).
struct oracle_result {
    double toi;          // +inf when no collision
    double t_width;      // w(I_t) of the returned level, 0 when no collision
    uint64_t n_checks;   // number of box checks, saturated at m_I
    uint64_t n_raw;      // number of box checks, not saturated
    uint8_t hit;         // toi <= 1
    uint8_t status;      // ORACLE_ST_* bits
    uint8_t pad[6];
    double box[6];       // t_lo, t_hi, u_lo, u_hi, v_lo, v_hi of the returned box (time
                         // endpoints normalized: t / t_max)
    int32_t level;
    int32_t depth[3];
};

enum { ORACLE_VF = 0, ORACLE_EE = 1 };
enum { ORACLE_ST_CAP = 1, ORACLE_ST_CARRY = 2, ORACLE_ST_DEPTH = 4 };
enum { ORACLE_OK = 0, ORACLE_EINVAL = -1 };

static const int kMaxDepth = 52;
static const double kCoordLimit = 1e300;

// ---------------------------------------------------------------------------
// Sec. 3: p(t) = (1-t) p^0 + t p^1. X[3k+c] is coordinate c of point k; points
// 0..3 are at t^0 and points 4..7 are the same vertices at t^1.
static double position(const double X[24], int k, int c, double t) {
    double s = 1.0 - t;
    double a = s * X[3 * k + c];
    double b = t * X[3 * (k + 4) + c];
    return a + b;
}

// Sec. 3, eq. F-vf: F = p(t) - ((1-u-v) v1(t) + u v2(t) + v v3(t)), points 0..3
// are p, v1, v2, v3.  eq. F-ee: F = ((1-u) p1(t) + u p2(t)) - ((1-v) p3(t) + v p4(t)),
// points 0..3 are p1, p2, p3, p4.
int oracle_F(int kind, const double X[24], double t, double u, double v, double out[3]) {
    for (int c = 0; c < 3; ++c) {
        double P0 = position(X, 0, c, t);
        double P1 = position(X, 1, c, t);
        double P2 = position(X, 2, c, t);
        double P3 = position(X, 3, c, t);
        if (kind == ORACLE_EE) {
            double ea = (1.0 - u) * P0;
            double eb = u * P1;
            double edge_a = ea + eb;
            double ec = (1.0 - v) * P2;
            double ed = v * P3;
            double edge_b = ec + ed;
            out[c] = edge_a - edge_b;
        } else {
            double w = (1.0 - u) - v;
            double s1 = w * P1;
            double s2 = u * P2;
            double s12 = s1 + s2;
            double s3 = v * P3;
            double on_face = s12 + s3;
            out[c] = P0 - on_face;
        }
    }
    return ORACLE_OK;
}

// Sec. 5.2 eq. ccd-error and Sec. 6.1 eq. msccd-error: eps_c = K gamma_c^3 with
// gamma_c = max(x_max, 1). The paper prints K in decimal; the values are the
// exact binary numbers 28, 30, 32 and 34 times 2^-52.
void oracle_filter(int kind, const double X[24], double min_sep, double eps[3]) {
    double K;
    if (min_sep > 0.0) K = (kind == ORACLE_EE) ? 0x1p-47 : 0x1.1p-47;     // 32, 34 * 2^-52
    else               K = (kind == ORACLE_EE) ? 0x1.cp-48 : 0x1.ep-48;   // 28, 30 * 2^-52
    for (int c = 0; c < 3; ++c) {
        double g = 1.0;
        for (int k = 0; k < 8; ++k) {
            double a = std::fabs(X[3 * k + c]);
            if (a > g) g = a;
        }
        eps[c] = ((K * g) * g) * g;
    }
}

// eq. ccd-error / eq. msccd-error with a given gamma per axis.
void oracle_filter_gamma(int kind, const double gamma[3], double min_sep, double eps[3]) {
    double K;
    if (min_sep > 0.0) K = (kind == ORACLE_EE) ? 0x1p-47 : 0x1.1p-47;
    else               K = (kind == ORACLE_EE) ? 0x1.cp-48 : 0x1.ep-48;
    for (int c = 0; c < 3; ++c) eps[c] = ((K * gamma[c]) * gamma[c]) * gamma[c];
}

static double gamma_min(const double X[24]) {
    double gmin = INFINITY;
    for (int c = 0; c < 3; ++c) {
        double g = 1.0;
        for (int k = 0; k < 8; ++k) {
            double a = std::fabs(X[3 * k + c]);
            if (a > g) g = a;
        }
        if (g < gmin) gmin = g;
    }
    return gmin;
}

// Sec. 5.2 eq. kappas, with u_i, v_j, t_i ranging over {0, 1}:
//   kappa_t = 3 max ||F(0,u,v) - F(1,u,v)||_inf, and likewise for u and v.
void oracle_kappa(int kind, const double X[24], double kappa[3]) {
    double Fc[2][2][2][3];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e)
                oracle_F(kind, X, (double)a, (double)b, (double)e, Fc[a][b][e]);
    double mt = 0.0, mu = 0.0, mv = 0.0;
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int c = 0; c < 3; ++c) {
                double dt = std::fabs(Fc[0][i][j][c] - Fc[1][i][j][c]);
                double du = std::fabs(Fc[i][0][j][c] - Fc[i][1][j][c]);
                double dv = std::fabs(Fc[i][j][0][c] - Fc[i][j][1][c]);
                if (dt > mt) mt = dt;
                if (du > mu) mu = du;
                if (dv > mv) mv = dv;
            }
    kappa[0] = 3.0 * mt;
    kappa[1] = 3.0 * mu;
    kappa[2] = 3.0 * mv;
}

// Alg. 2, SPLIT: c_x = w(I_x) kappa_x; the axis with the largest c is split,
// ties going to t, then u, then v. Returns 0 (t), 1 (u) or 2 (v).
int oracle_split_axis(const double kappa[3], const double width[3]) {
    double ct = width[0] * kappa[0];
    double cu = width[1] * kappa[1];
    double cv = width[2] * kappa[2];
    double c = ct;
    if (cu > c) c = cu;
    if (cv > c) c = cv;
    if (ct == c) return 0;
    if (cu == c) return 1;
    return 2;
}

// Sec. 5.2 eq. box plus the filter test, and Sec. 6.1 for d > 0.
//   box = {t_lo, t_hi, u_lo, u_hi, v_lo, v_hi}
//   collide: B enlarged by d meets C_eps;  inside: B enlarged by d lies in C_eps;
//   width: w(B) of the un-enlarged box.
void oracle_box_check(int kind, const double X[24], const double box[6], const double eps[3],
                      double min_sep, int* collide, int* inside, double* width,
                      double lo[3], double hi[3]) {
    double m[3] = {INFINITY, INFINITY, INFINITY};
    double M[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int e = 0; e < 2; ++e) {
                double f[3];
                oracle_F(kind, X, box[a], box[2 + b], box[4 + e], f);
                for (int c = 0; c < 3; ++c) {
                    if (f[c] < m[c]) m[c] = f[c];
                    if (f[c] > M[c]) M[c] = f[c];
                }
            }
    int col = 1, ins = 1;
    double w = 0.0;
    for (int c = 0; c < 3; ++c) {
        double lo_d = m[c] - min_sep;
        double hi_d = M[c] + min_sep;
        if (!(lo_d <= eps[c] && hi_d >= -eps[c])) col = 0;
        if (!(lo_d >= -eps[c] && hi_d <= eps[c])) ins = 0;
        double wc = M[c] - m[c];
        if (wc > w) w = wc;
        if (lo) lo[c] = m[c];
        if (hi) hi[c] = M[c];
    }
    *collide = col;
    *inside = ins;
    *width = w;
}

int oracle_validate(const double X[24], double delta, int64_t max_iter, double min_sep) {
    for (int i = 0; i < 24; ++i)
        if (!std::isfinite(X[i]) || std::fabs(X[i]) > kCoordLimit) return ORACLE_EINVAL;
    if (!(delta > 0.0) || !std::isfinite(delta)) return ORACLE_EINVAL;
    if (max_iter < 1) return ORACLE_EINVAL;
    if (!(min_sep >= 0.0) || !std::isfinite(min_sep)) return ORACLE_EINVAL;
    if (!(min_sep < gamma_min(X))) return ORACLE_EINVAL;   // Sec. 6.1: d < gamma
    return ORACLE_OK;
}

// ---------------------------------------------------------------------------
// Alg. 2. Boxes carry their level and per-axis bisection depth.
struct Box {
    double t[2], u[2], v[2];
    int level;
    int depth[3];
};

// ORDER: level first, then t_lo (then u_lo, v_lo). std::priority_queue pops the
// largest element, so "a comes after b" is the comparison.
struct After {
    bool operator()(const Box& a, const Box& b) const {
        if (a.level != b.level) return a.level > b.level;
        if (a.t[0] != b.t[0]) return a.t[0] > b.t[0];
        if (a.u[0] != b.u[0]) return a.u[0] > b.u[0];
        return a.v[0] > b.v[0];
    }
};

static void fill_result(oracle_result* out, double toi, double tw, uint64_t n, int64_t max_iter,
                        uint8_t status, const Box* b) {
    out->toi = toi;
    out->t_width = tw;
    out->n_raw = n;
    out->n_checks = (n > (uint64_t)max_iter) ? (uint64_t)max_iter : n;
    out->hit = (toi <= 1.0) ? 1 : 0;
    out->status = status;
    for (int i = 0; i < 6; ++i) out->pad[i] = 0;
    if (b) {
        out->box[0] = b->t[0]; out->box[1] = b->t[1];
        out->box[2] = b->u[0]; out->box[3] = b->u[1];
        out->box[4] = b->v[0]; out->box[5] = b->v[1];
        out->level = b->level;
        for (int i = 0; i < 3; ++i) out->depth[i] = b->depth[i];
    } else {
        for (int i = 0; i < 6; ++i) out->box[i] = NAN;
        out->level = -1;
        out->depth[0] = out->depth[1] = out->depth[2] = -1;
    }
}

// Alg. 2 on I = [0, t_max] x [0,1]^2.  Box.t holds the normalized time
// interval (s); time values are fl(t_max * s).  gamma: scene-wide gamma per
// axis, or NULL for the query's own.
int oracle_solve_full(int kind, const double X[24], double delta, int64_t max_iter,
                      double min_sep, double t_max, const double* gamma, int literal,
                      oracle_result* out) {
    if (kind != ORACLE_VF && kind != ORACLE_EE) return ORACLE_EINVAL;
    if (!(t_max > 0.0 && t_max <= 1.0)) return ORACLE_EINVAL;
    double eps[3], kappa[3];
    if (gamma) {
        // the query's own validity with min_sep checked against the scene gamma
        if (oracle_validate(X, delta, max_iter, 0.0) != ORACLE_OK) return ORACLE_EINVAL;
        if (!(min_sep >= 0.0) || !std::isfinite(min_sep)) return ORACLE_EINVAL;
        double gmin = INFINITY;
        for (int c = 0; c < 3; ++c) {
            if (!std::isfinite(gamma[c])) return ORACLE_EINVAL;
            double g = 1.0;
            for (int k = 0; k < 8; ++k) {
                double a = std::fabs(X[3 * k + c]);
                if (a > g) g = a;
            }
            if (!(gamma[c] >= g)) return ORACLE_EINVAL;
            if (gamma[c] < gmin) gmin = gamma[c];
        }
        if (!(min_sep < gmin)) return ORACLE_EINVAL;
        oracle_filter_gamma(kind, gamma, min_sep, eps);
    } else {
        if (oracle_validate(X, delta, max_iter, min_sep) != ORACLE_OK) return ORACLE_EINVAL;
        oracle_filter(kind, X, min_sep, eps);
    }
    oracle_kappa(kind, X, kappa);

    std::priority_queue<Box, std::vector<Box>, After> Q;
    Box root = {{0.0, 1.0}, {0.0, 1.0}, {0.0, 1.0}, 0, {0, 0, 0}};
    Q.push(root);

    uint64_t n = 0;
    int lp = -1;
    Box If = root;
    double t_pend = INFINITY, w_pend = 0.0;
    Box pend_box = root;

    while (!Q.empty()) {
        Box I = Q.top();
        Q.pop();
        const double t_lo = t_max * I.t[0];
        double box[6] = {t_lo, t_max * I.t[1], I.u[0], I.u[1], I.v[0], I.v[1]};
        int collide, inside;
        double width;
        oracle_box_check(kind, X, box, eps, min_sep, &collide, &inside, &width, nullptr, nullptr);
        n = n + 1;
        if (!collide) continue;

        bool first = (I.level != lp);
        double w_t = t_max * (I.t[1] - I.t[0]);
        if (first) {
            If = I;
            if (!literal && t_pend <= t_lo) {
                fill_result(out, t_pend, w_pend, n, max_iter, ORACLE_ST_CARRY, &pend_box);
                return ORACLE_OK;
            }
        }
        if (n >= (uint64_t)max_iter) {
            fill_result(out, t_max * If.t[0], w_t, n, max_iter, ORACLE_ST_CAP, &If);
            return ORACLE_OK;
        }

        double widths[3] = {w_t, I.u[1] - I.u[0], I.v[1] - I.v[0]};
        int axis = oracle_split_axis(kappa, widths);
        bool depth_capped = I.depth[axis] >= kMaxDepth;
        bool small = (width < delta) || inside;
        if (small || depth_capped) {
            if (first) {
                uint8_t st = small ? 0 : ORACLE_ST_DEPTH;
                fill_result(out, t_lo, w_t, n, max_iter, st, &I);
                return ORACLE_OK;
            }
            if (!literal && t_lo < t_pend) {
                t_pend = t_lo;
                w_pend = w_t;
                pend_box = I;
            }
        } else {
            Box c0 = I, c1 = I;
            c0.level = c1.level = I.level + 1;
            c0.depth[axis] = c1.depth[axis] = I.depth[axis] + 1;
            double* lo0; double* hi0; double* lo1;
            if (axis == 0)      { lo0 = &c0.t[0]; hi0 = &c0.t[1]; lo1 = &c1.t[0]; }
            else if (axis == 1) { lo0 = &c0.u[0]; hi0 = &c0.u[1]; lo1 = &c1.u[0]; }
            else                { lo0 = &c0.v[0]; hi0 = &c0.v[1]; lo1 = &c1.v[0]; }
            double mid = (*lo0 + *hi0) / 2.0;
            *hi0 = mid;
            *lo1 = mid;
            // Alg. 2 text: for vertex-face the domain is the prism u+v <= 1, and a
            // child is queued only if it meets it.
            if (kind == ORACLE_EE || c0.u[0] + c0.v[0] <= 1.0) Q.push(c0);
            if (kind == ORACLE_EE || c1.u[0] + c1.v[0] <= 1.0) Q.push(c1);
        }
        lp = I.level;
    }
    if (!literal && t_pend < INFINITY) {
        fill_result(out, t_pend, w_pend, n, max_iter, ORACLE_ST_CARRY, &pend_box);
        return ORACLE_OK;
    }
    fill_result(out, INFINITY, 0.0, n, max_iter, 0, nullptr);
    return ORACLE_OK;
}

int oracle_solve_tmax(int kind, const double X[24], double delta, int64_t max_iter,
                      double min_sep, double t_max, int literal, oracle_result* out) {
    return oracle_solve_full(kind, X, delta, max_iter, min_sep, t_max, nullptr, literal, out);
}

int oracle_solve(int kind, const double X[24], double delta, int64_t max_iter, double min_sep,
                 int literal, oracle_result* out) {
    return oracle_solve_full(kind, X, delta, max_iter, min_sep, 1.0, nullptr, literal, out);
}

// Batch driver over the structure-of-arrays layout pos[(3k+c)*n + q]. Per-query
// parameters are optional (NULL selects the scalar value). Returns the number of
// invalid queries (their status is 0xFF, toi NaN).
int64_t oracle_solve_batch(int64_t n, const double* pos, const uint8_t* kind, int default_kind,
                           const double* delta_q, double delta, const int64_t* max_iter_q,
                           int64_t max_iter, const double* min_sep_q, double min_sep, double t_max,
                           const double* gamma, int literal, double* toi, double* t_width,
                           uint8_t* hit, uint64_t* n_checks, uint8_t* status) {
    int64_t bad = 0;
    for (int64_t q = 0; q < n; ++q) {
        double X[24];
        for (int r = 0; r < 24; ++r) X[r] = pos[(int64_t)r * n + q];
        int k = kind ? kind[q] : default_kind;
        double dl = delta_q ? delta_q[q] : delta;
        int64_t mi = max_iter_q ? max_iter_q[q] : max_iter;
        double ms = min_sep_q ? min_sep_q[q] : min_sep;
        oracle_result r;
        if (oracle_solve_full(k, X, dl, mi, ms, t_max, gamma, literal, &r) != ORACLE_OK) {
            ++bad;
            toi[q] = NAN; t_width[q] = NAN; hit[q] = 0; n_checks[q] = 0; status[q] = 0xFF;
            continue;
        }
        toi[q] = r.toi;
        t_width[q] = r.t_width;
        hit[q] = r.hit;
        n_checks[q] = r.n_checks;
        status[q] = r.status;
    }
    return bad;
}

}  // extern "C"
