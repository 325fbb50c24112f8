// Device arithmetic of the inclusion-based CCD root finder (gfx950, binary64).
//
// Every function here is compiled with -ffp-contract=off: each operation below
// is one correctly rounded binary64 operation in the order written, so the
// values are reproducible bit for bit.  The evaluation order is the literal
// one of the paper's formulas:
//   p(t)  = (1-t) p0 + t p1                                 (Sec. 3)
//   F_ee  = ((1-u) p1 + u p2) - ((1-v) p3 + v p4)          (Sec. 3, eq. F-ee)
//   F_vf  = p - (((1-u-v) v1 + u v2) + v v3)                (Sec. 3, eq. F-vf)
// The complements 1-u and (1-u)-v are exact (u, v endpoints are dyadic with at
// most 52 fractional bits), and so is 1-t on the full time interval; on a
// shortened interval [0, t_max] the time values fl(t_max s) are not dyadic and
// 1-t is rounded once, which the static filter of Sec. 5.2 (derived for any
// inputs in [0,1]) still covers.
//
// Boxes are integer dyadic triples: on a level with per-axis bisection depths
// (dt, du, dv) the box (it, iu, iv) is
//   [it 2^-dt, (it+1) 2^-dt] x [iu 2^-du, (iu+1) 2^-du] x [iv 2^-dv, (iv+1) 2^-dv].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccd {

constexpr int kVF = 0;
constexpr int kEE = 1;
constexpr int kMaxDepth = 52;
constexpr double kCoordLimit = 1e300;

constexpr uint8_t kStCap = 0x01;
constexpr uint8_t kStCarry = 0x02;
constexpr uint8_t kStDepth = 0x04;
constexpr uint8_t kStOverflow = 0x08;
constexpr uint8_t kStInvalid = 0x80;
constexpr uint32_t kFlagLiteral = 0x1u;

// Filter constants of eq. ccd-error (d = 0) and eq. msccd-error (d > 0):
// 28, 30, 32 and 34 times 2^-52.
__device__ __forceinline__ double filter_constant(int kind, double min_sep) {
    if (min_sep > 0.0) return kind == kEE ? 0x1p-47 : 0x1.1p-47;
    return kind == kEE ? 0x1.cp-48 : 0x1.ep-48;
}

// gamma_c = max(1, max over the 8 points of |x^c|); eps_c = K gamma_c^3.
__device__ __forceinline__ void filter_eps(int kind, const double* X, double min_sep,
                                           double eps[3], double* gamma_min) {
    const double K = filter_constant(kind, min_sep);
    double gmin = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double g = 1.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) g = fmax(g, fabs(X[3 * k + c]));
        eps[c] = ((K * g) * g) * g;
        gmin = (c == 0) ? g : fmin(gmin, g);
    }
    *gamma_min = gmin;
}

// The 8 corner values of one coordinate of F over the box [t0,t1]x[u0,u1]x[v0,v1],
// from that coordinate of the 8 points: xc[k], points 0..3 at t = 0, 4..7 at
// t = 1.  f[(a<<2)|(b<<1)|e] = F(t_a, u_b, v_e).  Positions at t0 and t1 are
// shared between the corners (same bits as evaluating each corner on its own).
template <int KIND>
__device__ __forceinline__ void corner_values_axis(const double xc[8], double t0, double t1,
                                                   double u0, double u1, double v0, double v1,
                                                   double f[8]) {
    const double s0 = 1.0 - t0, s1 = 1.0 - t1;
    double P[2][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        P[0][k] = s0 * xc[k] + t0 * xc[k + 4];
        P[1][k] = s1 * xc[k] + t1 * xc[k + 4];
    }
    const double uu[2] = {u0, u1};
    const double vv[2] = {v0, v1};
    if (KIND == kEE) {
        const double cu[2] = {1.0 - u0, 1.0 - u1};
        const double cv[2] = {1.0 - v0, 1.0 - v1};
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            double ea[2], eb[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) ea[b] = cu[b] * P[a][0] + uu[b] * P[a][1];
#pragma unroll
            for (int e = 0; e < 2; ++e) eb[e] = cv[e] * P[a][2] + vv[e] * P[a][3];
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int e = 0; e < 2; ++e) f[(a << 2) | (b << 1) | e] = ea[b] - eb[e];
        }
    } else {
        double w[2][2];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 2; ++e) w[b][e] = (1.0 - uu[b]) - vv[e];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const double s12 = w[b][e] * P[a][1] + uu[b] * P[a][2];
                    const double face = s12 + vv[e] * P[a][3];
                    f[(a << 2) | (b << 1) | e] = P[a][0] - face;
                }
    }
}

// Coordinate c of F at the 8 corners, with the query as X[3k + c].
template <int KIND>
__device__ __forceinline__ void corner_values(const double* X, int c, double t0, double t1,
                                              double u0, double u1, double v0, double v1,
                                              double f[8]) {
    double xc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) xc[k] = X[3 * k + c];
    corner_values_axis<KIND>(xc, t0, t1, u0, u1, v0, v1, f);
}

struct CheckResult {
    bool collide;  // B (enlarged by d) meets the filter cube
    bool small;    // w(B) < delta, or B (enlarged by d) inside the filter cube
};

// Box check of Sec. 5.2 (eq. box, filter test) and Sec. 6.1 (enlargement by d).
// With want_kappa the box must be [0,1]^3 and kappa (eq. kappas) is produced
// from the same corner values.
template <int KIND>
__device__ __forceinline__ CheckResult box_check(const double* X, double t0, double t1, double u0,
                                                 double u1, double v0, double v1,
                                                 const double eps[3], double min_sep,
                                                 double delta, bool want_kappa,
                                                 double kappa[3]) {
    bool col = true, ins = true;
    double width = 0.0;
    double kt = 0.0, ku = 0.0, kv = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double f[8];
        corner_values<KIND>(X, c, t0, t1, u0, u1, v0, v1, f);
        double m = f[0], M = f[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) {
            m = fmin(m, f[i]);
            M = fmax(M, f[i]);
        }
        const double lo = m - min_sep;
        const double hi = M + min_sep;
        col = col && (lo <= eps[c]) && (hi >= -eps[c]);
        ins = ins && (lo >= -eps[c]) && (hi <= eps[c]);
        width = fmax(width, M - m);
        if (want_kappa) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                // j enumerates the two remaining corner coordinates of an edge
                const int jt = ((j >> 1) << 1) | (j & 1);              // (b, e)
                const int ju = ((j >> 1) << 2) | (j & 1);              // (a, e)
                const int jv = ((j >> 1) << 2) | ((j & 1) << 1);       // (a, b)
                kt = fmax(kt, fabs(f[jt] - f[4 | jt]));
                ku = fmax(ku, fabs(f[ju] - f[2 | ju]));
                kv = fmax(kv, fabs(f[jv] - f[1 | jv]));
            }
        }
    }
    if (want_kappa) {
        kappa[0] = 3.0 * kt;
        kappa[1] = 3.0 * ku;
        kappa[2] = 3.0 * kv;
    }
    CheckResult r;
    r.collide = col;
    r.small = (width < delta) || ins;
    return r;
}

// Alg. 2 SPLIT: c_x = w(I_x) kappa_x, split the largest, ties t > u > v.
__device__ __forceinline__ int split_axis(const double kappa[3], double wt, double wu, double wv) {
    const double ct = wt * kappa[0];
    const double cu = wu * kappa[1];
    const double cv = wv * kappa[2];
    const double c = fmax(ct, fmax(cu, cv));
    if (ct == c) return 0;
    if (cu == c) return 1;
    return 2;
}

// 2^-d for 0 <= d <= 60 (exact).
__device__ __forceinline__ double pow2neg(int d) { return __longlong_as_double((int64_t)(1023 - d) << 52); }

// i * 2^-d for 0 <= i < 2^52, 0 <= d <= 52, exactly: the bit pattern
// 2^(52-d) | i is the double 2^(52-d) + i 2^-d, and subtracting 2^(52-d)
// (same exponent, representable result) is exact.  bias = 2^(52-d).
__device__ __forceinline__ double dyadic(uint64_t i, int64_t bias_bits, double bias) {
    return __longlong_as_double(bias_bits | (int64_t)i) - bias;
}

// Lexicographic order of (t, u, v) box indices of one level.
__device__ __forceinline__ bool key_less(uint64_t at, uint64_t au, uint64_t av, uint64_t bt,
                                         uint64_t bu, uint64_t bv) {
    if (at != bt) return at < bt;
    if (au != bu) return au < bu;
    return av < bv;
}

// Prism test for vertex-face children (Alg. 2 text): keep a box iff
// u_lo + v_lo <= 1, decided exactly on the integers.
__device__ __forceinline__ bool vf_admit(uint64_t iu, int du, uint64_t iv, int dv) {
    const int D = du > dv ? du : dv;
    const uint64_t a = iu << (D - du);
    const uint64_t b = iv << (D - dv);
    return a + b <= (1ull << D);
}

// Scene-wide filter (Sec. 7: tolerances from the maximum over all the vertices
// of the scene): eps_c = K gamma_c^3 with the given gamma, valid for a query
// only if gamma_c is at least the query's own gamma_c (then the filter's bound
// covers it).  Returns false otherwise; gamma_min as filter_eps().
__device__ __forceinline__ bool filter_eps_scene(int kind, const double* X, double min_sep,
                                                 const double* gamma, double eps[3],
                                                 double* gamma_min) {
    const double K = filter_constant(kind, min_sep);
    bool ok = true;
    double gmin = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double g = 1.0;
#pragma unroll
        for (int k = 0; k < 8; ++k) g = fmax(g, fabs(X[3 * k + c]));
        const double s = gamma[c];
        ok = ok && (s >= g) && (s <= 1.7976931348623157e308);  // false for NaN
        eps[c] = ((K * s) * s) * s;
        gmin = (c == 0) ? s : fmin(gmin, s);
    }
    *gamma_min = gmin;
    return ok;
}

// Validation of a query (coordinates finite and bounded, parameters in range).
__device__ __forceinline__ bool query_valid(const double* X, double delta, int64_t max_iter,
                                            double min_sep, double gamma_min) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 24; ++i) ok = ok && (fabs(X[i]) <= kCoordLimit);  // false for NaN
    ok = ok && (delta > 0.0) && (delta <= 1.7976931348623157e308);
    ok = ok && (max_iter >= 1);
    ok = ok && (min_sep >= 0.0) && (min_sep < gamma_min);
    return ok;
}

}  // namespace ccd
