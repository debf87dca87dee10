// Edge compiler.
//
// The counting rule bins a pair by theta = acos(clamp(d, -1, 1)) against the
// edges e_k (paper, Section 3: angle from the dot product and arc-cosine;
// Section 2: results in theta space).  acos is non-increasing, so
//     theta >= e_k   <=>   clamp(d) <= D_k,
// with D_k the largest double in [-1, 1] whose acos is still >= e_k.  D_k is
// found here by bisection over the ordered doubles in [-1, 1], calling the
// same host libm acos that defines the rule, so the GPU never evaluates acos
// and still reproduces the rule bit for bit.  A window of doubles around
// each D_k is then checked exhaustively: every d below D_k must give
// acos(d) >= e_k and every d above must not.  The window is sized so that it
// covers every d whose exact arc-cosine lies within a few ulps of e_k; outside
// it a libm result within 1 ulp cannot reach e_k from the wrong side.
//
// This file must keep sin, cos and acos as plain libm calls (built with
// -fno-builtin and contraction off).
#include "edges.h"

#include <math.h>
#include <string.h>

#include <algorithm>
#include <cstdio>

namespace tpcf {

namespace {

inline int64_t okey(double d) {
    int64_t b;
    memcpy(&b, &d, 8);
    return b >= 0 ? b : -(b & 0x7fffffffffffffffLL);
}

inline double from_okey(int64_t k) {
    int64_t b = k >= 0 ? k : ((-k) | (int64_t)0x8000000000000000ULL);
    double d;
    memcpy(&d, &b, 8);
    return d;
}

inline bool reaches(double d, double e) { return acos(d) >= e; }

// Largest double d in [-1, 1] with acos(d) >= e, assuming acos is
// non-increasing; +inf / -inf for the two degenerate cases.
double threshold_of(double e) {
    if (!(e > 0.0))
        return HUGE_VAL;                       // theta >= 0 always
    if (!reaches(-1.0, e))
        return -HUGE_VAL;                      // no angle reaches e
    int64_t lo = okey(-1.0), hi = okey(1.0);   // reaches(lo) true, reaches(hi) false
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (reaches(from_okey(mid), e))
            lo = mid;
        else
            hi = mid;
    }
    return from_okey(lo);
}

// Half-width, in doubles, of the window checked around D (see above).
int64_t window_of(double e, double D) {
    double ulp_e = nextafter(e, HUGE_VAL) - e;
    double span = 8.0 * ulp_e * sin(e) + 1e-300;          // |d - D| that can matter
    double ulp_d = nextafter(fabs(D), HUGE_VAL) - fabs(D);
    double w = ulp_d > 0 ? span / ulp_d : 1e30;
    if (w > (double)(1 << 16))
        w = (double)(1 << 16);
    return (int64_t)w + 64;
}

bool verify_threshold(double e, double D, std::string *why) {
    if (isinf(D))
        return true;
    const int64_t w = window_of(e, D);
    const int64_t k = okey(D);
    const int64_t kmin = okey(-1.0), kmax = okey(1.0);
    for (int64_t t = std::max(kmin, k - w); t <= k; ++t) {
        if (!reaches(from_okey(t), e)) {
            char buf[160];
            snprintf(buf, sizeof buf, "acos not monotone below threshold %.17g for edge %.17g rad", D, e);
            *why = buf;
            return false;
        }
    }
    for (int64_t t = k + 1; t <= std::min(kmax, k + w); ++t) {
        if (reaches(from_okey(t), e)) {
            char buf[160];
            snprintf(buf, sizeof buf, "acos not monotone above threshold %.17g for edge %.17g rad", D, e);
            *why = buf;
            return false;
        }
    }
    return true;
}

inline float round_up32(double x) {
    float f = (float)x;
    if ((double)f < x)
        f = nextafterf(f, HUGE_VALF);
    return f;
}

inline float round_down32(double x) {
    float f = (float)x;
    if ((double)f > x)
        f = nextafterf(f, -HUGE_VALF);
    return f;
}

inline uint32_t fbits(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

inline float ffrom(uint32_t b) {
    float f;
    memcpy(&f, &b, 4);
    return f;
}

inline int32_t dhi(double d) {
    uint64_t b;
    memcpy(&b, &d, 8);
    return (int32_t)(uint32_t)(b >> 32);
}

inline double dfrom(uint64_t b) {
    double d;
    memcpy(&d, &b, 8);
    return d;
}

uint16_t encode(int s_min, int s_max) {
    if (s_min == s_max)
        return (uint16_t)s_min;
    if (s_max == s_min + 1)
        return (uint16_t)(0x8000 | s_min);
    return 0xFFFF;
}

void tally(CellTable *t) {
    t->n_certain = t->n_medium = t->n_multi = 0;
    for (uint16_t c : t->cells) {
        if (c == 0xFFFF)
            ++t->n_multi;
        else if (c & 0x8000)
            ++t->n_medium;
        else
            ++t->n_certain;
    }
}

}  // namespace

bool compile_edges(const double *edges_deg, int nbins, EdgeTables *out, std::string *err) {
    if (nbins < 1 || nbins > 256) {
        *err = "nbins must be in [1, 256]";
        return false;
    }
    if (!edges_deg) {
        *err = "bin_edges_deg is NULL";
        return false;
    }
    for (int k = 0; k <= nbins; ++k) {
        double v = edges_deg[k];
        if (!isfinite(v) || v < 0.0 || v > 180.0) {
            *err = "bin edges must be finite and within [0, 180] degrees";
            return false;
        }
        if (k > 0 && !(v > edges_deg[k - 1])) {
            *err = "bin edges must be strictly increasing";
            return false;
        }
    }
    const double deg = M_PI / 180.0;
    EdgeTables t;
    t.nbins = nbins;
    t.edge_rad.resize(nbins + 1);
    t.D.resize(nbins + 1);
    t.E.resize(nbins + 1);
    for (int k = 0; k <= nbins; ++k) {
        double e = edges_deg[k] * deg;
        t.edge_rad[k] = e;
        double D = threshold_of(e);
        std::string why;
        if (!verify_threshold(e, D, &why)) {
            *err = why;
            return false;
        }
        t.D[k] = D;
        if (D == HUGE_VAL)
            t.E[k] = -HUGE_VAL;
        else if (D == -HUGE_VAL)
            t.E[k] = HUGE_VAL;
        else
            t.E[k] = 1.0 - D;
    }
    *out = std::move(t);
    return true;
}

// Band of edge k.  Let v be the FP64 master vectors (| |v|^2 - 1 | <= delta),
// f = fl32(v) their FP32 copies, c_v = |v_i - v_j|, c_f = |f_i - f_j|.
//  * d, the counting rule's FP64 dot, is within eps_d = gamma_3 (1 + delta)
//    of v_i . v_j (recursive summation of 3 products), and
//    v_i . v_j = (|v_i|^2 + |v_j|^2 - c_v^2) / 2, so
//      c_v^2 >= 2(1 - D_k) + 2(delta + eps_d)  =>  d <= D_k,
//      c_v^2 <  2(1 - D_k) - 2(delta + eps_d)  =>  d >  D_k.
//  * |f - v| <= u |v| per vector (u = 2^-24), so |c_f - c_v| <= a = 2u(1 + delta).
//  * the kernel's q = fl(fma(dz, dz, fma(dy, dy, dx*dx))) with dx = fl(fx_i - fx_j)
//    etc. (or the same with separate multiply and add) satisfies
//    (1-u)^5 c_f^2 - tau <= q <= (1+u)^5 c_f^2 + tau (every term is
//    non-negative; tau covers gradual or flushed underflow).
//  Hence q >= qhi_k => d <= D_k and q < qlo_k => d > D_k with
//      qhi_k = RU32(((C+ + a)^2 (1+u)^5 + tau) s),
//      qlo_k = RD32((((C- - a)_+)^2 (1-u)^5 - tau) / s),
//  C+- = sqrt(2(1 - D_k) +- 2(delta + eps_d)), and s = 1 + 2^-20 absorbing
//  the rounding of this host arithmetic (a few ulps of FP64).
Band32 make_band32(const EdgeTables &t, double delta, float q0) {
    const double U = ldexp(1.0, -53), u = ldexp(1.0, -24);
    const double eps_d = 3.0 * U / (1.0 - 3.0 * U) * (1.0 + delta);
    const double a = 2.0 * u * (1.0 + delta);
    // with a floor the chord term may see six roundings (a separate multiply
    // and add in place of the first fused step), the floor three
    const double grow = pow(1.0 + u, q0 > 0.0f ? 6.0 : 5.0), shrink = pow(1.0 - u, q0 > 0.0f ? 6.0 : 5.0);
    const double fgrow = (double)q0 * pow(1.0 + u, 3.0), fshrink = (double)q0 * pow(1.0 - u, 3.0);
    const double tau = ldexp(1.0, -120);
    const double s = 1.0 + ldexp(1.0, -20);
    const double slack = 2.0 * (delta + eps_d);
    Band32 b;
    b.delta = delta;
    b.q0 = q0;
    const int ne = (int)t.D.size();
    b.qlo.resize(ne);
    b.qhi.resize(ne);
    for (int k = 0; k < ne; ++k) {
        double D = t.D[k];
        if (D == HUGE_VAL) {
            b.qlo[k] = b.qhi[k] = -HUGE_VALF;
            continue;
        }
        if (D == -HUGE_VAL) {
            b.qlo[k] = b.qhi[k] = HUGE_VALF;
            continue;
        }
        double base = 2.0 * (1.0 - D);
        double cp = sqrt(base + slack);
        b.qhi[k] = round_up32(((cp + a) * (cp + a) * grow + fgrow + tau) * s);
        double tm = base - slack;
        if (tm <= 0.0) {
            b.qlo[k] = 0.0f;
        } else {
            double cm = sqrt(tm) - a;
            if (cm <= 0.0) {
                b.qlo[k] = 0.0f;
            } else {
                double v = (cm * cm * shrink + fshrink - tau) / s;
                b.qlo[k] = v > 0.0 ? round_down32(v) : 0.0f;
            }
        }
    }
    return b;
}

// Dot product of the FP32 copies.  With u = 2^-24 and U = 2^-53:
//  * |p - f_i . f_j| <= gamma_3(u) |f_i| |f_j| <= gamma_3(u) (1 + u)^2 (1 + delta)
//    (three roundings, fused or not; Cauchy-Schwarz for the sum of the
//    absolute products);
//  * |f_i . f_j - v_i . v_j| <= (2u + u^2)(1 + delta) (|f - v| <= u |v|);
//  * |d - v_i . v_j| <= gamma_3(U)(1 + delta) (the rule's own sum);
//  * 3 * 2^-126 for FP32 underflow in the products.
// The sum, widened by 2^-20 for this function's own rounding, bounds |p - d|.
double dot_error32(double delta) {
    const double u = ldexp(1.0, -24), U = ldexp(1.0, -53);
    const double g3 = 3.0 * u / (1.0 - 3.0 * u), G3 = 3.0 * U / (1.0 - 3.0 * U);
    return (g3 * (1.0 + u) * (1.0 + u) * (1.0 + delta) + (2.0 * u + u * u) * (1.0 + delta) + G3 * (1.0 + delta) +
            3.0 * ldexp(1.0, -126)) *
           (1.0 + ldexp(1.0, -20));
}

// The key q' = fl(2 - 2p): 2p is exact and the FMA rounds 2 - 2p once, with a
// relative error of at most u (no underflow: 2 - 2p is 0 or at least 2^-23
// for p near 1, and near 2 for tiny p).  With x = 2 - 2p and E = dot_error32:
//  * q' >= qhi_k with qhi_k >= 2 (1 - D_k + E)(1 + u) gives
//    x >= q'/(1 + u) >= 2 (1 - D_k + E), so p <= D_k - E and d <= D_k;
//  * q' < qlo_k with qlo_k <= 2 (1 - D_k - E)(1 - u) gives (q' >= 0)
//    x <= q'/(1 - u) < 2 (1 - D_k - E), so p > D_k + E and d > D_k.
// The kernel replaces a negative q' (x < 0, p > 1) by +0: a positive qlo_k
// means D_k + E < 1 < p, so q' = 0 < qlo_k is still right, and qhi_k > 0 for
// every finite D_k (D_k <= 1), so 0 never reaches it.  s = 1 + 2^-20 covers
// the rounding of 1 - D_k here.
Band32 make_band_dot32(const EdgeTables &t, double delta) {
    const double u = ldexp(1.0, -24), E = dot_error32(delta), s = 1.0 + ldexp(1.0, -20);
    Band32 b;
    b.delta = delta;
    const int ne = (int)t.D.size();
    b.qlo.resize(ne);
    b.qhi.resize(ne);
    for (int k = 0; k < ne; ++k) {
        const double D = t.D[k];
        if (D == HUGE_VAL) {
            b.qlo[k] = b.qhi[k] = -HUGE_VALF;
            continue;
        }
        if (D == -HUGE_VAL) {
            b.qlo[k] = b.qhi[k] = HUGE_VALF;
            continue;
        }
        b.qhi[k] = round_up32(2.0 * (1.0 - D + E) * (1.0 + u) * s);
        const double lo = 2.0 * (1.0 - D - E) * (1.0 - u) / s;
        b.qlo[k] = lo > 0.0 ? round_down32(lo) : 0.0f;
    }
    return b;
}

uint32_t dot_top_key(double delta) {
    // |p| <= (1 + delta)(1 + E'): q' <= 4 (1 + delta) + a few ulps
    return fbits(round_up32(4.0 * (1.0 + delta) * (1.0 + ldexp(1.0, -18))));
}

// p <= D_k - E gives d <= D_k and p > D_k + E gives d > D_k; the bounds are
// widened by s = 1 + 2^-20 (covering the FP64 rounding of D_k +- E s, which
// is far below E (s - 1)) and rounded outward to floats.
void make_pband32(const EdgeTables &t, double delta, std::vector<float> *plo, std::vector<float> *phi) {
    const double E = dot_error32(delta) * (1.0 + ldexp(1.0, -20));
    const int ne = (int)t.D.size();
    plo->resize(ne);
    phi->resize(ne);
    for (int k = 0; k < ne; ++k) {
        const double D = t.D[k];
        if (D == HUGE_VAL || D == -HUGE_VAL) {
            (*plo)[k] = (*phi)[k] = D == HUGE_VAL ? HUGE_VALF : -HUGE_VALF;
            continue;
        }
        (*plo)[k] = round_down32(D - E);
        (*phi)[k] = round_up32(D + E);
    }
}

// 3-D edges.  The counting rule bins a pair by r = sqrt(r2), r2 the FP64
// sum (dx^2 + dy^2) + dz^2 of the coordinate differences.  sqrt is
// non-decreasing (and correctly rounded), so r >= e_k <=> r2 >= S_k with S_k
// the smallest double whose square root is >= e_k, found by bisection over the
// ordered non-negative doubles with the same libm sqrt.  A window of doubles
// around S_k is checked exhaustively.
namespace {

inline bool reaches3(double s, double e) { return sqrt(s) >= e; }

double threshold3_of(double e) {
    int64_t lo = okey(0.0), hi = okey(1e300);    // reaches3(lo) false (e > 0), reaches3(hi) true
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        if (reaches3(from_okey(mid), e))
            hi = mid;
        else
            lo = mid;
    }
    return from_okey(hi);
}

bool verify_threshold3(double e, double S, std::string *why) {
    const int64_t k = okey(S);
    for (int64_t t = std::max(okey(0.0), k - 256); t <= k + 256; ++t) {
        if (reaches3(from_okey(t), e) != (t >= k)) {
            char buf[160];
            snprintf(buf, sizeof buf, "sqrt not monotone around threshold %.17g for edge %.17g", S, e);
            *why = buf;
            return false;
        }
    }
    return true;
}

}  // namespace

bool compile_edges_3d(const double *edges, int nbins, EdgeTables *out, std::string *err) {
    if (nbins < 1 || nbins > 256) {
        *err = "nbins must be in [1, 256]";
        return false;
    }
    if (!edges) {
        *err = "bin edges are NULL";
        return false;
    }
    for (int k = 0; k <= nbins; ++k) {
        double v = edges[k];
        if (!isfinite(v) || v < 0.0 || v > 1e150) {
            *err = "3-D bin edges must be finite and within [0, 1e150]";
            return false;
        }
        if (k > 0 && !(v > edges[k - 1])) {
            *err = "bin edges must be strictly increasing";
            return false;
        }
    }
    EdgeTables t;
    t.nbins = nbins;
    t.metric = 1;
    t.edge_rad.assign(edges, edges + nbins + 1);
    t.D.resize(nbins + 1);
    t.E.resize(nbins + 1);
    for (int k = 0; k <= nbins; ++k) {
        const double e = edges[k];
        if (!(e > 0.0)) {              // every distance reaches 0
            t.D[k] = HUGE_VAL;
            t.E[k] = -HUGE_VAL;
            continue;
        }
        const double S = threshold3_of(e);
        std::string why;
        if (!verify_threshold3(e, S, &why)) {
            *err = why;
            return false;
        }
        t.D[k] = -S;
        t.E[k] = S;
    }
    *out = std::move(t);
    return true;
}

// Band of 3-D edge k for points v (FP64, |v| <= R) and their FP32 copies f.
//  * The rule's r2 is within the factors (1 -+ U)^5 of c_v^2 = |v_i - v_j|^2
//    (U = 2^-53: one rounding for each difference, counted twice in the
//    square, the square and the two additions; every term is non-negative),
//    plus tau64 for gradual underflow.  So
//      c_v >= C+ = sqrt((S_k + tau64) / (1 - U)^5)  =>  r2 >= S_k,
//      c_v <  C- = sqrt((S_k - tau64)_+ / (1 + U)^5) =>  r2 <  S_k.
//  * |f - v| <= u |v| + 2^-149 per component (u = 2^-24), so
//    |c_f - c_v| <= a = 2 (u R + 2^-148).
//  * The kernel's q (differences of the FP32 copies, squares and sums, fused
//    or not) satisfies (1-u)^5 c_f^2 - tau <= q <= (1+u)^5 c_f^2 + tau.
//  Hence, as for angles, q >= qhi_k => r2 >= S_k and q < qlo_k => r2 < S_k:
//      qhi_k = RU32(((C+ + a)^2 (1+u)^5 + tau) s),
//      qlo_k = RD32((((C- - a)_+)^2 (1-u)^5 - tau) / s),   s = 1 + 2^-20.
Band32 make_band32_3d(const EdgeTables &t, double rmax) {
    const double U = ldexp(1.0, -53), u = ldexp(1.0, -24);
    const double a = 2.0 * (u * rmax + ldexp(1.0, -148));
    const double grow = pow(1.0 + u, 5.0), shrink = pow(1.0 - u, 5.0);
    const double grow64 = pow(1.0 + U, 5.0), shrink64 = pow(1.0 - U, 5.0);
    const double tau = ldexp(1.0, -120), tau64 = ldexp(1.0, -1020);
    const double s = 1.0 + ldexp(1.0, -20);
    Band32 b;
    b.delta = rmax;
    const int ne = (int)t.D.size();
    b.qlo.resize(ne);
    b.qhi.resize(ne);
    for (int k = 0; k < ne; ++k) {
        const double S = t.E[k];
        if (S == -HUGE_VAL) {
            b.qlo[k] = b.qhi[k] = -HUGE_VALF;
            continue;
        }
        const double cp = sqrt((S + tau64) / shrink64);
        const double hi = ((cp + a) * (cp + a) * grow + tau) * s;
        b.qhi[k] = round_up32(hi);     // +inf above the FP32 range: never certain
        const double cm = sqrt(std::max(0.0, S - tau64) / grow64) - a;
        if (cm <= 0.0) {
            b.qlo[k] = 0.0f;
        } else {
            const double v = (cm * cm * shrink - tau) / s;
            b.qlo[k] = v <= 0.0 ? 0.0f : round_down32(v);
        }
    }
    return b;
}

uint32_t qtop_key_3d(double rmax) {
    const double u = ldexp(1.0, -24);
    const double c = 2.0 * rmax * (1.0 + 2.0 * u) + ldexp(1.0, -140);
    const double q = c * c * pow(1.0 + u, 5.0) * 1.0001 + ldexp(1.0, -120);
    return fbits(q < 3.0e38 ? round_up32(q) : 3.0e38f);
}

// FP32 cells: key = bits(q) >> shift for q >= 0.  The bottom cell also holds
// every q below its range and the top cell every q above.
namespace {

// Largest q = fl32(|f_i - f_j|^2) the kernel can produce: |f_i - f_j| <=
// 2 sqrt(1 + delta) + a few FP32 ulps, and the rounding of q is far below the
// 1e-4 margin.
uint32_t qtop_key(double delta) {
    const double qtop_d = pow(2.0 * sqrt(1.0 + delta) + 4.0 * ldexp(1.0, -24), 2.0) * 1.0001;
    return fbits(round_up32(qtop_d));
}

// Entries of FP32 cells [lo, hi] (bit patterns c << shift .. ((c+1) << shift) - 1);
// the bottom cell reaches down to 0 and the top one up to +inf (a clamp sends
// every key outside the table there).
void fill_cells32(const Band32 &b, int ne, CellTable *ct) {
    const int n = ct->hi - ct->lo + 1;
    ct->cells.resize(n);
    for (int c = ct->lo; c <= ct->hi; ++c) {
        float lo = c == ct->lo ? 0.0f : ffrom((uint32_t)c << ct->shift);
        float hi = c == ct->hi ? HUGE_VALF : ffrom((((uint32_t)c + 1u) << ct->shift) - 1u);
        int s_min = 0, s_max = 0;
        for (int k = 0; k < ne; ++k) {
            if (lo >= b.qhi[k])
                ++s_min;
            if (hi >= b.qlo[k])
                ++s_max;
        }
        ct->cells[c - ct->lo] = encode(s_min, s_max);
    }
    tally(ct);
}

}  // namespace

float floor_for(const Band32 &b) {
    // smallest positive finite threshold of the band without a floor
    float tmin = HUGE_VALF;
    for (size_t k = 0; k < b.qlo.size(); ++k) {
        if (isfinite(b.qlo[k]) && b.qlo[k] > 0.0f)
            tmin = std::min(tmin, b.qlo[k]);
        if (isfinite(b.qhi[k]) && b.qhi[k] > 0.0f)
            tmin = std::min(tmin, b.qhi[k]);
    }
    if (!isfinite(tmin))
        return 1.0f;                // no positive threshold: any floor below the edges' range
    int ex = 0;
    frexpf(tmin, &ex);              // tmin in [2^(ex-1), 2^ex)
    return ldexpf(1.0f, std::max(ex - 3, -100));    // at most tmin / 4, never below 2^-100
}

CellTable make_cells32_wrap(const EdgeTables &t, const Band32 &b, double delta, int max_bytes,
                            int aux_bytes) {
    CellTable ct;
    if (!(delta <= ldexp(1.0, -10)) || !(b.q0 > 0.0f))
        return ct;
    // every q the kernel forms lies in [q0, qtop]: the floor is a lower bound
    // of each partial sum, and qtop (for the largest chord) grows by the floor
    const uint32_t klo_bits = fbits(b.q0);
    const double qtop_d = (pow(2.0 * sqrt(1.0 + delta) + 4.0 * ldexp(1.0, -24), 2.0) + b.q0) * 1.0001;
    const uint32_t ktop = fbits(round_up32(qtop_d));
    const int aux = (aux_bytes + 15) & ~15;
    for (int shift = 12; shift <= 23; ++shift) {
        const int64_t lo = klo_bits >> shift, hi = ktop >> shift, n = hi - lo + 1;
        // the smallest table that holds the cells, with the histograms and
        // thresholds after it, if that is smaller than holding them inside
        int64_t after = 0;
        for (int w = 8; w <= 16 && after == 0; ++w)
            if (((int64_t)1 << w) >= n)
                after = (int64_t)1 << w;
        for (int w = 8; w <= 16; ++w) {
            const int64_t size = (int64_t)1 << w, mask = size - 1;
            if (after && after + aux <= max_bytes && after + aux < size) {
                ct.shift = shift;
                ct.lo = (int32_t)lo;
                ct.hi = (int32_t)hi;
                ct.direct = true;
                ct.wrap_bits = 0;
                while (((int64_t)1 << ct.wrap_bits) < after)
                    ++ct.wrap_bits;
                ct.aux_off = (int32_t)after;
                ct.q0 = b.q0;
                fill_cells32(b, (int)t.D.size(), &ct);
                ct.image.assign((size_t)after, 0);
                for (int64_t c = lo; c <= hi; ++c)
                    ct.image[(size_t)(c & (after - 1))] = ct.cells[(size_t)(c - lo)];
                return ct;
            }
            if (size > max_bytes)
                break;
            if (n + aux + 32 > size)
                continue;
            // the cells' arc is [lo & mask, hi & mask] (mod size); the rest of
            // the table is never read, and the histograms and thresholds go into
            // its longest contiguous piece
            const int64_t f0 = (hi + 1) & mask, fn = size - n;
            int64_t start, len;
            if (f0 + fn <= size) {
                start = f0;
                len = fn;
            } else if (size - f0 >= fn - (size - f0)) {
                start = f0;
                len = size - f0;
            } else {
                start = 0;
                len = fn - (size - f0);
            }
            const int64_t a0 = (start + 15) & ~(int64_t)15;
            if (a0 + aux > start + len)
                continue;
            ct.shift = shift;
            ct.lo = (int32_t)lo;
            ct.hi = (int32_t)hi;
            ct.direct = true;
            ct.wrap_bits = w;
            ct.aux_off = (int32_t)a0;
            ct.q0 = b.q0;
            fill_cells32(b, (int)t.D.size(), &ct);
            ct.image.assign((size_t)size, 0);
            for (int64_t c = lo; c <= hi; ++c)
                ct.image[(size_t)(c & mask)] = ct.cells[(size_t)(c - lo)];
            return ct;
        }
    }
    return ct;
}

CellTable make_cells32(const EdgeTables &t, const Band32 &b, double delta, int max_cells) {
    return make_cells32_top(t, b, qtop_key(delta), max_cells);
}

CellTable make_cells32_top(const EdgeTables &t, const Band32 &b, uint32_t ktop, int max_cells) {
    const int ne = (int)t.D.size();
    // smallest positive finite threshold
    float tmin = HUGE_VALF;
    for (int k = 0; k < ne; ++k) {
        if (isfinite(b.qlo[k]) && b.qlo[k] > 0.0f)
            tmin = std::min(tmin, b.qlo[k]);
        if (isfinite(b.qhi[k]) && b.qhi[k] > 0.0f)
            tmin = std::min(tmin, b.qhi[k]);
    }
    CellTable ct;
    for (int shift = 12; shift <= 23; ++shift) {
        int64_t hi = ktop >> shift;
        int64_t lo = isfinite(tmin) ? (int64_t)(fbits(tmin) >> shift) - 1 : hi - 1;
        if (lo < 0)
            lo = 0;
        if (hi - lo + 1 <= max_cells || shift == 23) {
            if (hi - lo + 1 > max_cells)
                lo = hi - max_cells + 1;
            ct.shift = shift;
            ct.lo = (int32_t)lo;
            ct.hi = (int32_t)hi;
            break;
        }
    }
    fill_cells32(b, ne, &ct);
    return ct;
}

// FP64 cells: key = (int32) high word of e = fl(1 - d), arithmetic shift.
// e < 0 (d > 1 from rounding) falls into the bottom cell, whose range is
// taken to start at -inf.
CellTable make_cells64(const EdgeTables &t, int max_cells, double etop) {
    const int ne = (int)t.E.size();
    const int32_t ktop = dhi(etop);
    double tmin = HUGE_VAL;
    for (int k = 0; k < ne; ++k)
        if (isfinite(t.E[k]) && t.E[k] > 0.0)
            tmin = std::min(tmin, t.E[k]);
    CellTable ct;
    for (int shift = 9; shift <= 20; ++shift) {
        int64_t hi = ktop >> shift;
        int64_t lo = isfinite(tmin) ? (int64_t)(dhi(tmin) >> shift) - 1 : hi - 1;
        if (lo < 0)
            lo = 0;
        if (hi - lo + 1 <= max_cells || shift == 20) {
            if (hi - lo + 1 > max_cells)
                lo = hi - max_cells + 1;
            ct.shift = shift;
            ct.lo = (int32_t)lo;
            ct.hi = (int32_t)hi;
            break;
        }
    }
    const int n = ct.hi - ct.lo + 1;
    ct.cells.resize(n);
    for (int c = ct.lo; c <= ct.hi; ++c) {
        double lo = c == ct.lo ? -HUGE_VAL : dfrom((uint64_t)((uint32_t)c << ct.shift) << 32);
        double hi = c == ct.hi ? HUGE_VAL
                               : dfrom(((uint64_t)((((uint32_t)c + 1u) << ct.shift) - 1u) << 32) |
                                       0xffffffffULL);
        int s_min = 0, s_max = 0;
        for (int k = 0; k < ne; ++k) {
            // E_k = -inf (an edge at 0, D_k = +inf): every pair is past it,
            // the bottom cell's open end included
            if (lo > t.E[k] || t.E[k] == -HUGE_VAL)
                ++s_min;
            if (hi >= t.E[k])
                ++s_max;
        }
        ct.cells[c - ct.lo] = encode(s_min, s_max);
    }
    tally(&ct);
    return ct;
}

}  // namespace tpcf
