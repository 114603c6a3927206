// An enclosure of the correctly rounded spin-down factor RN(u^e) of Eq. 1,
// for decisions that depend monotonically on it.
//
// The explicit-template evaluation needs the power only through the column a
// track falls in: column(g) = trunc(RN(f0 RN(RN(g D) T_sft)) + shift), a
// composition of products by fixed factors, roundings to nearest, a fixed
// shift and truncation, each monotone, so column is monotone in g.  When it
// takes the same value at both ends of an interval that holds RN(u^e), that
// is its value at RN(u^e): the correctly rounded power is only needed when the
// interval straddles a column boundary.  An interval of relative width about
// 2^-40 around values near 6000 bins straddles a boundary for about one
// evaluation in 10^8.
//
// The approximation G of u^e is plain FP64 on the tables of the fast phase
// (log_table.h, exp2_table.h): for u = 2^k m >= 1, m in [1, 2), i the top
// 7 bits of m's fraction and r_i the table's 8-bit number near 1/m,
//   z = m r_i - 1 (exact by one FMA, |z| < 0.0056),
//   log u = k ln 2 + (-log r_i) + log1p(z), log1p(z) through z^6,
//   y = e log u = N ln2/256 + r, |r| <= ln2/512 (as in the fast phase),
//   u^e = 2^(N/256) e^r, e^r through r^4, 2^(j/256) the table's head.
// Error bound (absolute in log u, which becomes relative in u^e):
//   log1p's truncation |z|^7 / (7 (1 - |z|)) < 2^-55.1, its roundings below
//   2^-60; -log r_i rounded to a double, k ln 2 with ln 2 rounded to a
//   double, and the two sums, each within 2^-53 of terms whose magnitudes are
//   below 2.8 (|log u| + 0.0057) for u >= 1 (k >= 0 and -log r_i > 0, so
//   only log1p(z) can cancel them): |d log u| < 2^-51 |log u| + 2^-55;
//   |d y| < 2^-50.6 |y| + 2^-54.7 |e|;
//   e^r's truncation |r|^5/120 e^|r| < 2^-54.5 and roundings below 2^-52.4,
//   the table's head and the product 2^-53 each: 2^-51.2 relative;
// so |G - u^e| < 2^-50 (1 + |y| + |e|) u^e.  The interval is
// G (1 -+ eps), eps = 2^-42 (1 + |y| + |e|): the bound times 256, which also
// covers the rounding of RN(u^e) itself and of the interval's ends.
#pragma once
#include <cmath>
#include <cstdint>

#include "ddpow.h"
#include "exp2_table.h"
#include "log_table.h"

#pragma clang fp contract(off)

namespace ltgw {

// ln 2 to double precision (a CPU test checks it is the nearest double)
constexpr double kLn2rn = kLn2_1 + kLn2_2;

// The tables the enclosure reads, from the constant arrays: r_i and
// RN(-log r_i) for the log, RN(2^(j/256)) for the exponential.  A kernel may
// pass copies of the same values held in LDS.
struct EncloseTables {
    LTGW_HD void log_entry(int i, double *r, double *t) const {
        *r = kLogTab[i][0];
        *t = kLogTab[i][1] + kLogTab[i][2];
    }
    LTGW_HD double exp2_entry(int j) const { return kExp2Tab[j][0]; }
};

// The enclosure in three stages, so that a caller can run each stage over
// several arguments and overlap their table reads:
//   enclose_split: u = 2^k m and the log table's index i;
//   enclose_log:   with (r_i, RN(-log r_i)), y = e log u, N = rint(y 256/ln2)
//                  split as 256 k' + j, and E ~ e^r;
//   enclose_ends:  with RN(2^(j/256)), G = 2^k' 2^(j/256) E and the interval.
struct EncloseSplit {
    double m;
    int k, i;
    bool in;  // u in [1, 2^1000)
};
struct EncloseLog {
    double E, y;
    int j, k;
    bool ok;  // u in [1, 2^1000) and y in (-600, 700)
};

LTGW_HD EncloseSplit enclose_split(double u) {
    const uint64_t b = bits_of(u);
    EncloseSplit s;
    s.k = (int)(b >> 52) - 1023;
    s.m = from_bits((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
    s.i = (int)((b >> 45) & 127u);
    s.in = u >= 1.0 && u < 0x1p1000;
    return s;
}

// Branch-free; outside the domain (non-finite inputs included) ok is false
// and the rest means nothing.
LTGW_HD EncloseLog enclose_log(double e, const EncloseSplit &s, double ri, double ti) {
    const double z = std::fma(s.m, ri, -1.0);
    // log1p(z) = z + z^2 Q(z), Q = -1/2 + z/3 - z^2/4 + z^3/5 - z^4/6
    double q = std::fma(z, -kInvN[6], kInvN[5]);
    q = std::fma(z, q, -kInvN[4]);
    q = std::fma(z, q, kInvN[3]);
    q = std::fma(z, q, -0.5);
    const double p = std::fma(z * z, q, z);
    const double l = std::fma((double)s.k, kLn2rn, ti) + p;
    EncloseLog o;
    o.y = e * l;
    o.ok = s.in && o.y > -600.0 && o.y < 700.0;
    // clamped (NaN included), so that N below is a small integer on any input
    const double yc = std::fmin(std::fmax(o.y, -700.0), 700.0);
    const double nf = std::rint(yc * (kInvLn2 * 256.0));
    double r = std::fma(-nf, kLn2d256_1, yc);
    r = std::fma(-nf, kLn2d256_2, r);
    // e^r = 1 + r (1 + r (1/2 + r (1/6 + r/24)))
    double c = std::fma(r, 1.0 / 24.0, kInvN[6]);
    c = std::fma(r, c, 0.5);
    c = std::fma(r, c, 1.0);
    o.E = std::fma(r, c, 1.0);
    const int n = (int)nf;
    o.j = n & 255;
    o.k = (n - o.j) / 256;
    return o;
}

LTGW_HD double enclose_value(const EncloseLog &o, double x2) { return std::ldexp(o.E * x2, o.k); }

// [lo, hi] = G (1 -+ 2^-42 (1 + |y| + |e|))
LTGW_HD void enclose_ends(double G, double y, double e, double *lo, double *hi) {
    const double eps = ((1.0 + std::fabs(y)) + std::fabs(e)) * 0x1p-42;
    *lo = std::fma(-G, eps, G);
    *hi = std::fma(G, eps, G);
}

// G ~ u^e and y ~ e log u; true for u in [1, 2^1000) with y in (-600, 700),
// false outside that domain, where G and y are still written but mean nothing.
template <class Tables = EncloseTables>
LTGW_HD bool pow_enclose_value(double u, double e, double *G, double *y, const Tables &tab = Tables()) {
    const EncloseSplit s = enclose_split(u);
    double ri, ti;
    tab.log_entry(s.i, &ri, &ti);
    const EncloseLog o = enclose_log(e, s, ri, ti);
    *G = enclose_value(o, tab.exp2_entry(o.j));
    *y = o.y;
    return o.ok;
}

// true, with RN(u^e) in [*lo, *hi], for u in [1, 2^1000) and e log u in
// (-600, 700); false otherwise (then *lo and *hi mean nothing).
template <class Tables = EncloseTables>
LTGW_HD bool pow_enclose(double u, double e, double *lo, double *hi, const Tables &tab = Tables()) {
    double G, y;
    const bool ok = pow_enclose_value(u, e, &G, &y, tab);
    enclose_ends(G, y, e, lo, hi);
    return ok;
}

}  // namespace ltgw
