// Correctly rounded FP64 power u^e for the spin-down factor of Eq. 1
// (g = (1 + (t - T0)/tau)^(1/(1-n))), in double-double arithmetic.
//
// Building blocks are the error-free transformations of Knuth (TwoSum) and
// Dekker (Fast2Sum; exact product via a fused multiply-add), combined into
// double-double add/multiply/divide in the way of Hida, Li and Bailey's
// double-double arithmetic.  On top of them:
//   exp:  Y = N ln2/256 + r with a three-part ln2/256 (so N times its head
//         is exact for |N| < 2^18), |r| <= ln2/512, Taylor series of
//         expm1(r) to r^10, times 2^(j/256) (N = 256 k + j) from a
//         double-double table, times 2^k.
//   log:  one Newton step on exp: y0 = log(u) from the device math library,
//         d = u e^-y0 - 1, log u = y0 + d - d^2/2 (+O(d^3), |d| < 2^-50).
//   pow:  exp(e * log u); result error below 2^-98 relative.  The nearest
//         double is returned; when the double-double value lies too close to
//         a rounding boundary to decide, the caller is told (undecided = 1).
//
// That evaluation is the second phase of Ziv's strategy.  pow_cr first takes a
// cheaper one (pow_fast, below: table-driven log and exp to about 2^-70) and
// returns its nearest double when the value lies farther than its error bound
// from every rounding boundary; only the rest go through double-double.
//
// ln 2 / 256 is split as a 35-bit head plus two tails (each the nearest
// double of the remainder), and 2^(j/256) is tabulated as double-doubles;
// both come from exp2_table.h, whose values a host test checks against
// 60-digit decimal arithmetic.
//
// Everything here must be compiled without floating-point contraction.
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

#include "exp2_table.h"
#include "log_table.h"

#ifdef __HIPCC__
#define LTGW_HD __host__ __device__ inline
#else
#define LTGW_HD inline
#endif

#pragma clang fp contract(off)

namespace ltgw {

struct dd {
    double hi, lo;
};

constexpr double kInvLn2 = 0x1.71547652b82fep+0;
// 1/3 and 1/5 as double-doubles: hi = RN(1/m), lo = RN(1/m - hi) (relative
// error 3.1e-33, checked by a host test with exact rationals)
constexpr double kInv3_hi = 0x1.5555555555555p-2, kInv3_lo = 0x1.5555555555555p-56;
constexpr double kInv5_hi = 0x1.999999999999ap-3, kInv5_lo = -0x1.999999999999ap-57;
// RN(1/m) for the FP64 Taylor factors (indices 6..10 used)
constexpr double kRecip[11] = {0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5,
                               1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9, 1.0 / 10};

LTGW_HD dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
// requires |a| >= |b| or a == 0
LTGW_HD dd fast_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
LTGW_HD dd two_prod(double a, double b) {
    double p = a * b;
    double e = std::fma(a, b, -p);
    return {p, e};
}
LTGW_HD dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
LTGW_HD dd dd_add_d(dd a, double b) {
    dd s = two_sum(a.hi, b);
    s.lo += a.lo;
    return fast_two_sum(s.hi, s.lo);
}
LTGW_HD dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return fast_two_sum(p.hi, p.lo);
}
LTGW_HD dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return fast_two_sum(p.hi, p.lo);
}
// e^Y for -600 < Y.hi < 700 (below, the low part of the result would be
// subnormal and lose bits).  Y = N ln2/256 + r with N = rint(Y 256/ln2), so
// |r| <= ln2/512; e^Y = 2^k 2^(j/256) e^r with N = 256 k + j, 0 <= j < 256,
// 2^(j/256) from a double-double table.
LTGW_HD dd dd_exp(dd Y) {
    const double nf = std::rint(Y.hi * (kInvLn2 * 256.0));
    // N * head is exact (35-bit head, |N| < 2^18); Y.hi - N * head is exact
    // too: both are multiples of the finer of their last bits and the
    // difference is below 2^-9.5
    const double a = Y.hi - nf * kLn2d256_1;
    dd r = two_sum(a, Y.lo);
    dd nl = two_prod(nf, kLn2d256_2);
    nl.lo += nf * kLn2d256_3;
    r = dd_add(r, dd{-nl.hi, -nl.lo});
    // expm1(r) = r (1 + r/2 (1 + r/3 (... (1 + r/10)))), |r| < 1.36e-3.  The
    // inner factors r/10 ... r/6 (...) are formed in FP64 from r.hi: their
    // rounding reaches expm1(r) scaled by r^5/5! < 2^-54, i.e. below 2^-110
    // relative.  The outer four stay in double-double, dividing by 5 and 3 as
    // products with double-double reciprocals (by 4 and 2 exactly).
    double q = r.hi * kRecip[10];
    for (int m = 9; m >= 6; --m) q = ((q + 1.0) * r.hi) * kRecip[m];
    dd p = dd_mul(dd_mul(two_sum(1.0, q), r), dd{kInv5_hi, kInv5_lo});
    p = dd_mul(dd_add_d(p, 1.0), r);
    p = {p.hi * 0.25, p.lo * 0.25};
    p = dd_mul(dd_mul(dd_add_d(p, 1.0), r), dd{kInv3_hi, kInv3_lo});
    p = dd_mul(dd_add_d(p, 1.0), r);
    p = {p.hi * 0.5, p.lo * 0.5};
    p = dd_mul(dd_add_d(p, 1.0), r);
    const int n = (int)nf;
    const int jj = n & 255;       // the residue in [0, 256), also for n < 0
    const int k = (n - jj) / 256;  // exact
    const dd e = dd_mul(dd_add_d(p, 1.0), dd{kExp2Tab[jj][0], kExp2Tab[jj][1]});
    return {std::ldexp(e.hi, k), std::ldexp(e.lo, k)};
}

// log(u) for finite u > 0.
LTGW_HD dd dd_log(double u) {
    double y0 = std::log(u);
    dd E = dd_exp(dd{y0, 0.0});
    dd d = two_sum(u, -E.hi);
    double num = d.hi + (d.lo - E.lo);
    double dl = num / E.hi;
    double corr = dl - 0.5 * dl * dl;
    return fast_two_sum(y0, corr);
}

LTGW_HD uint64_t bits_of(double x) {
    uint64_t b;
    std::memcpy(&b, &x, 8);
    return b;
}
LTGW_HD double from_bits(uint64_t b) {
    double x;
    std::memcpy(&x, &b, 8);
    return x;
}

// RN(u^e) for finite u > 0, finite e, in double-double arithmetic.
// *undecided = 1 when the double-double result (relative error < 2^-98) is
// within that error of the midpoint between two doubles, and when e log u
// lies outside (-600, 700) (then the nearest double of exp(e log u) in FP64 is
// returned).
LTGW_HD double pow_dd(double u, double e, int *undecided) {
    *undecided = 0;
    if (u == 1.0) return 1.0;
    dd L = dd_log(u);
    dd Y = dd_mul_d(L, e);
    if (!(Y.hi > -600.0 && Y.hi < 700.0)) {
        *undecided = 1;
        return std::exp(Y.hi);
    }
    dd R = dd_exp(Y);
    R = fast_two_sum(R.hi, R.lo);
    double G = R.hi;
    uint64_t gb = bits_of(G);
    double up = from_bits(gb + 1) - G;   // G > 0 and normal
    double dn = G - from_bits(gb - 1);
    double tol = G * 0x1p-98;
    if (!(R.lo + tol < 0.5 * up) || !(R.lo - tol > -0.5 * dn)) *undecided = 1;
    return G;
}

// RN(x / d) from y = RN(1 / d), for normal d and a quotient far from underflow
// and overflow: q = RN(x y) is within one ulp of x / d, the residual
// x - q d is exact by one FMA, and RN(q + r y) is then the correctly rounded
// quotient (Markstein's correction theorem).  Three operations in place of a
// division, where one divisor serves many quotients.
LTGW_HD double div_rn(double x, double d, double y) {
    const double q = x * y;
    const double r = std::fma(-q, d, x);
    return std::fma(r, y, q);
}

// ---- fast phase ----------------------------------------------------------------
// RN(1/m) for the Taylor coefficients
constexpr double kInvN[10] = {0.0, 1.0, 1.0 / 2, 1.0 / 3, 1.0 / 4, 1.0 / 5, 1.0 / 6, 1.0 / 7, 1.0 / 8, 1.0 / 9};
// ln 2 in three parts (256 times those of ln 2 / 256: k times the head is exact
// for |k| < 2^18)
constexpr double kLn2_1 = 256.0 * kLn2d256_1, kLn2_2 = 256.0 * kLn2d256_2, kLn2_3 = 256.0 * kLn2d256_3;

// log(u) for normal u > 0 as hi + lo with absolute error below
// 2^-72 + 2^-104 |log u|, not normalised: |lo| < 2^-23, which may exceed |hi|
// near u = 1.  u = 2^k m, m in [1, 2); i is the top 7 bits of m's fraction and
// r_i an 8-bit number near 1/m (table), so z = m r_i - 1 is exact by one FMA
// and |z| < 0.0056; then log u = k ln 2 - log r_i + log1p(z), log1p by its
// Taylor series through z^9 (truncation below 2^-80), z - z^2/2 in
// double-double, the rest in FP64 (below 2^-74).  The table's head of
// -log r_i lies on the 2^-35 grid of ln 2's 35-bit head, so k ln2_head plus
// it is exact.
LTGW_HD dd log_fast(double u) {
    const uint64_t b = bits_of(u);
    const int k = (int)(b >> 52) - 1023;
    const double m = from_bits((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
    const int i = (int)((b >> 45) & 127u);
    const double z = std::fma(m, kLogTab[i][0], -1.0);
    // P(z) = 1/3 - z/4 + z^2/5 - z^3/6 + z^4/7 - z^5/8 + z^6/9
    double p = kInvN[9];
    p = std::fma(z, p, -kInvN[8]);
    p = std::fma(z, p, kInvN[7]);
    p = std::fma(z, p, -kInvN[6]);
    p = std::fma(z, p, kInvN[5]);
    p = std::fma(z, p, -kInvN[4]);
    p = std::fma(z, p, kInvN[3]);
    const dd z2 = two_prod(z, z);
    const dd h = fast_two_sum(z, -0.5 * z2.hi);  // |z| > z^2/2
    const double hlo = (h.lo - 0.5 * z2.lo) + (z2.hi * z) * p;
    const double kd = (double)k;
    const double s1 = kd * kLn2_1 + kLogTab[i][1];  // exact: both on the 2^-35 grid, below 2^10
    const dd s2 = two_sum(s1, h.hi);
    const double lo = (s2.lo + (hlo + kLogTab[i][2])) + (kd * kLn2_2 + kd * kLn2_3);
    return {s2.hi, lo};
}

// e^Y for normalised Y (|Y.lo| <= ulp(Y.hi)), -600 < Y.hi < 700, as a normalised
// double-double with relative error below 2^-70 (plus Y's own).  The reduced
// argument is r + rlo with |rlo| <= ulp(Y.hi) < 2^-43, so
// e^(r + rlo) = e^r (1 + rlo) to 2^-87, and e^r rlo is taken as
// rlo (1 + r + r^2/2) to 2^-75.  Y = N ln2/256 + r as in dd_exp, |r| <= ln2/512;
// e^r = 1 + r + r^2/2 + r^3 Q(r), Q = 1/6 + r/24 + r^2/120 + r^3/720
// (truncation below 2^-78), 1 + r and r^2 exact, the small terms in FP64.
LTGW_HD dd exp_fast(dd Y) {
    const double nf = std::rint(Y.hi * (kInvLn2 * 256.0));
    const double a = Y.hi - nf * kLn2d256_1;  // exact, as in dd_exp
    const dd nl = two_prod(nf, kLn2d256_2);
    const dd s = two_sum(a, -nl.hi);
    const double r = s.hi;
    const double rlo = ((s.lo + Y.lo) - nl.lo) - nf * kLn2d256_3;
    double q = std::fma(r, 1.0 / 720.0, 1.0 / 120.0);
    q = std::fma(r, q, 1.0 / 24.0);
    q = std::fma(r, q, kInvN[6]);
    const dd r2 = two_prod(r, r);
    const dd one = fast_two_sum(1.0, r);
    const double cross = rlo * (r + 0.5 * r2.hi);  // e^r rlo = rlo + cross
    const double lo = one.lo + (rlo + (0.5 * r2.hi + ((0.5 * r2.lo + cross) + (r2.hi * r) * q)));
    const dd E = fast_two_sum(one.hi, lo);
    const int n = (int)nf;
    const int jj = n & 255;
    const int k = (n - jj) / 256;
    const dd R = dd_mul(E, dd{kExp2Tab[jj][0], kExp2Tab[jj][1]});
    return {std::ldexp(R.hi, k), std::ldexp(R.lo, k)};
}

// The fast phase: *g = RN(u^e) and true when u^e, evaluated to relative error
// below (1 + |e|) 2^-70 + 2^-93, lies more than (1 + |e|) 2^-66 (sixteen times
// that bound) relative from the midpoint between two doubles; false otherwise
// (the caller takes pow_dd).  Normal u in [2^-1000, 2^1000); false when e log u
// lies outside (-600, 700).
// The fast phase's value of u^e before rounding (a normalised double-double),
// or false when e log u lies outside (-600, 700).
LTGW_HD bool pow_fast_value(double u, double e, dd *R) {
    const dd L = log_fast(u);
    dd Y = two_prod(e, L.hi);
    Y = two_sum(Y.hi, Y.lo + e * L.lo);  // L.lo may exceed L.hi near u = 1
    if (!(Y.hi > -600.0 && Y.hi < 700.0)) return false;
    const dd E = exp_fast(Y);
    *R = fast_two_sum(E.hi, E.lo);
    return true;
}

LTGW_HD bool pow_fast(double u, double e, double *g) {
    dd R;
    if (!pow_fast_value(u, e, &R)) return false;
    const double G = R.hi;
    // u^e lies within tol/8 of G + R.lo.  When G + RN(R.lo + tol) and
    // G + RN(R.lo - tol) both round to G, R.lo + tol <= up/2 (1 + 2^-53) and
    // R.lo - tol >= -dn/2 (1 + 2^-53) (up, dn: the gaps to G's neighbours),
    // so u^e lies strictly inside G's rounding interval: its nearest double
    // is G.
    const double tol = G * ((1.0 + std::fabs(e)) * 0x1p-66);
    if (!(G + (R.lo + tol) == G) || !(G + (R.lo - tol) == G)) return false;
    *g = G;
    return true;
}

// The double-double phase as a call.  Inlined, its registers would add to the
// fast phase's in every kernel that takes a power, and a kernel's register
// count sets its occupancy, although this phase runs for about one power in
// four thousand.  The result comes back by value (no pointer to a caller's
// local, which would put that local in scratch memory).
struct PowSlow {
    double g;
    int undecided;
};
#ifdef __HIPCC__
__host__ __device__
#endif
__attribute__((noinline)) inline PowSlow pow_dd_call(double u, double e) {
    PowSlow r;
    r.g = pow_dd(u, e, &r.undecided);
    return r;
}

// RN(u^e) for finite u > 0, finite e, with u^e a normal double: the fast phase,
// and where it cannot decide the double-double one (*slow = 1, when given).
// *undecided = 1 only when the double-double phase cannot decide either.
LTGW_HD double pow_cr(double u, double e, int *undecided, int *slow = nullptr) {
    *undecided = 0;
    if (slow) *slow = 0;
    if (u == 1.0) return 1.0;
    double g;
    if (u >= 0x1p-1000 && u < 0x1p1000 && pow_fast(u, e, &g)) return g;
    if (slow) *slow = 1;
    const PowSlow r = pow_dd_call(u, e);
    *undecided = r.undecided;
    return r.g;
}

}  // namespace ltgw
