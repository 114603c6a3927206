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
// e^Y for |Y.hi| < 700.  Y = N ln2/256 + r with N = rint(Y 256/ln2), so
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

// RN(u^e) for finite u > 0, finite e, with u^e a normal double.
// *undecided = 1 when the double-double result (relative error < 2^-98) is
// within that error of the midpoint between two doubles.
LTGW_HD double pow_cr(double u, double e, int *undecided) {
    *undecided = 0;
    if (u == 1.0) return 1.0;
    dd L = dd_log(u);
    dd Y = dd_mul_d(L, e);
    if (!(std::fabs(Y.hi) < 700.0)) {
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

}  // namespace ltgw
