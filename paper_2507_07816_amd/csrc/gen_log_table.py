"""Writes log_table.h for the fast phase of the correctly rounded power:
for i = 0..127 (the top 7 bits of a mantissa m in [1, 2)), r_i = K_i / 256 with
K_i = round(256 / c_i), c_i = 1 + (i + 1/2) / 128 the centre of the interval,
so that m r_i - 1 is exact in FP64 (an 8-bit r_i times a 53-bit m, minus 1,
fits 53 bits) and below 2^-7 in magnitude; and -log(r_i) = log(256 / K_i) as
hi + lo, hi the nearest multiple of 2^-35 and lo = RN(x - hi), from 60-digit
decimal arithmetic.  On the 2^-35 grid hi adds to k times the 35-bit head of
ln 2 exactly (|k| < 2^10), and hi + lo is still within 2^-89 of -log(r_i).
Run from this directory:
    python gen_log_table.py > log_table.h
"""
from decimal import Decimal, getcontext
from fractions import Fraction


def split35(x):
    hi = Fraction(round(x * 2 ** 35), 2 ** 35)
    lo = float(x - hi)
    return float(hi), lo


def entries():
    out = []
    for i in range(128):
        c = Fraction(1) + Fraction(2 * i + 1, 256)
        K = round(Fraction(256) / c)
        out.append((i, K))
    return out


def main():
    getcontext().prec = 60
    lines = ["// r_i = K_i / 256 near 1 / (1 + (i + 1/2) / 128) and -log(r_i) = hi + lo with hi on the",
             "// 2^-35 grid, written by gen_log_table.py from 60-digit decimal arithmetic (checked by a",
             "// CPU test).",
             "#pragma once", "", "namespace ltgw {", "",
             "// [i][r_i, hi, lo]", "constexpr double kLogTab[128][3] = {"]
    for i, K in entries():
        x = Fraction((Decimal(256) / Decimal(K)).ln())
        hi, lo = split35(x)
        lines.append(f"    {{{float(Fraction(K, 256)).hex()}, {hi.hex()}, {lo.hex()}}},")
    lines += ["};", "", "}  // namespace ltgw"]
    print("\n".join(lines))


if __name__ == "__main__":
    main()
