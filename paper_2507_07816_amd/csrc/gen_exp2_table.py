"""Writes exp2_table.h: 2^(j/256), j = 0..255, as double-doubles (hi = RN(x),
lo = RN(x - hi)), and ln 2 / 256 split into a 35-bit head and two tails,
all from 60-digit decimal arithmetic.  Run from this directory:
    python gen_exp2_table.py > exp2_table.h
"""
from decimal import Decimal, getcontext
from fractions import Fraction


def dd(x):
    hi = float(x)
    lo = float(x - Fraction(hi))
    return hi, lo


def head(x, bits):
    """x rounded to `bits` significant bits (a double)."""
    f = Fraction(x)
    e = 0
    while abs(f) >= 2:
        f /= 2
        e += 1
    while abs(f) < 1:
        f *= 2
        e -= 1
    m = round(f * 2 ** (bits - 1))
    return float(Fraction(m, 2 ** (bits - 1)) * Fraction(2) ** e)


def main():
    getcontext().prec = 60
    ln2 = Fraction(Decimal(2).ln())
    out = ["// 2^(j/256) as double-doubles and ln 2 / 256 in three parts, written by",
           "// gen_exp2_table.py from 60-digit decimal arithmetic (checked by a CPU test).",
           "#pragma once", "", "namespace ltgw {", ""]
    c = ln2 / 256
    h1 = head(c, 35)
    h2 = float(c - Fraction(h1))
    h3 = float(c - Fraction(h1) - Fraction(h2))
    out.append(f"constexpr double kLn2d256_1 = {h1.hex()};  // 35 significant bits: N * it is exact for |N| < 2^18")
    out.append(f"constexpr double kLn2d256_2 = {h2.hex()};")
    out.append(f"constexpr double kLn2d256_3 = {h3.hex()};")
    out.append("")
    out.append("// [j][hi, lo]")
    out.append("constexpr double kExp2Tab[256][2] = {")
    for j in range(256):
        x = Fraction(Decimal(2) ** (Decimal(j) / Decimal(256)))
        hi, lo = dd(x)
        out.append(f"    {{{hi.hex()}, {lo.hex()}}},")
    out.append("};")
    out.append("")
    out.append("}  // namespace ltgw")
    print("\n".join(out))


if __name__ == "__main__":
    main()
