"""Exact-real reference for the track and its bin, for pinning the oracle.

The frequency of a template in the detector frame is (Eqs. 1-2 of the paper)
    f^(t) = f0 * (1 + (t - T0)/tau)^(1/(1-n)) * (1 + v(t).n/c)
and the bin it selects is the nearest multiple of 1/T_sft.  This module
evaluates that real number from the exact values of the FP64 inputs using
rational arithmetic for +,-,*,/ and 50-digit decimal ln/exp for the power,
so it shares no rounding sequence with the oracle.  It is used only to check
properties (nearest bin, exact special cases), never as a bit-exact twin.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction

getcontext().prec = 50
C_LIGHT = 299792458


def _dec(fr: Fraction) -> Decimal:
    return Decimal(fr.numerator) / Decimal(fr.denominator)


def true_spin(t, t0, tau, brake) -> Decimal:
    u = 1 + (Fraction(t) - Fraction(t0)) / Fraction(tau)
    e = Fraction(1) / (1 - Fraction(brake))
    return (_dec(e) * _dec(u).ln()).exp()


def true_doppler(v, n) -> Decimal:
    vn = sum(Fraction(a) * Fraction(b) for a, b in zip(v, n))
    return _dec(1 + vn / C_LIGHT)


def true_x(f0, t, t0, tau, brake, v, n, t_sft) -> Decimal:
    """f^ * T_sft as a 50-digit decimal."""
    return _dec(Fraction(f0)) * true_spin(t, t0, tau, brake) * true_doppler(v, n) * _dec(Fraction(t_sft))


def true_bin(f0, t, t0, tau, brake, v, n, t_sft, k_lo):
    """(column, distance of x from the nearest half-integer)."""
    x = true_x(f0, t, t0, tau, brake, v, n, t_sft)
    k = int((x + Decimal("0.5")).to_integral_value(rounding="ROUND_FLOOR"))
    frac = x - int(x.to_integral_value(rounding="ROUND_FLOOR"))
    margin = abs(frac - Decimal("0.5"))
    return k - int(k_lo), float(margin)


def correctly_rounded_pow(u: float, e: float) -> float:
    """RN(u^e) for FP64 u > 0 and e, via a 50-digit decimal power (rounded once by float())."""
    return float((Decimal(u).ln() * Decimal(e)).exp())
