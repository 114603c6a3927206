"""The library's correctly rounded power (the device code of Eq. 1, built for
the host here) against the oracle's spin factor, bit for bit.

The kernels form u = 1 + (t - T0)/tau and e = 1/(1 - n) in FP64 exactly as the
oracle does and take RN(u^e) in double-double arithmetic, flagging the cases
they cannot decide; the oracle takes the power in binary128.  Over the
parameter ranges of Sec. 1 (and beyond: tau down to 300 s, n from 1.5 to 9,
a day of segments), every decided power must equal the oracle's.
"""
import os
import subprocess

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_07816_amd", "csrc")

DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ddpow.h"
int main(int argc, char **argv) {
    FILE *fi = std::fopen(argv[1], "rb");
    FILE *fo = std::fopen(argv[2], "wb");
    long n = std::atol(argv[3]);
    std::vector<double> in(4 * n), g(n);
    std::vector<int> und(n);
    if (std::fread(in.data(), 8, 4 * n, fi) != (size_t)(4 * n)) return 1;
    for (long i = 0; i < n; ++i) {
        const double t = in[4 * i], t0 = in[4 * i + 1], tau = in[4 * i + 2], brake = in[4 * i + 3];
        const double e = 1.0 / (1.0 - brake);
        if (t < t0) { g[i] = 0.0; und[i] = 0; continue; }
        const double dt = t - t0;
        const double q = dt / tau;
        const double u = 1.0 + q;
        g[i] = ltgw::pow_cr(u, e, &und[i]);
    }
    std::fwrite(g.data(), 8, n, fo);
    std::fwrite(und.data(), 4, n, fo);
    return 0;
}
'''


def _driver(tmp_path):
    src = tmp_path / "ddpow_driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "ddpow_driver"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I", CSRC,
                    str(src), "-o", str(exe)], check=True)
    return exe


def _run(exe, tmp_path, rows):
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    fi, fo = tmp_path / "in.bin", tmp_path / "out.bin"
    rows.tofile(fi)
    subprocess.run([str(exe), str(fi), str(fo), str(len(rows))], check=True)
    raw = np.fromfile(fo, dtype=np.uint8)
    n = len(rows)
    g = raw[:8 * n].view(np.float64)
    und = raw[8 * n:].view(np.int32)
    return g, und


def test_pow_matches_oracle_over_the_search_ranges(tmp_path):
    exe = _driver(tmp_path)
    r = np.random.default_rng(41)
    n_pairs, n_t = 300, 1500
    tau = np.exp(r.uniform(np.log(300.0), np.log(40000.0), n_pairs))
    brake = r.uniform(1.5, 9.0, n_pairs)
    brake[:20] = [3.0, 5.0, 7.0, 2.0, 4.0, 6.0, 9.0, 1.5, 2.5, 3.5, 4.5, 5.5, 6.5, 7.5, 8.0, 8.5,
                  3.25, 4.75, 5.125, 6.875]
    t0 = r.choice([0.0, 1000.0, 3.5], n_pairs)
    rows, ref = [], []
    for k in range(n_pairs):
        t = np.sort(r.uniform(0.0, 86400.0, n_t))
        t[:3] = [t0[k], t0[k] + 8.0, 86400.0]          # u = 1, one segment after T0, the end
        rows.append(np.column_stack([t, np.full(n_t, t0[k]), np.full(n_t, tau[k]), np.full(n_t, brake[k])]))
        ref.append(oracle.spin_factor_array(t, t0[k], tau[k], brake[k]))
    rows = np.concatenate(rows)
    ref = np.concatenate(ref)
    g, und = _run(exe, tmp_path, rows)
    decided = und == 0
    assert decided.mean() > 0.9999
    bad = np.nonzero(decided & (g.view(np.int64) != ref.view(np.int64)))[0]
    assert bad.size == 0, (bad[:5], g[bad[:5]], ref[bad[:5]], rows[bad[:5]])
    # an undecided power is still within one ulp of the correctly rounded one
    if (~decided).any():
        assert np.all(np.abs(g[~decided] - ref[~decided]) <= np.spacing(ref[~decided]))
    assert np.all(g[rows[:, 0] == rows[:, 1]] == 1.0)


def test_pow_exact_powers(tmp_path):
    """u^e with an exactly representable result: (2^k)^(-1/2), (2^k)^(-1/4),
    and u^(-1) at powers of two."""
    exe = _driver(tmp_path)
    rows, want = [], []
    for k in range(0, 40, 2):
        u = 2.0 ** k
        for brake, p in ((3.0, -0.5), (5.0, -0.25), (2.0, -1.0)):
            if k % 4 and brake == 5.0:
                continue
            tau = 1000.0
            t = (u - 1.0) * tau                 # u = 1 + t/tau exactly
            rows.append([t, 0.0, tau, brake])
            want.append(u ** p)
    g, und = _run(exe, tmp_path, np.array(rows))
    assert np.array_equal(g, np.array(want))


ERR_DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ddpow.h"
using namespace ltgw;
// rows of (u, e) -> the fast phase's relative error against the double-double
// phase (both unrounded), and whether pow_cr took the slow phase
int main(int argc, char **argv) {
    FILE *fi = std::fopen(argv[1], "rb");
    FILE *fo = std::fopen(argv[2], "wb");
    long n = std::atol(argv[3]);
    std::vector<double> in(2 * n), err(n), g(n), gd(n);
    std::vector<int> slow(n), und(n), undd(n);
    if (std::fread(in.data(), 8, 2 * n, fi) != (size_t)(2 * n)) return 1;
    for (long i = 0; i < n; ++i) {
        const double u = in[2 * i], e = in[2 * i + 1];
        dd R;
        pow_fast_value(u, e, &R);
        dd Rd = dd_exp(dd_mul_d(dd_log(u), e));
        err[i] = ((R.hi - Rd.hi) + (R.lo - Rd.lo)) / Rd.hi;
        g[i] = pow_cr(u, e, &und[i], &slow[i]);
        gd[i] = pow_dd(u, e, &undd[i]);
    }
    std::fwrite(err.data(), 8, n, fo);
    std::fwrite(g.data(), 8, n, fo);
    std::fwrite(gd.data(), 8, n, fo);
    std::fwrite(slow.data(), 4, n, fo);
    std::fwrite(und.data(), 4, n, fo);
    std::fwrite(undd.data(), 4, n, fo);
    return 0;
}
'''


def test_fast_phase_error_bound_and_slow_rate(tmp_path):
    """The fast phase's value (before rounding) against the double-double
    phase over a million (u, e) pairs: u log-uniform in [2^-20, 2^20] and in
    the search's [1, 30], e in [-2, 2]: its relative error stays below 2^-72,
    a quarter of the 2^-70 (1 + |e|) the rounding test assumes (which it
    widens sixteen times); the slow phase is taken for under 0.1% of the
    pairs; and the two-phase power equals the double-double one wherever that
    one decides."""
    src = tmp_path / "err_driver.cpp"
    src.write_text(ERR_DRIVER)
    exe = tmp_path / "err_driver"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    r = np.random.default_rng(43)
    n = 1_000_000
    u = np.where(r.uniform(size=n) < 0.5, np.exp(r.uniform(np.log(2.0 ** -20), np.log(2.0 ** 20), n)),
                 np.exp(r.uniform(0.0, np.log(30.0), n)))
    e = r.uniform(-2.0, 2.0, n)
    e[: n // 2] = 1.0 / (1.0 - r.uniform(1.5, 9.0, n // 2))     # the search's exponents
    rows = np.ascontiguousarray(np.column_stack([u, e]))
    fi, fo = tmp_path / "in.bin", tmp_path / "out.bin"
    rows.tofile(fi)
    subprocess.run([str(exe), str(fi), str(fo), str(n)], check=True)
    raw = np.fromfile(fo, dtype=np.uint8)
    err = raw[:8 * n].view(np.float64)
    g = raw[8 * n:16 * n].view(np.float64)
    gd = raw[16 * n:24 * n].view(np.float64)
    slow = raw[24 * n:28 * n].view(np.int32)
    und = raw[28 * n:32 * n].view(np.int32)
    undd = raw[32 * n:].view(np.int32)
    worst = np.max(np.abs(err) / (1.0 + np.abs(e)))
    print(f"worst fast-phase error {np.log2(worst):.1f} bits, slow phase {slow.mean():.2e}")
    assert worst < 2.0 ** -72
    assert slow.mean() < 1e-3
    assert np.all(und[slow == 0] == 0)
    # the fast phase's decisions are the double-double phase's, bit for bit
    assert not undd.any()
    assert np.array_equal(g.view(np.int64), gd.view(np.int64))


DIV_DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "ddpow.h"
// rows of (x, d) -> 1 where div_rn(x, d, RN(1/d)) differs from x / d
int main(int argc, char **argv) {
    FILE *fi = std::fopen(argv[1], "rb");
    FILE *fo = std::fopen(argv[2], "wb");
    long n = std::atol(argv[3]);
    std::vector<double> in(2 * n);
    std::vector<int> bad(n);
    if (std::fread(in.data(), 8, 2 * n, fi) != (size_t)(2 * n)) return 1;
    for (long i = 0; i < n; ++i) {
        const double x = in[2 * i], d = in[2 * i + 1];
        const double y = 1.0 / d;
        bad[i] = ltgw::div_rn(x, d, y) != x / d;
    }
    std::fwrite(bad.data(), 4, n, fo);
    return 0;
}
'''


def test_div_rn_equals_division(tmp_path):
    """The explicit-template kernel forms (t - T0)/tau and v.n/c from RN(1/tau)
    and RN(1/c) with one FMA correction (Markstein's theorem says the result
    is the correctly rounded quotient).  Checked against the division itself
    over two million quotients of the search's kind: segment times over
    random tau (log-uniform 300 s .. 10^6 s, a seventh of them with an
    all-ones low significand, the hardest reciprocals), random reals over
    random divisors, and velocities over c."""
    src = tmp_path / "div_driver.cpp"
    src.write_text(DIV_DRIVER)
    exe = tmp_path / "div_driver"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    r = np.random.default_rng(47)
    n = 700_000
    tau = np.exp(r.uniform(np.log(300.0), np.log(1e6), n))
    tb = tau.view(np.uint64)
    tb[::7] |= np.uint64(0x000FFFFFFFFFFF00)
    dt = np.floor(r.uniform(0, 10800, n)) * 8.0 + 4.0
    dt[:3] = [0.0, 8.0, 86400.0]
    x2 = r.uniform(-1e5, 1e5, n)
    d2 = np.exp(r.uniform(-30.0, 30.0, n)) * np.where(r.uniform(size=n) < 0.5, -1.0, 1.0)
    vn = r.uniform(-4e4, 4e4, n)
    rows = np.concatenate([np.column_stack([dt, tau]), np.column_stack([x2, d2]),
                           np.column_stack([vn, np.full(n, 299792458.0)])])
    rows = np.ascontiguousarray(rows)
    fi, fo = tmp_path / "in.bin", tmp_path / "out.bin"
    rows.tofile(fi)
    subprocess.run([str(exe), str(fi), str(fo), str(len(rows))], check=True)
    bad = np.fromfile(fo, dtype=np.int32)
    assert bad.size == len(rows)
    assert not bad.any(), rows[np.nonzero(bad)[0][:5]]


ENC_DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "pow_enclose.h"
using namespace ltgw;
// mode 0: rows of (u, e) -> ok, G, y, lo, hi, the double-double value
//   (unrounded), RN(u^e) from the two-phase power and its undecided flag
// mode 1: rows of (u, e, f0, D, t_sft, shift) -> the column by the
//   explicit-template kernel's rule (enclosure, else the double-double power),
//   whether the rule took the double-double power, and the column of the
//   two-phase power's RN(u^e)
static unsigned column(double g, double D, double tsft, double f0, double shift) {
    const double h = g * D;
    const double H = h * tsft;
    const double x = f0 * H;
    const double v = x + shift;
    return (unsigned)(int)v;   // truncation toward zero; the rows keep v in int range
}
int main(int argc, char **argv) {
    int mode = std::atoi(argv[4]);
    if (mode == 2) { std::printf("%a\n", kLn2rn); return 0; }
    FILE *fi = std::fopen(argv[1], "rb");
    FILE *fo = std::fopen(argv[2], "wb");
    long n = std::atol(argv[3]);
    int w = mode == 0 ? 2 : 6;
    std::vector<double> in(w * n);
    if (std::fread(in.data(), 8, w * n, fi) != (size_t)(w * n)) return 1;
    for (long i = 0; i < n; ++i) {
        const double *r = &in[w * i];
        const double u = r[0], e = r[1];
        if (mode == 0) {
            double o[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            double G = 0, y = 0, lo = 0, hi = 0;
            const bool ok = pow_enclose_value(u, e, &G, &y) && pow_enclose(u, e, &lo, &hi);
            int und = 0;
            o[0] = ok; o[1] = G; o[2] = y; o[3] = lo; o[4] = hi;
            if (u > 0 && u < 0x1p1000) {
                const dd Rd = dd_exp(dd_mul_d(dd_log(u), e));
                o[5] = Rd.hi + Rd.lo;
                o[6] = pow_cr(u, e, &und);
            }
            o[7] = und;
            std::fwrite(o, 8, 8, fo);
        } else {
            const double f0 = r[2], D = r[3], tsft = r[4], shift = r[5];
            double lo = 0, hi = 0;
            const bool enc = pow_enclose(u, e, &lo, &hi);
            unsigned idx = column(lo, D, tsft, f0, shift);
            int took = 0;
            if (!enc || column(hi, D, tsft, f0, shift) != idx) {
                idx = column(pow_dd_call(u, e).g, D, tsft, f0, shift);
                took = 1;
            }
            int und = 0;
            const unsigned want = column(pow_cr(u, e, &und), D, tsft, f0, shift);
            int o[4] = {(int)idx, took, (int)want, und};
            std::fwrite(o, 4, 4, fo);
        }
    }
    return 0;
}
'''


def _enc_driver(tmp_path):
    src = tmp_path / "enc_driver.cpp"
    src.write_text(ENC_DRIVER)
    exe = tmp_path / "enc_driver"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    return exe


def _enc_run(exe, tmp_path, rows, mode):
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    fi, fo = tmp_path / "in.bin", tmp_path / "out.bin"
    rows.tofile(fi)
    subprocess.run([str(exe), str(fi), str(fo), str(len(rows)), str(mode)], check=True)
    return np.fromfile(fo, dtype=np.float64 if mode == 0 else np.int32).reshape(len(rows), -1)


def test_power_enclosure_error_bound_and_containment(tmp_path):
    """The enclosure the explicit-template kernel takes in place of RN(u^e)
    (Eq. 1), over 1.2 million (u, e) pairs: u log-uniform in [1, 2^20], just
    above 1 (down to 1 + 2^-52), at both ends of every log-table interval at
    several binades, and the search's 1 + (t - T0)/tau; e the search's
    1/(1 - n) and uniform in [-20, 20].  Its value G stays within the stated
    2^-50 (1 + |y| + |e|) of u^e (the double-double value; the worst case
    seen is printed); the interval holds the correctly rounded power every
    time; it declines outside u >= 1 and -600 < e log u < 700.  ln 2's
    constant is the nearest double (60-digit decimal arithmetic)."""
    from decimal import Decimal, getcontext

    exe = _enc_driver(tmp_path)
    getcontext().prec = 60
    got = subprocess.run([str(exe), "-", "-", "0", "2"], capture_output=True, text=True, check=True).stdout
    assert float.fromhex(got.strip()) == float(Decimal(2).ln())

    r = np.random.default_rng(53)
    n = 200_000
    parts = [np.exp(r.uniform(0.0, np.log(2.0 ** 20), n)),
             1.0 + np.floor(r.uniform(0, 4096, n)) * 2.0 ** -52,
             1.0 + r.uniform(0.0, 2.0 ** -20, n),
             1.0 + np.floor(r.uniform(0, 10800, n)) * 8.0 / np.exp(r.uniform(np.log(300.0), np.log(40000.0), n))]
    ends = []
    for i in range(128):
        for k in (0, 1, 5, 13):
            lo = (1.0 + i / 128.0) * 2.0 ** k
            hi = (1.0 + (i + 1) / 128.0) * 2.0 ** k
            ends += [lo, np.nextafter(lo, np.inf), np.nextafter(hi, 0.0), (lo + hi) / 2]
    ends = np.array(ends)
    u = np.concatenate(parts + [np.tile(ends, 40)])
    m = len(u)
    e = np.where(r.uniform(size=m) < 0.5, 1.0 / (1.0 - r.uniform(1.5, 9.0, m)), r.uniform(-20.0, 20.0, m))
    e[:50] = [-0.5, -0.25, -1.0, -2.0, 0.5] * 10
    out = _enc_run(exe, tmp_path, np.column_stack([u, e]), 0)
    ok, G, y, lo, hi, gd, gcr, und = out.T
    ok = ok.astype(bool)
    inside = (np.abs(e * np.log(u)) < 590.0)
    assert np.all(ok[inside])
    rel = np.abs(G[ok] - gd[ok]) / gd[ok] / (1.0 + np.abs(y[ok]) + np.abs(e[ok]))
    print(f"worst enclosure error {np.log2(rel.max()):.2f} bits of (1 + |y| + |e|), over {ok.sum()} pairs")
    assert rel.max() < 2.0 ** -50
    dec = ok & (und == 0)
    assert np.all(lo[dec] <= gcr[dec]) and np.all(gcr[dec] <= hi[dec])
    # the domain
    bad_u = np.array([0.5, 1.0 - 2.0 ** -53, 0.0, -1.0, np.inf, np.nan, 2.0 ** 1000, 1.0])
    bad_e = np.array([-0.5, -0.5, -0.5, -0.5, -0.5, -0.5, -0.5, np.nan])
    far = np.array([[2.0 ** 900, 2.0], [2.0 ** 900, -2.0], [30.0, 300.0], [30.0, -300.0]])
    out = _enc_run(exe, tmp_path, np.concatenate([np.column_stack([bad_u, bad_e]), far]), 0)
    assert not out[:, 0].any()


def test_column_decision_by_enclosure_equals_correct_rounding(tmp_path):
    """The explicit-template kernel's column rule (the column at both ends of
    the enclosure, else the double-double power) against the column of the
    correctly rounded power, over 2.2 million evaluations of the realistic
    search's kind (f0 500-1500 Hz, T_sft = 4 s, Doppler factors 1 +- 1e-4,
    tau 300-40000 s, n 1.5-9), a fifth of them placed within 1e-9 bins of a
    column boundary so that the rule has to fall back: identical columns
    everywhere, and the fallback taken only near boundaries."""
    exe = _enc_driver(tmp_path)
    r = np.random.default_rng(59)
    n = 2_200_000
    tau = np.exp(r.uniform(np.log(300.0), np.log(40000.0), n))
    dt = np.floor(r.uniform(0, 10800, n)) * 8.0
    u = 1.0 + dt / tau
    e = 1.0 / (1.0 - r.uniform(1.5, 9.0, n))
    f0 = r.uniform(500.0, 1500.0, n)
    D = 1.0 + r.uniform(-1e-4, 1e-4, n)
    tsft = np.full(n, 4.0)
    shift = np.full(n, 1.5 - 1900.0)
    near = r.uniform(size=n) < 0.2
    # move f0 so that f0 g D T_sft + shift lies within 1e-9 of an integer
    g = u ** e
    x = f0 * g * D * tsft + shift
    target = np.round(x) + r.uniform(-1e-9, 1e-9, n)
    f0 = np.where(near, (target - shift) / (g * D * tsft), f0)
    out = _enc_run(exe, tmp_path, np.column_stack([u, e, f0, D, tsft, shift]), 1)
    idx, took, want, und = out.T
    assert not und.any()
    assert np.array_equal(idx, want)
    print(f"fallback: {took[near].mean():.3f} of the near-boundary rows, {took[~near].sum()} of the others")
    assert took[near].mean() > 0.5
    assert took[~near].sum() <= 2
