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
