"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: exact
special cases of Eq. 1 and Eq. 2, the exact-real bin from rational/decimal
arithmetic (tests/truth.py), closed-form sums on constructed spectrograms
(single hot pixel, constant, bin checksum, noiseless injection), linearity,
the noise moments behind Eq. 4, a library sort for the ranking and torch's
format conversions for the storage formats.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import truth

C = oracle.C_LIGHT
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_det(seed=0, n_seg=8, n_bins=256, k_lo=1900, t_sft=4.0, vmag=3.0e5, rho=None,
              weights=None, t_seg=None, values=None):
    rng = np.random.default_rng(seed)
    if t_seg is None:
        t_seg = np.arange(n_seg) * 300.0 + 2.0
    v = rng.normal(size=(n_seg, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * vmag
    if rho is None:
        rho = np.zeros((n_seg, n_bins), np.float32)
    return oracle.Detector(rho, t_seg, v, k_lo, t_sft, weights=weights, values=values)


def small_grid(n_f0=24, f0_min=478.0, f0_step=2.625, t0=0.0):
    sky = np.array([[0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])
    return oracle.Grid(f0_min, f0_step, n_f0, [5000.0, 20000.0], [3.0, 5.0], sky, t0)


def truth_bins(det, grid):
    """[n_templates, n_seg] exact-real columns and the smallest tie margin."""
    out = np.empty((grid.n_templates, det.n_seg), np.int64)
    margin = np.inf
    for t in range(grid.n_templates):
        f0, tau, brake, isky = grid.params(t)
        for j in range(det.n_seg):
            if det.t_seg[j] < grid.t0:
                out[t, j] = np.iinfo(np.int64).min
                continue
            b, m = truth.true_bin(float(f0), det.t_seg[j], grid.t0, tau, brake, det.v[j],
                                  grid.sky[isky], det.t_sft, det.k_lo)
            out[t, j] = b
            margin = min(margin, m)
    return out, margin


def in_band(b, n_bins):
    return (b >= 0) & (b < n_bins)


# ---------------------------------------------------------------- Eq. 1 -----
def test_golden_closed_forms():
    """Exact values of Eq. 1 where the power is exact: u = 1 (t = T0) gives 1;
    n = 5, u = 16 and n = 3, u = 4 give 1/2; n = 2, u = 4 gives 1/4."""
    with open(os.path.join(GOLDEN, "spin_factor_closed_forms.json")) as fh:
        cases = json.load(fh)["cases"]
    assert len(cases) >= 5
    for c in cases:
        g = oracle.spin_factor(c["t"], c["t0"], c["tau"], c["brake"])
        assert g == c["g"], c


def test_spin_factor_correctly_rounded_vs_decimal():
    """g = RN(u^e) for the FP64 u and e (Eq. 1), checked against a 50-digit
    decimal power rounded once, over the parameter ranges of the paper
    (tau 3500-35000 s, n 3-7) and two days of segment times."""
    rng = np.random.default_rng(11)
    ns = list(np.linspace(3.0, 7.0, 9)) + list(rng.uniform(3.0, 7.0, 8))
    for k in range(240):
        t = float(rng.uniform(0.0, 2.0e5))
        t0 = float(rng.choice([0.0, 17.0, 1234.5]))
        tau = float(np.exp(rng.uniform(np.log(3500.0), np.log(35000.0))))
        n = float(ns[k % len(ns)])
        if t < t0:
            continue
        u = 1.0 + (t - t0) / tau
        e = 1.0 / (1.0 - n)
        assert oracle.spin_factor(t, t0, tau, n) == truth.correctly_rounded_pow(u, e)


def test_masked_before_t0():
    assert oracle.spin_factor(99.0, 100.0, 3500.0, 5.0) == 0.0


# ---------------------------------------------------------------- Eq. 2 -----
def test_doppler_exact_cases():
    """D = 1 + v.n/c (Eq. 2): v = c 2^-13 along n gives exactly 1 + 2^-13, the
    opposite direction 1 - 2^-13, each axis separately, orthogonal gives 1."""
    a = C * 2.0 ** -13
    e = 2.0 ** -13
    assert oracle.doppler([a, 0, 0], [1, 0, 0]) == 1.0 + e
    assert oracle.doppler([a, 0, 0], [-1, 0, 0]) == 1.0 - e
    assert oracle.doppler([0, a, 0], [0, 1, 0]) == 1.0 + e
    assert oracle.doppler([0, 0, 2 * a], [0, 0, -1]) == 1.0 - 2 * e
    assert oracle.doppler([a, 0, 0], [0, 1, 0]) == 1.0
    assert oracle.doppler([0, a, 0], [1, 0, 0]) == 1.0


# ---------------------------------------------------------------- bins ------
def test_bin_ties_go_up_and_exact_track():
    """x = f0 T_sft exactly at t = T0 with v = 0: 500.125 * 4 = 2000.5 -> 2001;
    at u = 16, n = 5 the track is f0/2 exactly: 550.25 * 4 / 2 = 1100.5 -> 1101."""
    assert oracle.bin_index(500.125, 1.0, 1.0, 4.0, 0) == 2001
    assert oracle.bin_index(500.0, 1.0, 1.0, 4.0, 1600) == 400
    g = oracle.spin_factor(15 * 512.0, 0.0, 512.0, 5.0)
    assert g == 0.5
    assert oracle.bin_index(550.25, g, 1.0, 4.0, 0) == 1101
    assert oracle.bin_index(550.0, g, 1.0, 4.0, 1000) == 100


def test_bins_are_nearest_to_exact_frequency():
    """Every oracle column equals the nearest bin of the exact-real Doppler-shifted
    track (Eqs. 1-2) unless the exact x lies within 1e-9 of a half-integer."""
    det = small_det(seed=3)
    grid = small_grid()
    tb, margin = truth_bins(det, grid)
    assert margin > 1e-9
    for t in range(grid.n_templates):
        f0, tau, brake, isky = grid.params(t)
        ob = oracle.track_bins(det, float(f0), tau, brake, grid.sky[isky], grid.t0)
        assert np.array_equal(ob, tb[t]), t


# --------------------------------------------------------- the statistic ---
def test_single_hot_pixel_point_transform():
    """rho = 1 at one pixel: s = w_j* exactly for the templates whose track
    selects that pixel and 0 for all others (Sec. 2, sum over selected bins)."""
    det0 = small_det(seed=5)
    grid = small_grid()
    tb, _ = truth_bins(det0, grid)
    w = np.linspace(0.5, 2.0, det0.n_seg).astype(np.float32)
    hits = 0
    ib = in_band(tb, det0.n_bins)
    picks = [(j, int(tb[t, j])) for (t, j) in [(5, 0), (30, 3), (61, 6), (90, 7)] if ib[t, j]]
    assert len(picks) >= 3
    for (js, bs) in picks + [(2, 0), (4, 255)]:
        rho = np.zeros((det0.n_seg, det0.n_bins), np.float32)
        rho[js, bs] = 1.0
        det = oracle.Detector(rho, det0.t_seg, det0.v, det0.k_lo, det0.t_sft, weights=w)
        res = oracle.evaluate(det, grid)
        expect = np.where(tb[:, js] == bs, np.float64(w[js]), 0.0)
        hits += int((tb[:, js] == bs).sum())
        assert np.array_equal(res["s"], expect)
        assert np.all(res["c"] == 0)
    assert hits > 0


def test_constant_spectrogram_gives_in_band_counts():
    """rho = 1 everywhere: s = W1 = sum of in-band weights, N = in-band count,
    W2 = sum of squared in-band weights; no pixel exceeds 1.6."""
    det0 = small_det(seed=6)
    grid = small_grid()
    tb, _ = truth_bins(det0, grid)
    w = np.array([0.5, 1.0, 2.0, 1.5, 0.75, 1.25, 1.0, 0.5], np.float32)
    det = oracle.Detector(np.ones((det0.n_seg, det0.n_bins), np.float32), det0.t_seg, det0.v,
                          det0.k_lo, det0.t_sft, weights=w)
    res = oracle.evaluate(det, grid)
    ib = in_band(tb, det.n_bins)
    assert np.array_equal(res["N"], ib.sum(axis=1))
    assert np.allclose(res["W1"], (ib * w.astype(np.float64)).sum(axis=1), rtol=0, atol=1e-12)
    assert np.allclose(res["W2"], (ib * w.astype(np.float64) ** 2).sum(axis=1), rtol=0, atol=1e-12)
    assert np.array_equal(res["s"], res["W1"])
    assert np.all(res["c"] == 0)
    assert 0 < ib.mean() < 1  # both in-band and out-of-band cases occur


def test_bin_checksum_pins_every_bin():
    """rho[j, b] = b: s = sum of the selected columns, exact in FP64."""
    det0 = small_det(seed=7)
    grid = small_grid()
    tb, _ = truth_bins(det0, grid)
    rho = np.tile(np.arange(det0.n_bins, dtype=np.float32), (det0.n_seg, 1))
    det = oracle.Detector(rho, det0.t_seg, det0.v, det0.k_lo, det0.t_sft)
    res = oracle.evaluate(det, grid)
    ib = in_band(tb, det.n_bins)
    assert np.array_equal(res["s"], np.where(ib, tb, 0).sum(axis=1).astype(np.float64))
    # columns above 1.6 are counted: every selected b >= 2
    assert np.array_equal(res["c"], (ib & (tb >= 2)).sum(axis=1))


def test_noiseless_injection_recovers_its_power():
    """A track of amplitude A*w_j on an empty spectrogram: the injected template
    sums to A * sum(w_j) over its in-band segments, counts those whose injected
    power exceeds 1.6, and no other template exceeds its sum."""
    det0 = small_det(seed=8)
    grid = small_grid()
    tb, _ = truth_bins(det0, grid)
    w = np.linspace(0.5, 2.0, det0.n_seg).astype(np.float32)
    tpl = 7 + grid.n_f0 * 2  # some on-grid template with in-band segments
    assert in_band(tb[tpl], det0.n_bins).sum() >= 3
    A = np.float32(2.5)
    rho = np.zeros((det0.n_seg, det0.n_bins), np.float32)
    for j, b in enumerate(tb[tpl]):
        if 0 <= b < det0.n_bins:
            rho[j, b] += A * w[j]
    det = oracle.Detector(rho, det0.t_seg, det0.v, det0.k_lo, det0.t_sft, weights=w)
    res = oracle.evaluate(det, grid)
    ib = in_band(tb[tpl], det0.n_bins)
    expect = sum(float(w[j]) * float(np.float32(A * w[j])) for j in range(det0.n_seg) if ib[j])
    assert res["s"][tpl] == pytest.approx(expect, rel=1e-15)
    above = [ib[j] and np.float32(A * w[j]) > np.float32(1.6) for j in range(det0.n_seg)]
    assert res["N"][tpl] == ib.sum()
    assert res["c"][tpl] == sum(above) < ib.sum()
    assert res["s"].max() == res["s"][tpl]


def test_linearity():
    det0 = small_det(seed=9)
    grid = small_grid()
    r = np.random.default_rng(1)
    v1 = r.exponential(size=(det0.n_seg, det0.n_bins))
    v2 = r.exponential(size=(det0.n_seg, det0.n_bins))
    mk = lambda vals: oracle.Detector(vals.astype(np.float32), det0.t_seg, det0.v, det0.k_lo,
                                      det0.t_sft, values=vals)
    s1 = oracle.evaluate(mk(v1), grid)["s"]
    s2 = oracle.evaluate(mk(v2), grid)["s"]
    s12 = oracle.evaluate(mk(2.5 * v1 - 0.75 * v2), grid)["s"]
    assert np.allclose(s12, 2.5 * s1 - 0.75 * s2, rtol=1e-13, atol=1e-12)


def test_count_threshold_is_strict_fp32():
    """rho exactly equal to the FP32 threshold is not counted; the next float up is."""
    det0 = small_det(seed=10)
    grid = small_grid()
    th = np.float32(1.6)
    for val, counted in [(th, False), (np.nextafter(th, np.float32(2)), True)]:
        rho = np.full((det0.n_seg, det0.n_bins), val, np.float32)
        det = oracle.Detector(rho, det0.t_seg, det0.v, det0.k_lo, det0.t_sft)
        res = oracle.evaluate(det, grid)
        assert np.array_equal(res["c"], res["N"] if counted else np.zeros_like(res["c"]))


def test_segments_before_t0_are_masked():
    det = small_det(seed=12, rho=np.random.default_rng(2).exponential(size=(8, 256)).astype(np.float32))
    t0 = float(det.t_seg[3] + 1.0)
    grid = small_grid(t0=t0)
    full = oracle.evaluate(det, grid)
    keep = slice(4, 8)
    tail = oracle.Detector(det.rho[keep], det.t_seg[keep], det.v[keep], det.k_lo, det.t_sft)
    part = oracle.evaluate(tail, grid)
    for k in ("s", "c", "N", "W1", "W2"):
        assert np.array_equal(full[k], part[k])


def test_two_detectors_add():
    r = np.random.default_rng(3)
    d1 = small_det(seed=13, rho=r.exponential(size=(8, 256)).astype(np.float32))
    d2 = small_det(seed=14, rho=r.exponential(size=(8, 256)).astype(np.float32), k_lo=1890)
    grid = small_grid()
    a, b, ab = oracle.evaluate(d1, grid), oracle.evaluate(d2, grid), oracle.evaluate([d1, d2], grid)
    for k in ("c", "N"):
        assert np.array_equal(ab[k], a[k] + b[k])
    assert np.allclose(ab["s"], a["s"] + b["s"], rtol=1e-14)


# ---------------------------------------------------------------- Eq. 4 -----
def test_psi_closed_forms():
    res = {"s": np.array([110.0, 100.0, 7.0]), "c": np.array([30, 20, 0], np.int32),
           "N": np.array([100, 100, 0], np.int32), "W1": np.array([100.0, 100.0, 0.0]),
           "W2": np.array([100.0, 100.0, 0.0])}
    p = oracle.psi_power(res)
    assert p[0] == 1.0 and p[1] == 0.0 and math.isnan(p[2])
    q = math.exp(-float(np.float32(1.6)))
    pc = oracle.psi_count(res)
    assert pc[0] == pytest.approx((30 - 100 * q) / math.sqrt(100 * q * (1 - q)), rel=1e-15)
    assert math.isnan(pc[2])


def test_psi_is_standardised_under_noise():
    """Under Exp(1) noise the critical ratios of Eq. 4 have mean 0 and
    variance 1, for the weighted power sum and for the number count."""
    det0 = small_det(seed=15, n_seg=48, n_bins=96, k_lo=1960, t_seg=np.arange(48) * 8.0 + 4.0)
    grid = oracle.Grid(492.0, 1.25, 8, [20000.0], [5.0], [[0.6, 0.0, 0.8]])
    w = np.random.default_rng(4).uniform(0.5, 2.0, det0.n_seg).astype(np.float32)
    R = 1500
    pp, pc = [], []
    for r in range(R):
        rho = np.random.default_rng(1000 + r).exponential(size=(det0.n_seg, det0.n_bins)).astype(np.float32)
        det = oracle.Detector(rho, det0.t_seg, det0.v, det0.k_lo, det0.t_sft, weights=w)
        res = oracle.evaluate(det, grid)
        assert np.all(res["N"] > 20)
        pp.append(oracle.psi_power(res))
        pc.append(oracle.psi_count(res))
    for arr in (np.array(pp), np.array(pc)):
        m, v = arr.mean(axis=0), arr.var(axis=0)
        assert np.all(np.abs(m) < 4.5 / math.sqrt(R)), m
        assert np.all(np.abs(v - 1.0) < 0.16), v


# --------------------------------------------------------------- ranking ----
def test_topk_order_matches_sorted():
    r = np.random.default_rng(5)
    psi = np.round(r.normal(size=500), 1)  # many exact ties
    psi[r.integers(0, 500, 40)] = np.nan
    psi[17] = -0.0
    psi[18] = 0.0
    ref = sorted((i for i in range(500) if not math.isnan(psi[i])), key=lambda i: (-psi[i], i))
    for k in (1, 10, 64, 460, 600):
        assert list(oracle.topk(psi, k)) == ref[:k]


# ------------------------------------------------------- storage formats ----
def test_bf16_matches_torch_rne():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(6)
    bits = np.concatenate([r.integers(0, 2 ** 32, 1 << 20, dtype=np.uint64),
                           np.arange(0x3f7f0000, 0x3f810000, dtype=np.uint64)]).astype(np.uint32)
    x = bits.view(np.float32)
    x = x[np.isfinite(x)]
    ours = oracle.bf16_rne(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_e4m3_matches_torch_and_saturates():
    torch = pytest.importorskip("torch")
    r = np.random.default_rng(7)
    x = np.concatenate([r.uniform(-460, 460, 200000), r.exponential(size=100000) * 0.01,
                        np.array([0.0, -0.0, 448.0, -448.0, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10, 0.0029296875])]
                       ).astype(np.float32)
    x = x[np.abs(x) <= 448.0]
    ours = oracle.e4m3_rne_sat(x)
    ref = torch.from_numpy(x.copy()).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)
    big = np.array([449.0, 464.0, 1e6, -500.0], np.float32)
    assert list(oracle.e4m3_rne_sat(big)) == [0x7e, 0x7e, 0x7e, 0xfe]
    assert oracle.e4m3_decode(0x7e) == 448.0 and oracle.e4m3_decode(0x01) == 2.0 ** -9


def test_dequantised_fp8_scale():
    rho = np.array([[0.0, 0.0], [1.0, 448.0 * 3]], np.float32)
    vals, sc = oracle.dequantised(rho, "fp8")
    assert sc[0] == 1.0 and sc[1] == np.float32(448.0 * 3) / np.float32(448.0)
    assert vals[1, 1] == 448.0 * 3 and vals[0, 0] == 0.0


# ------------------------------------------------ explicit templates (Sec. 2) ---
def _random_params(rng, n, sky=None):
    """(f0, tau, n, sky) drawn uniformly over ranges around the small grid's."""
    out = np.empty((n, 6))
    out[:, 0] = rng.uniform(478.0, 540.0, n)
    out[:, 1] = np.exp(rng.uniform(math.log(3500.0), math.log(35000.0), n))
    out[:, 2] = rng.uniform(3.0, 7.0, n)
    s = rng.normal(size=(n, 3)) if sky is None else np.tile(sky, (n, 1))
    out[:, 3:] = s / np.linalg.norm(s, axis=1, keepdims=True)
    return out


def test_explicit_templates_bin_checksum_against_exact_tracks():
    """Random (f0, tau, n, sky) off any lattice, on rho[j, b] = b: the power sum
    is the sum of the exact-real in-band columns of each template's track."""
    det0 = small_det(seed=17)
    rng = np.random.default_rng(18)
    params = _random_params(rng, 40)
    rho = np.tile(np.arange(det0.n_bins, dtype=np.float32), (det0.n_seg, 1))
    det = oracle.Detector(rho, det0.t_seg, det0.v, det0.k_lo, det0.t_sft)
    res = oracle.evaluate_params(det, params, t0=0.0)
    n_in = 0
    for q in range(len(params)):
        cols = []
        for j in range(det.n_seg):
            b, _ = truth.true_bin(float(params[q, 0]), det.t_seg[j], 0.0, params[q, 1], params[q, 2], det.v[j],
                                  params[q, 3:], det.t_sft, det.k_lo)
            if 0 <= b < det.n_bins:
                cols.append(b)
        n_in += len(cols)
        assert res["s"][q] == float(sum(cols))
        assert res["N"][q] == len(cols)
    assert n_in > 100


def test_explicit_templates_equal_the_lattice_on_lattice_points():
    """A template given by its parameters evaluates exactly as the same lattice
    template (noise, weights, two masked segments)."""
    det = small_det(seed=19, rho=np.random.default_rng(20).exponential(size=(8, 256)).astype(np.float32),
                    weights=np.linspace(0.5, 2.0, 8).astype(np.float32),
                    t_seg=np.arange(8) * 300.0 - 298.0)
    grid = small_grid(t0=100.0)
    res = oracle.evaluate(det, grid)
    f0, tau, brake, isky = grid.params(np.arange(grid.n_templates))
    params = np.column_stack([f0, tau, brake, grid.sky[isky]])
    lst = oracle.evaluate_params(det, params, t0=grid.t0)
    for k in ("s", "c", "N", "W1", "W2"):
        assert np.array_equal(lst[k], res[k]), k
    assert (res["N"] > 0).sum() > 10
