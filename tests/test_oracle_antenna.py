"""Pins of the oracle's antenna response (the weighting of Sec. 2) and of the
statistic weighted by it.

The response F+^2 + Fx^2 of an interferometer is fixed by geometry:
- arms along x and y, a wave from the zenith (or nadir): 1; from along an
  arm: 1/4; from the in-plane bisector: 0;
- averaged over the sky, 2/5 sin^2(zeta) for arms at an angle zeta (2/5 for
  perpendicular arms);
- unchanged by n -> -n, by swapping the arms, and by turning the detector and
  the direction together about the rotation axis (the Earth rotation angle).
The weighted statistic: a source at the zenith of a detector whose arms lie in
the equatorial plane gets weight w_j (response 1); a source along an arm at
rotation angle 0 gets w_j / 4, so s and W1 scale by 1/4 and W2 by 1/16
exactly, and Psi of the power is unchanged.
"""
import math

import numpy as np
import pytest

import oracle
import synth

XY = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]]
S2 = 1.0 / math.sqrt(2.0)


@pytest.mark.parametrize("era,n,want", [
    (0.0, [0, 0, 1], 1.0), (0.0, [0, 0, -1], 1.0), (1.234, [0, 0, 1], 1.0),
    (0.0, [1, 0, 0], 0.25), (0.0, [0, 1, 0], 0.25), (0.0, [S2, S2, 0], 0.0),
    (math.pi / 2, [0, 1, 0], 0.25), (math.pi / 4, [S2, S2, 0], 0.25), (math.pi / 4, [S2, -S2, 0], 0.25),
    (math.pi / 4, [1, 0, 0], 0.0),
])
def test_antenna_closed_forms(era, n, want):
    assert oracle.antenna(XY, era, n) == pytest.approx(want, abs=1e-15)


@pytest.mark.parametrize("zeta_deg", [90.0, 60.0, 30.0])
def test_antenna_sky_average(zeta_deg):
    z = math.radians(zeta_deg)
    arms = [[1.0, 0.0, 0.0], [math.cos(z), math.sin(z), 0.0]]
    pts = synth.fibonacci_cap(40000, [0.0, 0.0, 1.0], math.pi)
    vals = np.array([oracle.antenna(arms, 0.3, p) for p in pts])
    assert vals.mean() == pytest.approx(0.4 * math.sin(z) ** 2, abs=2e-4)
    assert vals.min() >= -1e-15 and vals.max() <= math.sin(z) ** 2 + 1e-12


def test_antenna_symmetries():
    r = np.random.default_rng(43)
    for _ in range(200):
        a = r.normal(size=3)
        a /= np.linalg.norm(a)
        b = np.cross(a, r.normal(size=3))
        b /= np.linalg.norm(b)
        n = r.normal(size=3)
        n /= np.linalg.norm(n)
        era = r.uniform(-7.0, 7.0)
        base = oracle.antenna([a, b], era, n)
        c, s = math.cos(-era), math.sin(-era)
        n_back = np.array([c * n[0] - s * n[1], s * n[0] + c * n[1], n[2]])
        assert oracle.antenna([a, b], 0.0, n_back) == pytest.approx(base, abs=1e-13)
        assert oracle.antenna([a, b], era, -n) == pytest.approx(base, abs=1e-13)
        assert oracle.antenna([b, a], era, n) == pytest.approx(base, abs=1e-13)
        assert -1e-15 <= base <= 1.0 + 1e-12


def _det(arms=None, era=None, seed=44, n_seg=64, n_bins=200):
    r = np.random.default_rng(seed)
    t = np.arange(n_seg) * 120.0 + 4.0
    v = r.normal(size=(n_seg, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * 3.0e4
    rho = r.exponential(size=(n_seg, n_bins)).astype(np.float32)
    w = r.uniform(0.5, 2.0, n_seg).astype(np.float32)
    return oracle.Detector(rho, t, v, 1900, 4.0, weights=w, arms=arms, era=era)


def test_statistic_zenith_source_equals_plain_weights():
    era = synth.earth_rotation_angle(np.arange(64) * 120.0 + 4.0)
    plain = _det()
    ant = _det(arms=XY, era=era)
    g = oracle.Grid(477.0, 0.25, 120, [3000.0, 20000.0], [3.0, 5.0], [[0.0, 0.0, 1.0]])
    a, b = oracle.evaluate(plain, g), oracle.evaluate(ant, g)
    assert np.array_equal(a["c"], b["c"]) and np.array_equal(a["N"], b["N"])
    for k in ("s", "W1", "W2"):
        assert np.allclose(b[k], a[k], rtol=1e-14, atol=0.0), k
    assert (a["N"] > 0).sum() > 100


def test_statistic_source_along_an_arm_scales_exactly():
    plain = _det(seed=45)
    ant = _det(arms=XY, era=np.zeros(64), seed=45)
    g = oracle.Grid(477.0, 0.25, 120, [3000.0, 20000.0], [3.0, 5.0], [[1.0, 0.0, 0.0]])
    a, b = oracle.evaluate(plain, g), oracle.evaluate(ant, g)
    assert np.array_equal(a["c"], b["c"]) and np.array_equal(a["N"], b["N"])
    assert np.array_equal(b["s"], 0.25 * a["s"])
    assert np.array_equal(b["W1"], 0.25 * a["W1"])
    assert np.array_equal(b["W2"], a["W2"] / 16.0)
    pa, pb = oracle.psi_power(a), oracle.psi_power(b)
    assert np.array_equal(np.isnan(pa), np.isnan(pb))
    ok = ~np.isnan(pa)
    assert np.allclose(pa[ok], pb[ok], rtol=1e-12, atol=1e-12)


def test_explicit_templates_with_antenna_equal_the_lattice():
    arms = synth.site_arms(*synth.SITE_L, synth.ARM_AZ_L)
    t = np.arange(64) * 120.0 + 4.0
    det = _det(arms=arms, era=synth.earth_rotation_angle(t), seed=46)
    g = oracle.Grid(477.0, 0.25, 60, [3000.0, 20000.0], [3.0, 5.0],
                    [[0.6, 0.0, 0.8], synth.sky_vector(2.0, -0.4)], 100.0)
    res = oracle.evaluate(det, g)
    f0, tau, brake, isky = g.params(np.arange(g.n_templates))
    lst = oracle.evaluate_params(det, np.column_stack([f0, tau, brake, g.sky[isky]]), t0=g.t0)
    for k in ("s", "c", "N", "W1", "W2"):
        assert np.array_equal(lst[k], res[k]), k
    plain = oracle.evaluate(_det(seed=46), g)
    assert not np.allclose(plain["s"], res["s"])
