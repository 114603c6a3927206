"""Host logic of the sensitivity campaign (Sec. 3, Figs. 3-4) and its oracle.

- The efficiency fit: on exact logistic efficiencies both the library's
  Newton fit and the oracle's general-purpose minimiser return the curve's
  (mu, sigma) and A90 = exp(mu + sigma ln 9); on a binomial sample they agree.
- The close neighbourhood: the library's lattice region (nearest grid point
  +-2 f0, +-1 tau in log, +-1 n) and random-bank box equal the oracle's
  direct scans, for random injections including ones at the grid's edges.
- The oracle's realisation adds A * w_j in FP32 at exactly the track's bins.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import campaign as oc
from paper_2507_07816_amd import campaign as pc
from paper_2507_07816_amd.proposer import close_region


@pytest.mark.parametrize("mu,sigma", [(math.log(2.5), 0.3), (0.1, 0.05), (1.5, 0.8)])
def test_fits_recover_exact_logistic(mu, sigma):
    amps = np.exp(mu + sigma * np.linspace(-3, 3, 7))
    n = np.full(7, 1.0e6)
    k = n / (1.0 + np.exp(-(np.log(amps) - mu) / sigma))
    for fit in (pc.fit_logistic(amps, k, n), oc.fit_logistic(amps, k, n)):
        assert fit["mu"] == pytest.approx(mu, abs=1e-6)
        assert fit["sigma"] == pytest.approx(sigma, rel=1e-6)
        assert fit["a90"] == pytest.approx(math.exp(mu + sigma * math.log(9.0)), rel=1e-6)


def test_fits_agree_on_a_binomial_sample():
    r = np.random.default_rng(51)
    amps = np.array([1.0, 1.5, 2.0, 3.0, 4.5, 6.0])
    n = np.full(6, 64)
    k = r.binomial(n, 1.0 / (1.0 + np.exp(-(np.log(amps) - 0.9) / 0.35)))
    a, b = pc.fit_logistic(amps, k, n), oc.fit_logistic(amps, k, n)
    assert a["mu"] == pytest.approx(b["mu"], abs=1e-5)
    assert a["sigma"] == pytest.approx(b["sigma"], rel=1e-5)


def fits_agree(a, b, amps_rel=1e-4):
    """Same case (separable / not rising) and, where A90 is meaningful (a rising
    curve with sigma < 10 in ln A), the same A90; a separable step is the same
    midpoint."""
    if a["separable"] != b["separable"]:
        return False
    if a["separable"]:
        return a["a90"] == pytest.approx(b["a90"], rel=1e-12)
    meaningful = lambda f: f["rising"] and f["sigma"] < 10
    if not (meaningful(a) or meaningful(b)):
        return True
    return a["rising"] and b["rising"] and abs(a["a90"] - b["a90"]) <= amps_rel * b["a90"]


def test_fits_agree_over_small_samples():
    """Random outcome patterns (including separable, flat and decreasing ones)
    of 4 levels x 6 and 6 levels x 8 injections."""
    r = np.random.default_rng(57)
    for amps, per in (([1.0, 2.0, 3.5, 6.0], 6), ([1.0, 1.5, 2.0, 2.5, 3.0, 4.0], 8)):
        n = np.full(len(amps), per)
        for _ in range(150):
            k = r.integers(0, per + 1, len(amps))
            a, b = pc.fit_logistic(amps, k, n), oc.fit_logistic(amps, k, n)
            assert fits_agree(a, b), (k, a, b)
    sep = pc.fit_logistic([1.0, 2.0, 4.0], [0, 3, 6], [6, 6, 6])
    assert sep["separable"] and sep["a90"] == pytest.approx(2.0)
    assert pc.fit_logistic([1.0, 2.0, 4.0], [0, 0, 6], [6, 6, 6])["a90"] == pytest.approx(math.sqrt(8.0))
    assert not pc.fit_logistic([1.0, 2.0, 4.0], [6, 4, 1], [6, 6, 6])["rising"]


def _grid():
    wl = synth.tiny()
    g = wl.grid
    return g, oracle.Grid(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])


def _rows_set(rows):
    return sorted(tuple(np.round(r, 12)) for r in rows)


def test_lattice_region_equals_oracle_scan():
    g, og = _grid()
    r = np.random.default_rng(52)
    injs = [(500.1, 3000.0, 2.0), (599.9, 40000.0, 8.0), (550.0, 7000.0, 5.0), (500.0, 3500.0, 3.0)]
    injs += [(r.uniform(495, 605), math.exp(r.uniform(math.log(3000), math.log(40000))), r.uniform(2.5, 7.5))
             for _ in range(40)]
    for inj in injs:
        idx = close_region(g, np.asarray([inj]))[0]
        got = pc.lattice_params(g, idx[idx >= 0])
        want = oc.lattice_region(og, inj)
        assert _rows_set(got) == _rows_set(want), inj
        f0, tau, brake, isky = og.params(idx[idx >= 0])
        assert np.array_equal(got[:, 0], f0) and np.array_equal(got[:, 1], tau)


def test_bank_region_equals_oracle_scan():
    g, og = _grid()
    bank = synth.random_bank(3000, (500.0, 600.0), (3500.0, 35000.0), (3.0, 7.0), g["sky"][0], seed=53)
    r = np.random.default_rng(54)
    for _ in range(40):
        inj = (r.uniform(500, 600), math.exp(r.uniform(math.log(3500), math.log(35000))), r.uniform(3, 7))
        got = bank[pc.random_bank_region(bank, g, inj)]
        want = oc.bank_region(bank, og, inj)
        assert _rows_set(got) == _rows_set(want)
    assert len(pc.random_bank_region(bank, g, (550.0, 10000.0, 5.0))) > 5


def test_oracle_realisation_injects_at_the_track():
    wl = synth.tiny()
    d = wl.dets[0]
    geo = dict(t_seg=d["t_seg"], v=d["v"], weights=np.linspace(0.5, 2.0, 1024).astype(np.float32),
               k_lo=d["k_lo"], t_sft=d["t_sft"], n_bins=800)
    sky = wl.grid["sky"][0]
    inj = (552.3, 9000.0, 5.0, 3.0)
    base = oc.realisation(geo, 9, 2, 4)
    sig = oc.realisation(geo, 9, 2, 4, inj, sky)
    b = oracle.track_bins(base, inj[0], inj[1], inj[2], sky, 0.0)
    diff = np.argwhere(sig.rho != base.rho)
    assert len(diff) == int(np.sum((b >= 0) & (b < 800)))
    for j, col in diff:
        assert col == b[j]
        assert sig.rho[j, col] == np.float32(base.rho[j, col] + np.float32(np.float32(3.0) * geo["weights"][j]))
