"""Pins of the data-preparation reference (oracle/sft.py, Sec. 2).

- A cosine at the centre of bin k0 has the Hann spectrum X_k0 = A N/4,
  X_{k0 +- 1} = -A N/8 and zero elsewhere (the window's three Fourier terms).
- Gaussian white noise normalised by the running median is Exp(1)-like: mean
  near 1 (the median estimate carries a small bias), P(rho > 1.6) near e^-1.6.
- rho does not change when the strain is scaled.
- A linear ramp P_k = k has the centre value as its running median, so
  rho = ln 2 in every bin (to the two roundings of P ln2 / P).
"""
import math

import numpy as np
import pytest

from oracle import sft


@pytest.mark.parametrize("N,k0,A", [(1024, 100, 1.0), (4096, 1000, 3.5), (32768, 4321, 0.25)])
def test_hann_spectrum_of_a_bin_centred_cosine(N, k0, A):
    n = np.arange(N)
    x = A * np.cos(2.0 * np.pi * k0 * n / N)
    P = sft.power(x, N)[0]
    assert P[k0] == pytest.approx((A * N / 4) ** 2, rel=1e-10)
    assert P[k0 - 1] == pytest.approx((A * N / 8) ** 2, rel=1e-10)
    assert P[k0 + 1] == pytest.approx((A * N / 8) ** 2, rel=1e-10)
    rest = np.delete(P, [k0 - 1, k0, k0 + 1])
    assert rest.max() < 1e-18 * P[k0]


def test_white_noise_normalises_to_exp1():
    r = np.random.default_rng(61)
    N, n_seg = 4096, 64
    x = r.normal(0.0, 2.5, N * n_seg)
    rho = sft.normalised_power(x, N, 300, 1200, 101)
    assert rho.shape == (n_seg, 1200)
    assert rho.mean() == pytest.approx(1.0, abs=0.03)
    assert np.mean(rho > 1.6) == pytest.approx(math.exp(-1.6), abs=0.01)
    # the Hann window's noise gain: E[P] = sigma^2 sum w^2 = sigma^2 3N/8
    P = sft.power(x, N)
    assert P[:, 300:1500].mean() == pytest.approx(2.5 ** 2 * 3 * N / 8, rel=0.03)


def test_scale_invariance():
    r = np.random.default_rng(62)
    x = r.normal(size=2048 * 8)
    a = sft.normalised_power(x, 2048, 100, 500, 51)
    b = sft.normalised_power(7.0 * x, 2048, 100, 500, 51)
    assert np.allclose(a, b, rtol=1e-12, atol=0)


def test_running_median_of_a_ramp():
    P = np.tile(np.arange(1.0, 3001.0), (3, 1))
    rho = sft.normalise(P, 200, 2000, 101)
    assert np.allclose(rho, math.log(2.0), rtol=5e-16, atol=0.0)
    # a step in the floor is normalised away bin for bin: each window's median
    # is the level of the majority of its bins, which is the centre bin's level
    P = np.ones((2, 3000))
    P[:, 1000:] = 10.0
    rho = sft.normalise(P, 200, 2000, 101)
    assert np.allclose(rho, math.log(2.0), rtol=5e-16, atol=0.0)
