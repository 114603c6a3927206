"""End to end on the GPU: strain with a continuously phased msMagnetar chirp
(Eq. 1, Doppler-shifted by Eq. 2) -> the data preparation (Sec. 2) -> ingest
-> the lattice search -> top-k, against the FP64 oracle's data preparation and
statistic on the same strain.

Bar, stage by stage: rho within 2e-5 (1 + rho) of the oracle's data
preparation; the search on the GPU's rho against the oracle's statistic on the
same rho (the count list identical, the power list identical up to float
near-ties); the whole chain's loudest template equal to the oracle chain's
(the count compares each pixel with 1.6, so a pixel within the rho tolerance
of it may count differently between the chains) and next to the injected
parameters.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_topk_count, assert_topk_power, run_gpu
from oracle import sft

pytestmark = pytest.mark.gpu


def _chirp_strain(fs, n_seg, t_sft, f0, tau, brake, sky, amp, seed):
    """Gaussian noise plus amp cos(phase), the phase the integral of
    2 pi f0 u(t)^(1/(1-n)) (1 + v(t).n/c) sampled at fs (FP64)."""
    n = int(fs * t_sft) * n_seg
    t = np.arange(n, dtype=np.float64) / fs
    u = 1.0 + t / tau
    f = f0 * u ** (1.0 / (1.0 - brake))
    v = synth.velocity(t)
    f = f * (1.0 + (v @ np.asarray(sky)) / synth.C_LIGHT)
    phase = 2.0 * np.pi * np.cumsum(f) / fs
    r = np.random.default_rng(seed)
    return (r.normal(size=n) + amp * np.cos(phase)).astype(np.float32)


def test_strain_to_candidates():
    import torch
    from paper_2507_07816_amd import ltgw

    fs, t_sft, n_seg = 1024, 8.0, 96
    f0, tau, brake = 301.0, 2000.0, 5.0
    sky = synth.sky_vector(1.0, 0.3)
    x = _chirp_strain(fs, n_seg, t_sft, f0, tau, brake, sky, amp=0.08, seed=66)
    n_fft, k_lo, n_bins, window = int(fs * t_sft), 2000, 480, 101       # 250 .. 309.875 Hz
    print("case: end to end, 96 segments of 8 s at 1024 Hz", flush=True)
    t_seg = np.arange(n_seg, dtype=np.float64) * t_sft       # segment start times (T0 = 0)
    v = synth.velocity(t_seg)
    rho_ref = sft.normalised_power(x, n_fft, k_lo, n_bins, window).astype(np.float32)
    ctx = ltgw.Context(0)
    try:
        rho_gpu = ctx.sft_normalise(torch.from_numpy(x).cuda(), n_fft, k_lo, n_bins, window)
        det_gpu = oracle.Detector(rho_gpu.cpu().numpy(), t_seg, v, k_lo, t_sft)
        grid = oracle.Grid(296.0, 0.125, 64, [1000.0, 2000.0, 4000.0], [3.0, 5.0, 7.0], [sky])
        gpu = run_gpu([det_gpu], grid, k=5, ctx=ctx)
    finally:
        ctx.close()
    rho_g = det_gpu.rho.astype(np.float64)
    assert np.all(np.abs(rho_g - rho_ref) <= 2e-5 * (1.0 + rho_ref))
    ref = oracle.evaluate(det_gpu, grid)                      # the search stage on the GPU's rho
    assert_topk_count(gpu["top_count"], ref, 5)
    assert_topk_power(gpu["top_power"], ref, 5)
    chain = oracle.evaluate(oracle.Detector(rho_ref, t_seg, v, k_lo, t_sft), grid)
    assert gpu["top_power"][0]["index"] == int(oracle.topk(oracle.psi_power(chain), 1)[0])
    best = gpu["top_power"][0]
    assert abs(best["f0"] - f0) <= 0.25 and best["tau"] == tau and best["brake"] == brake
    assert best["psi"] > 10.0
