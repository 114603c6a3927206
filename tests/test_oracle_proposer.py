"""Pins of the proposer's reference definitions (oracle/proposer.py, oracle/cnn.py
operand rounding and Adam).

- the coarse map is the S x 2 block sum, rounded to bfloat16 (hand values, a
  tie, groups of 2 and of 4 segments);
- the coarse critical ratio against the fine oracle: with each group of S
  segments sharing one time and velocity and power constant on S x 2 blocks,
  the coarse ratio is sqrt(2) times the fine one, for S = 2, 4 and 8;
- only the first segment of a pair places the coarse column;
- noise-free constant power gives Psi = 0 on every in-band template;
- the coarse count: hand values at the strict FP32 threshold; with count
  bits constant on S x 2 blocks of duplicated groups the coarse count ratio is
  sqrt(2) times the fine one (Eq. 4 for the count); every pixel above the
  threshold gives the closed form sqrt(N 2 S (1 - q) / q);
- cells <-> templates is a bijection; best_template's tie rule;
- BF16 operand rounding; Adam's first step on a constant gradient moves every
  parameter by lr against the gradient's sign.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import cnn
from oracle import proposer as op


def _geometry(n_seg, seed=0, spacing=40.0, dup=False):
    r = np.random.default_rng(seed)
    t = np.arange(n_seg) * spacing + 2.0
    v = r.normal(size=(n_seg, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * 3.0e4
    if dup:
        t[1::2] = t[0::2]
        v[1::2] = v[0::2]
    return t, v


GRID = dict(f0_min=480.0, f0_step=0.25, n_f0=24, tau=[4000.0, 15000.0], brake=[3.0, 5.0],
            sky=[[0.6, 0.0, 0.8]], t0=0.0)


def _grid():
    return oracle.Grid(GRID["f0_min"], GRID["f0_step"], GRID["n_f0"], GRID["tau"], GRID["brake"],
                       GRID["sky"], GRID["t0"])


def test_coarse_power_groups_of_four_segments():
    P = np.zeros((8, 4), np.float32)
    P[0:4, 0:2] = 1.0          # 8 ones in the first coarse pixel
    P[4, 2], P[7, 3] = 127.5, 1.5
    C = op.coarse_power(P, S=4)
    assert C.shape == (2, 2) and C[0, 0] == 8.0 and C[1, 1] == 129.0 and C[0, 1] == 0.0
    assert np.allclose(op.coarse_weights(np.array([1, 2, 3, 4, 1, 1, 1, 1], np.float32), 8, 4), [2.5, 1.0])


def test_coarse_power_block_sums_and_bf16_tie():
    P = np.zeros((4, 6), np.float32)
    P[0, 0], P[0, 1], P[1, 0], P[1, 1] = 1.0, 2.0, 3.0, 4.0
    P[2, 4], P[3, 5] = 128.5, 128.5          # 257 ties between 256 and 258 -> 256
    P[2, 2] = 3.0                             # 3 exact
    C = op.coarse_power(P)
    assert C.shape == (2, 3)
    assert C[0, 0] == 10.0 and C[1, 2] == 256.0 and C[1, 1] == 3.0
    assert C[0, 1] == 0.0 and C[0, 2] == 0.0 and C[1, 0] == 0.0


@pytest.mark.parametrize("S", [2, 4, 8])
def test_coarse_psi_is_sqrt2_times_fine_on_duplicated_groups(S):
    """Each group of S segments shares one time and velocity, the weights are
    equal within a group and the power is constant on S x 2 blocks: the fine
    sum is S w q per group, the coarse one 2 S w q, so the coarse ratio is
    sqrt(2) times the fine one for every S (with weights whose group sums are
    exact in FP32)."""
    n_seg, n_bins, k_lo, t_sft = 64, 96, 1900, 4.0
    t, v = _geometry(n_seg)
    for k in range(1, S):
        t[k::S] = t[0::S]
        v[k::S] = v[0::S]
    r = np.random.default_rng(3)
    q = r.integers(0, 6, size=(n_seg // S, n_bins // 2)).astype(np.float32)
    P = np.repeat(np.repeat(q, S, axis=0), 2, axis=1)        # constant on S x 2 blocks
    # equal within a group, and dyadic (k / 8) so that the FP32 sums of a group's
    # weights are exact and the coarse weight is the fine one
    w = np.repeat((r.integers(4, 17, n_seg // S) / 8.0).astype(np.float32), S)
    det = oracle.Detector(P, t, v, k_lo, t_sft, weights=w)
    g = _grid()
    fine = oracle.psi_power(oracle.evaluate(det, g))
    coarse = op.coarse_psi(det, g, P, S=S)
    ok = np.isfinite(fine)
    assert ok.sum() > 50
    assert np.array_equal(ok, np.isfinite(coarse))
    assert np.allclose(coarse[ok], math.sqrt(2.0) * fine[ok], rtol=1e-12, atol=1e-12)


def test_coarse_psi_uses_the_first_segment_of_each_pair():
    n_seg, n_bins, k_lo, t_sft = 48, 128, 1890, 4.0
    t, v = _geometry(n_seg, seed=5)
    P = np.random.default_rng(6).exponential(size=(n_seg, n_bins)).astype(np.float32)
    g = _grid()
    a = op.coarse_psi(oracle.Detector(P, t, v, k_lo, t_sft), g, P)
    t2, v2 = t.copy(), v.copy()
    t2[1::2] += 17.0
    v2[1::2] *= -1.0
    b = op.coarse_psi(oracle.Detector(P, t2, v2, k_lo, t_sft), g, P)
    assert np.array_equal(a, b, equal_nan=True)
    t3 = t.copy()
    t3[0::2] += 17.0                           # moving the first segments does matter
    c = op.coarse_psi(oracle.Detector(P, t3, v, k_lo, t_sft), g, P)
    assert not np.array_equal(a, c, equal_nan=True)


def test_coarse_psi_constant_power_is_zero():
    n_seg, n_bins = 32, 64
    t, v = _geometry(n_seg)
    P = np.ones((n_seg, n_bins), np.float32)
    det = oracle.Detector(P, t, v, 1900, 4.0)
    psi = op.coarse_psi(det, _grid(), P, nan_to_zero=True)
    assert np.all(psi == 0.0)


def test_coarse_count_hand_values_and_strict_threshold():
    P = np.zeros((4, 4), np.float32)
    P[0, 0], P[1, 1], P[0, 1] = 1.7, 2.0, np.float32(1.6)   # 1.6f itself is not above 1.6f
    P[2, 2], P[3, 3], P[3, 2] = 5.0, 1.6000001, 0.5
    C = op.coarse_count(P, S=2)
    assert C.tolist() == [[2, 0], [0, 2]]
    assert op.coarse_count(P, S=4).tolist() == [[2, 2]]


@pytest.mark.parametrize("S", [2, 4])
def test_coarse_count_psi_is_sqrt2_times_fine_on_duplicated_groups(S):
    """Duplicated groups of S segments and count bits constant on S x 2
    blocks: a template collects S bits per group on the fine map and 2 S on
    the coarse one, over S times fewer segments, so the coarse count ratio is
    sqrt(2) times the fine one."""
    n_seg, n_bins, k_lo, t_sft = 64, 96, 1900, 4.0
    t, v = _geometry(n_seg, seed=11)
    for k in range(1, S):
        t[k::S] = t[0::S]
        v[k::S] = v[0::S]
    r = np.random.default_rng(12)
    bits = r.integers(0, 2, size=(n_seg // S, n_bins // 2))
    P = np.repeat(np.repeat(np.where(bits == 1, 2.5, 0.5).astype(np.float32), S, axis=0), 2, axis=1)
    det = oracle.Detector(P, t, v, k_lo, t_sft)
    g = _grid()
    fine = oracle.psi_count(oracle.evaluate(det, g))
    coarse = op.coarse_psi_count(det, g, P, S=S)
    ok = np.isfinite(fine)
    assert ok.sum() > 50
    assert np.array_equal(ok, np.isfinite(coarse))
    assert np.allclose(coarse[ok], math.sqrt(2.0) * fine[ok], rtol=1e-12, atol=1e-12)


def test_coarse_count_psi_all_above_threshold():
    """Every pixel above the threshold: each in-band coarse segment adds 2 S
    counts, so Psi = (2 S N - 2 S N q) / sqrt(2 S N q (1 - q))."""
    n_seg, n_bins, S = 32, 64, 4
    t, v = _geometry(n_seg)
    P = np.full((n_seg, n_bins), 3.0, np.float32)
    det = oracle.Detector(P, t, v, 1900, 4.0)
    g = _grid()
    psi = op.coarse_psi_count(det, g, P, S=S)
    q = oracle.count_q(1.6)
    n = np.zeros(g.n_templates)
    for k in range(g.n_templates):
        f0, tau, brake, _ = g.params(k)
        b = oracle.track_bins(det, float(f0), float(tau), float(brake), g.sky[0], g.t0)[0::S]
        n[k] = np.count_nonzero((b >= 0) & (b // 2 < n_bins // 2))
    ok = n > 0
    assert ok.sum() > 10 and np.all(np.isnan(psi[~ok]))
    assert np.allclose(psi[ok], np.sqrt(n[ok] * 2 * S * (1 - q) / q), rtol=1e-12)


def test_cells_templates_bijection_and_best():
    L, c_out = 7, 6
    cells = np.arange(c_out * L)
    tpl = op.cell_to_template(cells, L)
    assert sorted(tpl.tolist()) == list(range(c_out * L))
    assert np.array_equal(op.template_to_cell(tpl, L), cells)
    assert op.cell_to_template([1 * L + 3], L)[0] == 0 * 2 * L + 2 * 3 + 1
    assert op.best_template([1.0, np.nan, 3.0, 3.0], [9, 1, 7, 4]) == (4, 3.0)
    assert op.best_template([np.nan], [0]) == (-1, -np.inf)


def test_bf16_operands_and_adam_first_step():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -9, -2.0 ** -130, 3.4e38])
    assert np.array_equal(cnn.bf16_operands(x)[:3], [1.0, 1.0, 1.0078125])
    assert cnn.bf16_operands(x)[3] == -2.0 ** -130 and np.isinf(cnn.bf16_operands(x)[4])
    g = np.array([0.3, -2.0, 1e-3, -5e2])
    p0 = np.zeros(4)
    p, m, v = cnn.adam(p0, g, np.zeros(4), np.zeros(4), 1e-2, 0.9, 0.999, 1e-12, 1)
    assert np.allclose(p, -1e-2 * np.sign(g), rtol=1e-9)
    p, m, v = cnn.adam(p, g, m, v, 1e-2, 0.9, 0.999, 1e-12, 2)
    assert np.allclose(p, -2e-2 * np.sign(g), rtol=1e-9)
