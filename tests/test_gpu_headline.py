"""GPU parity at the realistic single search (10800 segments x 8000 bins,
2,304,000 templates, U[0.5, 2] weights, 20 injections): every template
against the FP64 oracle, in the tile shape the autotuner picks for it (the
benchmark's launch configuration) and in every other tile shape, plus the
device's Eq. 1 and Eq. 2 tables bit for bit.

Bar: c and N bit-exact for all templates; s within 1e-5 relative; every
critical ratio (Eq. 4) within the tolerance the sum allows (count ratios to
rounding); the count top-10 identical to the oracle's, the power top-10
identical up to float near-ties; g = RN(u^e) (Eq. 1) identical to the
oracle's correctly rounded power for all 288 x 10800 entries, and the track
factor RN(RN(g D) T_sft) (Eq. 2) identical to the one formed from the
oracle's g and Doppler factors.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_sums_close, assert_topk_count, assert_topk_power, psi_tolerance

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def realistic():
    """The realistic workload with its injections added at the oracle's bins,
    and the oracle's statistic of every template."""
    wl = synth.realistic()
    d = wl.dets[0]
    g = wl.grid
    rho = d["rho"]
    det = oracle.Detector(rho, d["t_seg"], d["v"], d["k_lo"], d["t_sft"], weights=d["weights"])
    for inj in wl.injections:
        b = oracle.track_bins(det, inj["f0"], inj["tau"], inj["brake"], inj["sky"], g["t0"])
        ok = (b >= 0) & (b < det.n_bins)
        j = np.nonzero(ok)[0]
        rho[j, b[ok]] += np.float32(inj["amp"]) * d["weights"][j]
    det = oracle.Detector(rho, d["t_seg"], d["v"], d["k_lo"], d["t_sft"], weights=d["weights"])
    grid = oracle.Grid(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    print(f"oracle: all {grid.n_templates} templates on {oracle.threads()} threads", flush=True)
    ref = oracle.evaluate(det, grid)
    return det, grid, ref


def _load(ctx, det, store="f32"):
    import torch

    ctx.load_spectrogram(0, torch.from_numpy(det.rho).cuda(), det.k_lo, det.t_sft, det.t_seg, weights=det.w,
                         store=store)
    ctx.set_velocity_table(0, det.v)


def _eval(ctx, grid):
    s, c, N = ctx.eval_templates(grid.f0_min, grid.f0_step, grid.n_f0, grid.tau, grid.brake, grid.sky, grid.t0)
    return s.cpu().numpy().astype(np.float64), c.cpu().numpy(), N.cpu().numpy()


def _check_all(s, c, N, ref):
    assert np.array_equal(N, ref["N"])
    assert np.array_equal(c, ref["c"])
    return assert_sums_close(s, ref["s"])


def test_realistic_every_template_in_the_tuned_shape(realistic):
    """The benchmark's sequence: load, autotune, evaluate; the variant the
    diagnostics report is the tuned one, and every template matches the
    oracle; so do the ratios and both top-10 lists."""
    from paper_2507_07816_amd import ltgw

    det, grid, ref = realistic
    ctx = ltgw.Context(0)
    _load(ctx, det)
    tuned = ctx.autotune(grid.f0_min, grid.f0_step, grid.n_f0, grid.tau, grid.brake, grid.sky, grid.t0)
    print(f"case: realistic, every template, tuned variant {tuned}", flush=True)
    s, c, N = _eval(ctx, grid)
    dg = ctx.diagnostics()
    assert dg["tile_shape"] == tuned
    assert dg["pow_undecided"] == 0
    assert dg["in_band"] == int(ref["N"].astype(np.int64).sum())
    assert dg["evals"] == grid.n_templates * det.n_seg
    worst = _check_all(s, c, N, ref)
    print(f"worst relative s error {worst:.3g}", flush=True)
    n = grid.n_templates
    pp, pc = ctx.psi("power", n).cpu().numpy(), ctx.psi("count", n).cpu().numpy()
    po, co = oracle.psi_power(ref), oracle.psi_count(ref)
    assert np.array_equal(np.isnan(pp), np.isnan(po)) and np.array_equal(np.isnan(pc), np.isnan(co))
    ok = ~np.isnan(po)
    assert np.all(np.abs(pp[ok] - po[ok]) <= psi_tolerance(ref)[ok] + 1e-12)
    assert np.allclose(pc[ok], co[ok], rtol=1e-13, atol=1e-13)
    assert_topk_count(ctx.topk("count", 10), ref, 10)
    got, want = assert_topk_power(ctx.topk("power", 10), ref, 10)
    print(f"power top-10 {got} oracle {want}", flush=True)
    ctx.close()


def test_realistic_every_template_in_every_shape(realistic):
    """Whichever shape the autotuner picks on a given device, its results are
    the oracle's: all 16 tile shapes (templates per lane, gather batch,
    generations, segment slabs) over every template."""
    from paper_2507_07816_amd import ltgw

    det, grid, ref = realistic
    ctx = ltgw.Context(0)
    _load(ctx, det)
    first = None
    for v in range(16):
        print(f"case: realistic, every template, variant {v}", flush=True)
        ctx.set_tile_shape(v)
        s, c, N = _eval(ctx, grid)
        assert ctx.diagnostics()["tile_shape"] == v
        if first is None:
            _check_all(s, c, N, ref)
            first = (s, c, N)
        else:  # the same operations in the same order: identical to the checked shape
            assert np.array_equal(s, first[0]) and np.array_equal(c, first[1]) and np.array_equal(N, first[2])
    ctx.close()


def test_realistic_tables_bitwise(realistic):
    """T12: the device's Eq. 1 table g[(i_n, i_tau)][j] equals the oracle's
    correctly rounded power for all 288 x 10800 entries, and its Eq. 2 track
    factor RN(RN(g D) T_sft) equals the one formed from the oracle's g and
    Doppler factors D = 1 + v.n/c."""
    from paper_2507_07816_amd import ltgw

    det, grid, _ = realistic
    ctx = ltgw.Context(0)
    _load(ctx, det)
    print("case: realistic, Eq. 1 and Eq. 2 tables", flush=True)
    _eval(ctx, grid)
    g_dev, h_dev = ctx.read_tables(0)
    ctx.close()
    assert g_dev.shape == (len(grid.tau) * len(grid.brake), det.n_seg)
    g_ref = np.stack([oracle.spin_factor_array(det.t_seg, grid.t0, ta, b) for b in grid.brake for ta in grid.tau])
    bad = np.nonzero(g_dev.view(np.uint64) != g_ref.view(np.uint64))
    assert bad[0].size == 0, f"{bad[0].size} spin factors differ; first at {bad[0][:3]}, {bad[1][:3]}"
    D = np.array([oracle.doppler(det.v[j], grid.sky[0]) for j in range(det.n_seg)])
    h_ref = (g_ref * D[None, :]) * det.t_sft
    assert h_dev.shape == h_ref.shape
    assert np.array_equal(h_dev.view(np.uint64), h_ref.view(np.uint64))
