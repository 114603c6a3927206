"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Bar: number count c and in-band count N bit-exact; the power sum s within
1e-5 relative of the FP64 oracle (the FP32 accumulation is well inside it);
bin indices exact (checksum spectrogram rho[j, b] = b makes s an exact
integer that encodes every selected bin); top-k identical for the count and
identical up to float near-ties for the power.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_util import (assert_sums_close, assert_topk_count, assert_topk_power, psi_tolerance,
                      run_gpu)

pytestmark = pytest.mark.gpu


def tiny_oracle(with_injection=True, rho=None, store=None):
    wl = synth.tiny()
    d = wl.dets[0]
    r = d["rho"].copy() if rho is None else rho
    det = oracle.Detector(r, d["t_seg"], d["v"], d["k_lo"], d["t_sft"])
    g = wl.grid
    grid = oracle.Grid(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    if with_injection:
        for inj in wl.injections:
            b = oracle.track_bins(det, inj["f0"], inj["tau"], inj["brake"], inj["sky"], g["t0"])
            for j, bj in enumerate(b):
                if 0 <= bj < det.n_bins:
                    r[j, bj] += np.float32(inj["amp"])
        det = oracle.Detector(r, d["t_seg"], d["v"], d["k_lo"], d["t_sft"])
    return det, grid, wl


def test_tiny_workload_parity():
    det, grid, wl = tiny_oracle()
    print("case: tiny workload FP32, 4800 templates x 1024 segments", flush=True)
    ref = oracle.evaluate(det, grid)
    gpu = run_gpu([det], grid)
    assert np.array_equal(gpu["N"], ref["N"])
    assert np.array_equal(gpu["c"], ref["c"])
    worst = assert_sums_close(gpu["s"], ref["s"])
    assert worst < 1e-6
    assert_topk_count(gpu["top_count"], ref, 10)
    assert_topk_power(gpu["top_power"], ref, 10)
    # the injected template (f0 = 550, tau = 7000, n = 5) is the loudest by power
    inj = wl.injections[0]
    want = (1 * 4 + 1) * 400 + 200  # i_n = 1 (n = 5), i_tau = 1 (7000), i_f0 = 200
    assert gpu["top_power"][0]["index"] == want
    assert gpu["top_power"][0]["f0"] == inj["f0"] and gpu["top_power"][0]["tau"] == inj["tau"]
    assert gpu["diag"]["pow_undecided"] == 0
    assert gpu["diag"]["in_band"] == int(ref["N"].sum())
    assert gpu["diag"]["evals"] == grid.n_templates * det.n_seg


def test_tiny_psi_all_templates():
    det, grid, _ = tiny_oracle()
    ref = oracle.evaluate(det, grid)
    gpu = run_gpu([det], grid)
    pc = oracle.psi_count(ref)
    assert np.array_equal(np.isnan(gpu["psi_count"]), np.isnan(pc))
    ok = ~np.isnan(pc)
    assert np.allclose(gpu["psi_count"][ok], pc[ok], rtol=1e-14, atol=1e-14)
    pp = oracle.psi_power(ref)
    tol = psi_tolerance(ref)
    ok = ~np.isnan(pp)
    assert np.all(np.abs(gpu["psi_power"][ok] - pp[ok]) <= tol[ok] + 1e-12)


def test_tiny_bin_checksum_exact():
    """rho[j, b] = b: every template's s is an exact integer sum of its bins,
    so equality pins every bin of every template and segment (0 mismatches)."""
    rho = np.tile(np.arange(800, dtype=np.float32), (1024, 1))
    det, grid, _ = tiny_oracle(with_injection=False, rho=rho)
    ref = oracle.evaluate(det, grid)
    gpu = run_gpu([det], grid)
    assert np.array_equal(gpu["s"], ref["s"])
    assert np.array_equal(gpu["N"], ref["N"])
    assert np.array_equal(gpu["c"], ref["c"])


def _small(seed, n_seg, n_bins, k_lo=1900, t_sft=4.0, vmag=3.0e5, spacing=300.0, weights=True):
    """weights: True = U[0.5, 2]; 'wide' = 2^U[-6, 6] (beyond the fixed-point
    moment range, so the statistic kernel accumulates W1, W2 itself)."""
    rng = np.random.default_rng(seed)
    t_seg = np.arange(n_seg) * spacing + 2.0
    v = rng.normal(size=(n_seg, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * vmag
    rho = rng.exponential(size=(n_seg, n_bins)).astype(np.float32)
    if weights == "wide":
        w = np.exp2(rng.uniform(-6.0, 6.0, n_seg)).astype(np.float32)
    else:
        w = rng.uniform(0.5, 2.0, n_seg).astype(np.float32) if weights else None
    return oracle.Detector(rho, t_seg, v, k_lo, t_sft, weights=w)


@pytest.mark.parametrize("n_seg,n_bins,n_f0,t0,weights", [
    (1, 1, 1, 0.0, True),           # degenerate: one segment, one bin, one template
    (77, 33, 300, 0.0, True),       # ragged everywhere (segments not a multiple of 8/32, f0 not of 256)
    (5, 800, 257, 0.0, True),
    (40, 256, 513, 700.0, True),    # T0 inside the data: the first 19 segments are masked
    (129, 97, 64, 0.0, True),
    (129, 97, 300, 0.0, "wide"),    # weights over 12 binades: moments accumulated in the kernel
    (77, 120, 257, 0.0, False),     # unit weights
])
def test_ragged_shapes_weighted(n_seg, n_bins, n_f0, t0, weights):
    print(f"case: ragged n_seg={n_seg} n_bins={n_bins} n_f0={n_f0} t0={t0} w={weights}", flush=True)
    det = _small(n_seg + n_bins, n_seg, n_bins, k_lo=1990 - n_bins // 4, spacing=37.0,
                 weights=weights)
    grid = oracle.Grid(490.0 + 0.03 * n_bins, 0.25, n_f0, [512.0, 5000.0, 35000.0], [2.5, 5.0],
                       [[0.6, 0.0, 0.8], [0.0, -1.0, 0.0]], t0)
    ref = oracle.evaluate(det, grid)
    gpu = run_gpu([det], grid, k=7)
    assert np.array_equal(gpu["N"], ref["N"])
    assert np.array_equal(gpu["c"], ref["c"])
    assert_sums_close(gpu["s"], ref["s"])
    pp = oracle.psi_power(ref)
    ok = ~np.isnan(pp)
    assert np.array_equal(np.isnan(gpu["psi_power"]), ~ok)
    assert np.all(np.abs(gpu["psi_power"][ok] - pp[ok]) <= psi_tolerance(ref)[ok] + 1e-9)
    if (ref["N"] > 0).sum() >= 7:
        assert_topk_count(gpu["top_count"], ref, 7)
        assert_topk_power(gpu["top_power"], ref, 7)


def test_two_detectors_sum():
    d1 = _small(1, 60, 256, k_lo=1900)
    d2 = _small(2, 45, 200, k_lo=1930, t_sft=4.0)
    grid = oracle.Grid(478.0, 0.5, 200, [5000.0, 20000.0], [3.0, 5.0, 7.0], [[0.6, 0.0, 0.8]])
    ref = oracle.evaluate([d1, d2], grid)
    gpu = run_gpu([d1, d2], grid)
    assert np.array_equal(gpu["N"], ref["N"])
    assert np.array_equal(gpu["c"], ref["c"])
    assert_sums_close(gpu["s"], ref["s"])
    assert_topk_count(gpu["top_count"], ref, 10)
    # a detector mask selects one of them
    ref1 = oracle.evaluate([d2], grid)
    gpu1 = run_gpu([d1, d2], grid, det_mask=2)
    assert np.array_equal(gpu1["N"], ref1["N"])
    assert_sums_close(gpu1["s"], ref1["s"])


def test_all_out_of_band():
    det = _small(3, 16, 64, k_lo=1900)
    grid = oracle.Grid(900.0, 1.0, 40, [5000.0], [5.0], [[0.6, 0.0, 0.8]])  # far above the band
    gpu = run_gpu([det], grid)
    assert np.all(gpu["N"] == 0) and np.all(gpu["c"] == 0) and np.all(gpu["s"] == 0)
    assert np.all(np.isnan(gpu["psi_power"]))
    assert gpu["top_power"] == [] and gpu["top_count"] == []


def test_closed_forms_on_gpu():
    """Hot pixel, constant spectrogram and noiseless injection, as in the oracle pins."""
    det0 = _small(4, 8, 256, spacing=300.0)
    grid = oracle.Grid(478.0, 2.625, 24, [5000.0, 20000.0], [3.0, 5.0],
                       [[0.6, 0.0, 0.8], [0.0, -1.0, 0.0]])
    rho = np.zeros((8, 256), np.float32)
    rho[3, 100] = 1.0
    rho[5, 37] = 2.0
    rho[0, 0] = 1.75
    cases = [rho, np.ones((8, 256), np.float32)]
    tb = oracle.track_bins(det0, 499.0, 20000.0, 5.0, grid.sky[0], 0.0)
    inj = np.zeros((8, 256), np.float32)
    for j, b in enumerate(tb):
        if 0 <= b < 256:
            inj[j, b] = 3.0
    cases.append(inj)
    for r in cases:
        det = oracle.Detector(r, det0.t_seg, det0.v, det0.k_lo, det0.t_sft, weights=det0.w)
        ref = oracle.evaluate(det, grid)
        gpu = run_gpu([det], grid, k=5)
        assert np.array_equal(gpu["N"], ref["N"])
        assert np.array_equal(gpu["c"], ref["c"])
        assert_sums_close(gpu["s"], ref["s"])


def test_repeat_is_bitwise_deterministic():
    det, grid, _ = tiny_oracle()
    a = run_gpu([det], grid)
    b = run_gpu([det], grid)
    for k in ("s", "c", "N", "psi_power", "psi_count"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("store", ["bf16", "fp8"])
def test_quantised_stores(store):
    """Codes bit-exact against the oracle's format definitions; sums within
    1e-5 of the FP64 oracle over the same dequantised values; count exact
    (decided on the FP32 input)."""
    torch = pytest.importorskip("torch")
    from paper_2507_07816_amd import ltgw

    det, grid, _ = tiny_oracle()
    rho = det.rho.copy()
    rho[7, :] = 0.0                       # an all-zero row: FP8 scale 1
    rho[9, 3] = np.float32(1.6)           # exactly at the threshold: not counted
    rho[9, 4] = np.nextafter(np.float32(1.6), np.float32(2))
    rho[11, 5] = 5000.0                   # a loud pixel that sets the FP8 row scale
    vals, sc = oracle.dequantised(rho, store)
    qdet = oracle.Detector(rho, det.t_seg, det.v, det.k_lo, det.t_sft, values=vals)
    ctx = ltgw.Context(0)
    gpu = run_gpu([qdet], grid, store=store, ctx=ctx)
    codes, gsc = ctx.read_store(0)
    ctx.close()
    bit = (rho > np.float32(1.6))
    if store == "bf16":
        want = oracle.bf16_rne(rho) | (bit.astype(np.uint16) << 15)
    else:
        want = oracle.e4m3_rne_sat(rho / sc[:, None]) | (bit.astype(np.uint8) << 7)
        assert np.array_equal(gsc, sc)
    assert np.array_equal(codes, want)
    ref = oracle.evaluate(qdet, grid)
    assert np.array_equal(gpu["c"], ref["c"])
    assert np.array_equal(gpu["N"], ref["N"])
    assert_sums_close(gpu["s"], ref["s"])
    assert_topk_count(gpu["top_count"], ref, 10)


def test_fp8_decode_all_codes():
    """Every E4M3 code decodes to the format's value (via a one-row store whose
    codes are all 128 non-negative patterns and a checksum-style evaluation)."""
    pytest.importorskip("torch")
    vals = np.array([oracle.e4m3_decode(c) for c in range(0x7f)], np.float32)  # 0x7f is NaN
    assert np.array_equal(oracle.e4m3_rne_sat(vals), np.arange(0x7f, dtype=np.uint8))
    rho = (vals * np.float32(0.5))[None, :]  # row max 224 -> scale 0.5, codes reproduce vals
    vals_q, sc = oracle.dequantised(rho, "fp8")
    assert sc[0] == np.float32(0.5) and np.array_equal(vals_q[0], rho[0].astype(np.float64))
    # one template per column: f0 = (k_lo + b)/T_sft with v = 0, t = T0 selects column b
    det = oracle.Detector(rho, [0.0], np.zeros((1, 3)), 2000, 4.0, values=vals_q)
    grid = oracle.Grid(500.0, 0.25, 0x7f, [5000.0], [5.0], [[1.0, 0.0, 0.0]], 0.0)
    ref = oracle.evaluate(det, grid)
    assert np.array_equal(ref["s"], rho[0].astype(np.float64))
    gpu = run_gpu([det], grid, store="fp8")
    assert np.array_equal(gpu["s"], ref["s"])


def test_inject_matches_oracle_bins():
    torch = pytest.importorskip("torch")
    from paper_2507_07816_amd import ltgw

    wl = synth.realistic(n_seg=600, n_bins=1000, n_f0=64)
    d = wl.dets[0]
    ctx = ltgw.Context(0)
    z = torch.zeros(d["rho"].shape, dtype=torch.float32, device="cuda")
    ctx.load_spectrogram(0, z, d["k_lo"], d["t_sft"], d["t_seg"], weights=d["weights"])
    ctx.set_velocity_table(0, d["v"])
    det = oracle.Detector(np.zeros_like(d["rho"]), d["t_seg"], d["v"], d["k_lo"], d["t_sft"],
                          weights=d["weights"])
    for inj in wl.injections[:5]:
        z.zero_()
        ctx.inject_track(0, z, inj["f0"], inj["tau"], inj["brake"], inj["sky"], 0.0, inj["amp"])
        got = z.cpu().numpy()
        tb = oracle.track_bins(det, inj["f0"], inj["tau"], inj["brake"], inj["sky"], 0.0)
        want = np.zeros_like(got)
        for j, b in enumerate(tb):
            if 0 <= b < det.n_bins:
                want[j, b] = np.float32(inj["amp"]) * d["weights"][j]
        assert np.array_equal(got, want)
    ctx.close()


def test_error_paths_leave_context_usable():
    torch = pytest.importorskip("torch")
    from paper_2507_07816_amd import ltgw

    det, grid, _ = tiny_oracle(with_injection=False)
    ctx = ltgw.Context(0)
    E = ltgw.LtgwError
    p = torch.from_numpy(det.rho).cuda()
    # eval and top-k before anything is loaded
    with pytest.raises(E) as ei:
        ctx.eval_templates(500.0, 0.25, 10, [3500.0], [5.0], [[1.0, 0, 0]])
    assert ei.value.code == ltgw.LTGW_E_STATE
    with pytest.raises(E) as ei:
        ctx.topk("power", 5)
    assert ei.value.code == ltgw.LTGW_E_STATE
    with pytest.raises(E) as ei:
        ctx.set_velocity_table(0, det.v)
    assert ei.value.code == ltgw.LTGW_E_STATE
    bad = p.clone()
    bad[3, 4] = -1.0
    for args, code in [((0, bad, det.k_lo, 4.0, det.t_seg), ltgw.LTGW_E_INVALID_ARG),
                       ((0, p, 1, 4.0, det.t_seg), ltgw.LTGW_E_INVALID_ARG),
                       ((0, p, det.k_lo, 0.0, det.t_seg), ltgw.LTGW_E_INVALID_ARG),
                       ((ltgw.LTGW_MAX_DET, p, det.k_lo, 4.0, det.t_seg), ltgw.LTGW_E_INVALID_ARG)]:
        with pytest.raises(E) as ei:
            ctx.load_spectrogram(*args)
        assert ei.value.code == code, args
    nanp = p.clone()
    nanp[0, 0] = float("nan")
    with pytest.raises(E):
        ctx.load_spectrogram(0, nanp, det.k_lo, 4.0, det.t_seg)
    ctx.load_spectrogram(0, p, det.k_lo, 4.0, det.t_seg)
    with pytest.raises(E) as ei:  # velocity missing
        ctx.eval_templates(500.0, 0.25, 10, [3500.0], [5.0], [[1.0, 0, 0]])
    assert ei.value.code == ltgw.LTGW_E_STATE
    fast = det.v.copy()
    fast[5] = [3.1e8, 0, 0]
    with pytest.raises(E) as ei:
        ctx.set_velocity_table(0, fast)
    assert ei.value.code == ltgw.LTGW_E_INVALID_ARG
    with pytest.raises(E) as ei:
        ctx.set_velocity_table(0, det.v[:-1])
    assert ei.value.code == ltgw.LTGW_E_INVALID_ARG
    ctx.set_velocity_table(0, det.v)
    for kw, code in [(dict(brake=[1.0]), ltgw.LTGW_E_INVALID_ARG),
                     (dict(tau=[-5.0]), ltgw.LTGW_E_INVALID_ARG),
                     (dict(f0_min=float("nan")), ltgw.LTGW_E_INVALID_ARG),
                     (dict(sky=[[1.0, 1.0, 0.0]]), ltgw.LTGW_E_INVALID_ARG),
                     (dict(det_mask=2), ltgw.LTGW_E_STATE),
                     (dict(f0_min=3.0e8), ltgw.LTGW_E_INVALID_ARG)]:
        args = dict(f0_min=500.0, f0_step=0.25, n_f0=10, tau=[3500.0], brake=[5.0],
                    sky=[[1.0, 0, 0]], t0=0.0, det_mask=0)
        args.update(kw)
        with pytest.raises(E) as ei:
            ctx.eval_templates(**args)
        assert ei.value.code == code, kw
        assert ltgw.ltgw_last_error(ctx.h)
    with pytest.raises(E):
        ctx.topk("power", 5)  # the failed eval left no results
    # the context still works
    s, c, N = ctx.eval_templates(500.0, 0.25, 10, [3500.0], [5.0], [[1.0, 0.0, 0.0]])
    assert int(N.sum()) > 0
    with pytest.raises(E) as ei:
        ctx.topk("power", 0)
    assert ei.value.code == ltgw.LTGW_E_INVALID_ARG
    with pytest.raises(E):
        ctx.topk("power", ltgw.LTGW_MAX_TOPK + 1)
    assert len(ctx.topk("power", 5)) == 5
    ctx.close()


def test_topk_large_k_and_ties():
    """k = 256 over a constant spectrogram: all power ratios tie at 0, so the
    order is the index order of templates with N > 0."""
    rho = np.ones((1024, 800), np.float32)
    det, grid, _ = tiny_oracle(with_injection=False, rho=rho)
    ref = oracle.evaluate(det, grid)
    gpu = run_gpu([det], grid, k=256)
    want = list(oracle.topk(oracle.psi_power(ref), 256))
    assert [t["index"] for t in gpu["top_power"]] == want
    assert_topk_count(gpu["top_count"], ref, 256)


def _realistic_det(checksum=False):
    wl = synth.realistic()
    d = wl.dets[0]
    g = wl.grid
    grid = oracle.Grid(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    if checksum:
        rho = np.tile(np.arange(d["rho"].shape[1], dtype=np.float32), (d["rho"].shape[0], 1))
        return oracle.Detector(rho, d["t_seg"], d["v"], d["k_lo"], d["t_sft"]), grid, wl
    rho = d["rho"]
    det = oracle.Detector(rho, d["t_seg"], d["v"], d["k_lo"], d["t_sft"], weights=d["weights"])
    for inj in wl.injections:
        b = oracle.track_bins(det, inj["f0"], inj["tau"], inj["brake"], inj["sky"], g["t0"])
        ok = (b >= 0) & (b < det.n_bins)
        j = np.nonzero(ok)[0]
        rho[j, b[ok]] += np.float32(inj["amp"]) * d["weights"][j]
    det = oracle.Detector(rho, d["t_seg"], d["v"], d["k_lo"], d["t_sft"], weights=d["weights"])
    return det, grid, wl


def _sample_indices(n, seed=0):
    """Contiguous runs (block edges, ragged tail) plus random templates."""
    r = np.random.default_rng(seed)
    runs = [np.arange(a, min(a + 300, n)) for a in (0, 7000, 8000 * 37 + 100, n // 2, n - 300)]
    return np.unique(np.concatenate(runs + [r.integers(0, n, 1500)]))


@pytest.mark.slow
def test_realistic_full_size_sampled():
    """The realistic search at full size (10800 segments x 8000 bins, 2,304,000
    templates, per-segment weights, 20 injections) in the untuned default tile
    shape; sampled templates against the oracle one by one.  (Every template
    in the tuned shape and in all others: test_gpu_headline.)"""
    print("case: realistic full size, weighted FP32", flush=True)
    det, grid, wl = _realistic_det()
    gpu = run_gpu([det], grid)
    idx = _sample_indices(grid.n_templates)
    top_p = [t["index"] for t in gpu["top_power"]]
    top_c = [t["index"] for t in gpu["top_count"]]
    idx = np.unique(np.concatenate([idx, top_p, top_c]))
    ref = oracle.evaluate_list(det, grid, idx)
    assert np.array_equal(gpu["N"][idx], ref["N"])
    assert np.array_equal(gpu["c"][idx], ref["c"])
    assert_sums_close(gpu["s"][idx], ref["s"])
    pp = oracle.psi_power(ref)
    pc = oracle.psi_count(ref)
    tol = psi_tolerance(ref)
    pos = {t: i for i, t in enumerate(idx)}
    # candidate records agree with the oracle, in non-increasing order
    for lst, psi, key in ((gpu["top_power"], pp, "s"), (gpu["top_count"], pc, "c")):
        prev = math.inf
        for t in lst:
            o = pos[t["index"]]
            assert t["n_valid"] == ref["N"][o]
            if key == "c":
                assert t["stat"] == ref["c"][o] and t["psi"] == pytest.approx(psi[o], rel=1e-13)
            else:
                assert abs(t["stat"] - ref["s"][o]) <= 1e-5 * ref["s"][o]
                assert abs(t["psi"] - psi[o]) <= tol[o] + 1e-12
            assert t["psi"] <= prev
            prev = t["psi"]
    # no sampled template outside the lists outranks the 10th candidate
    ok = ~np.isnan(pp) & ~np.isin(idx, top_p)
    assert np.all(pp[ok] <= gpu["top_power"][-1]["psi"] + tol[ok] + 1e-9)
    ok = ~np.isnan(pc) & ~np.isin(idx, top_c)
    assert np.all(pc[ok] <= gpu["top_count"][-1]["psi"] + 1e-12)
    assert gpu["diag"]["pow_undecided"] == 0
    assert gpu["diag"]["evals"] == grid.n_templates * det.n_seg


@pytest.mark.slow
def test_realistic_full_size_bin_checksum():
    """Bin checksum at full size: every sampled template's s (an exact integer)
    equals the oracle's, so every selected bin matches."""
    print("case: realistic full size, bin checksum", flush=True)
    det, grid, _ = _realistic_det(checksum=True)
    gpu = run_gpu([det], grid)
    idx = _sample_indices(grid.n_templates, seed=1)
    ref = oracle.evaluate_list(det, grid, idx)
    # sums reach 7e7 > 2^24, beyond what the FP32 output holds exactly; with
    # unit weights Psi = (s - N)/sqrt(N) in FP64 gives the exact sum back
    N = gpu["N"][idx].astype(np.float64)
    with np.errstate(invalid="ignore"):
        s_exact = np.where(N > 0, np.rint(gpu["psi_power"][idx] * np.sqrt(N) + N), 0.0)
    assert np.array_equal(s_exact, ref["s"])
    assert np.array_equal(gpu["N"][idx], ref["N"])
    assert np.array_equal(gpu["s"][idx], ref["s"].astype(np.float32).astype(np.float64))
    frac = gpu["diag"]["in_band"] / gpu["diag"]["evals"]
    assert 0.6 < frac < 0.8
