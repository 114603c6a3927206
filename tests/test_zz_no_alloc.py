"""GPU test of ltgw_eval_templates_noalloc, the evaluation that allocates no
device memory (every buffer is a slice of the library's static scratch
array), against ltgw_eval_templates on the same detector and grid.

Bar: the same kernels in the same order, so s, c and N are identical bit for
bit; two calls in a row, the second on a smaller search, so the second reads
a scratch array that still holds the first call's contents; the device's
free memory is unchanged across the calls.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _det(n_seg, n_bins, seed):
    """A weighted detector (noise-floor weights U[0.5, 2]: the fixed-point
    moments) with 8-s segments from 500 Hz."""
    t_sft, k_lo = 8.0, 4000
    t_seg = synth.segment_times(n_seg, t_sft)
    w = np.random.Generator(np.random.PCG64(seed + 1)).uniform(0.5, 2.0, n_seg).astype(np.float32)
    return dict(rho=synth.exp_noise(n_seg, n_bins, seed), t_seg=t_seg, v=synth.velocity(t_seg), k_lo=k_lo,
                t_sft=t_sft, weights=w)


def _grid(n_f0, n_tau, n_brake):
    return dict(f0_min=500.0, f0_step=0.125, n_f0=n_f0, tau=np.geomspace(3500.0, 35000.0, n_tau),
                brake=np.linspace(3.0, 7.0, n_brake), sky=synth.sky_vector(1.0, 0.3)[None, :], t0=0.0)


def _load(ctx, d):
    import torch

    ctx.load_spectrogram(0, torch.from_numpy(d["rho"]).cuda(), d["k_lo"], d["t_sft"], d["t_seg"],
                         weights=d["weights"])
    ctx.set_velocity_table(0, d["v"])


def _n(g):
    return g["n_f0"] * len(g["tau"]) * len(g["brake"]) * len(g["sky"])


def _reference(ctx, g):
    s, c, N = ctx.eval_templates(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    return s.cpu().numpy(), c.cpu().numpy(), N.cpu().numpy()


def _outputs(n):
    import torch

    return (torch.empty(n, dtype=torch.float32, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"),
            torch.empty(n, dtype=torch.int32, device="cuda"))


def _noalloc(ctx, g, out):
    from paper_2507_07816_amd import ltgw

    grid, _keep = ltgw.make_grid(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    ltgw.ltgw_eval_templates_noalloc(ctx.h, grid, ltgw.LTGW_STAT_POWER | ltgw.LTGW_STAT_COUNT, *out)


def _same(out, ref, what):
    s, c, N = (t.cpu().numpy() for t in out)
    assert np.array_equal(N, ref[2]), f"{what}: N differs"
    assert np.array_equal(c, ref[1]), f"{what}: c differs"
    assert np.array_equal(s.view(np.uint32), ref[0].view(np.uint32)), f"{what}: s differs"


@pytest.mark.parametrize("shape", [-1, 11])
def test_two_calls_second_smaller(shape):
    """2600 segments x 1200 bins; a ragged 1100-f0 x 6 tau x 4 n lattice, then
    300 f0 x 2 tau x 3 n, in the default tile shape and in the slab shape
    (segments walked in three slabs that resume from stored sums)."""
    from paper_2507_07816_amd import ltgw

    print(f"case: no-allocation evaluation, tile shape {shape}", flush=True)
    d = _det(2600, 1200, 31)
    big, small = _grid(1100, 6, 4), _grid(300, 2, 3)
    ctx = ltgw.Context(0)
    _load(ctx, d)
    ctx.set_tile_shape(shape)
    ref_big, ref_small = _reference(ctx, big), _reference(ctx, small)
    out_big, out_small = _outputs(_n(big)), _outputs(_n(small))
    _noalloc(ctx, big, out_big)
    assert ctx.diagnostics()["tile_shape"] == (1 if shape < 0 else shape)
    _noalloc(ctx, small, out_small)
    _same(out_big, ref_big, "first call")
    _same(out_small, ref_small, "second, smaller call")
    # the results are not kept: ranking needs an ltgw_eval_templates
    with pytest.raises(ltgw.LtgwError) as e:
        ctx.topk("power", 5)
    assert e.value.code == ltgw.LTGW_E_STATE
    ctx.close()


def test_allocates_nothing_and_rejects_oversized():
    """On a context whose only device buffers are the detector's, two calls
    (the second smaller) after a first one leave the device's free memory
    unchanged; a search
    beyond the scratch array is refused before anything is queued, and the
    next call still matches."""
    import torch
    from paper_2507_07816_amd import ltgw

    print("case: no-allocation evaluation, free memory and limits", flush=True)
    d = _det(2600, 1200, 37)
    big, small = _grid(1100, 6, 4), _grid(300, 2, 3)
    ref = ltgw.Context(0)
    _load(ref, d)
    ref_big, ref_small = _reference(ref, big), _reference(ref, small)
    ref.close()
    ctx = ltgw.Context(0)
    _load(ctx, d)
    out_big, out_small, out_w = _outputs(_n(big)), _outputs(_n(small)), _outputs(_n(small))
    # a first call lets the runtime set up the context's streams (its queues
    # are the runtime's, not the library's); the counted calls follow
    _noalloc(ctx, small, out_w)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _noalloc(ctx, big, out_big)
    _noalloc(ctx, small, out_small)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    _same(out_w, ref_small, "warm-up call")
    _same(out_big, ref_big, "first call")
    _same(out_small, ref_small, "second, smaller call")
    # 4,000,000 f0 x 24 groups: about 3 GB of per-template sums
    huge = _grid(4000000, 6, 4)
    with pytest.raises(ltgw.LtgwError) as e:
        _noalloc(ctx, huge, (None, None, None))
    assert e.value.code == ltgw.LTGW_E_UNSUPPORTED and "scratch" in str(e.value)
    too_many = _grid(300, ltgw.LTGW_NOALLOC_MAX_AXIS + 1, 1)
    with pytest.raises(ltgw.LtgwError) as e:
        _noalloc(ctx, too_many, (None, None, None))
    assert e.value.code == ltgw.LTGW_E_UNSUPPORTED
    out2 = _outputs(_n(small))
    _noalloc(ctx, small, out2)
    _same(out2, ref_small, "call after the refusals")
    ctx.close()


@pytest.mark.slow
def test_realistic_day_then_smaller():
    """The realistic day (10800 segments x 8000 bins, 2,304,000 templates) in
    the tile shape the autotuner picks for it, then a smaller lattice on the
    same detector."""
    from paper_2507_07816_amd import ltgw

    print("case: no-allocation evaluation, realistic day", flush=True)
    wl = synth.realistic()
    d = wl.dets[0]
    big = dict(wl.grid)
    small = _grid(3000, 8, 3)
    ctx = ltgw.Context(0)
    _load(ctx, d)
    tuned = ctx.autotune(big["f0_min"], big["f0_step"], big["n_f0"], big["tau"], big["brake"], big["sky"],
                         big["t0"])
    ref_big, ref_small = _reference(ctx, big), _reference(ctx, small)
    out_big, out_small = _outputs(_n(big)), _outputs(_n(small))
    _noalloc(ctx, big, out_big)
    assert ctx.diagnostics()["tile_shape"] == tuned
    _noalloc(ctx, small, out_small)
    _same(out_big, ref_big, "realistic day")
    _same(out_small, ref_small, "smaller lattice after it")
    ctx.close()
