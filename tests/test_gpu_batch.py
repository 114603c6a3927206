"""GPU tests of the batched path: many uneven searches in one persistent,
graph-captured launch, tile shapes and the autotuner.

- every search of a batch equals its own single-search evaluation bit for bit
  (the batch forms the track factor on the fly with the same operations),
  and a sample of them the oracle;
- a replayed graph reads the live buffers (new data in the same slot) and
  is rebuilt when what it baked in changes (weights);
- every tile shape gives bit-identical results;
- the tuning cache round-trips through its JSON file.
"""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_util import assert_sums_close, assert_topk_count

pytestmark = pytest.mark.gpu

SKY = np.array([[0.6, 0.0, 0.8], [0.0, -1.0, 0.0], [0.48, 0.6, 0.64], [-0.6, 0.8, 0.0]])


def _det(seed, n_seg, n_bins, k_lo, weights, t_sft=4.0, spacing=40.0):
    r = np.random.default_rng(seed)
    t_seg = np.arange(n_seg) * spacing + 2.0
    v = r.normal(size=(n_seg, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * 2.0e5
    rho = r.exponential(size=(n_seg, n_bins)).astype(np.float32)
    if weights == "rand":
        w = r.uniform(0.5, 2.0, n_seg).astype(np.float32)
    elif weights is None:
        w = None
    else:
        w = np.full(n_seg, weights, np.float32)
    return oracle.Detector(rho, t_seg, v, k_lo, t_sft, weights=w)


def _setup(ctx, store="f32"):
    import torch

    dets = [_det(1, 300, 256, 1900, "rand"), _det(2, 200, 400, 1880, None),
            _det(3, 150, 300, 1890, None), _det(4, 77, 200, 1910, 0.5),
            _det(5, 120, 256, 1900, None), _det(6, 90, 256, 1905, None)]
    for d, det in enumerate(dets):
        ctx.load_spectrogram(d, torch.from_numpy(det.rho).cuda(), det.k_lo, det.t_sft, det.t_seg,
                             weights=det.w, store=store)
        ctx.set_velocity_table(d, det.v)
    searches = [
        dict(f0_min=478.0, f0_step=0.25, n_f0=300, tau=[5000.0, 20000.0], brake=[3.0, 5.0],
             sky=SKY[:2], t0=0.0, dets=[0]),
        dict(f0_min=474.0, f0_step=0.25, n_f0=257, tau=[3500.0, 35000.0], brake=[5.0], sky=SKY[:3],
             t0=0.0, dets=[1, 2]),
        dict(f0_min=480.0, f0_step=0.125, n_f0=513, tau=[7000.0], brake=[2.5, 7.0], sky=SKY[:1],
             t0=0.0, dets=[3]),
        dict(f0_min=476.0, f0_step=0.5, n_f0=100, tau=[9000.0, 30000.0], brake=[4.0], sky=SKY,
             t0=1500.0, dets=[4, 5]),
        dict(f0_min=490.0, f0_step=0.25, n_f0=64, tau=[12000.0], brake=[3.0, 6.0], sky=SKY[2:],
             t0=0.0, dets=[0]),
    ]
    return dets, searches


def _n_tpl(s):
    return s["n_f0"] * len(s["tau"]) * len(s["brake"]) * len(s["sky"])


def _single(ctx, s):
    mask = sum(1 << d for d in s["dets"])
    out = ctx.eval_templates(s["f0_min"], s["f0_step"], s["n_f0"], s["tau"], s["brake"], s["sky"],
                             s["t0"], det_mask=mask)
    n = _n_tpl(s)
    return {"s": out[0].cpu().numpy(), "c": out[1].cpu().numpy(), "N": out[2].cpu().numpy(),
            "pp": ctx.psi("power", n).cpu().numpy(), "pc": ctx.psi("count", n).cpu().numpy(),
            "top_p": ctx.topk("power", 8), "top_c": ctx.topk("count", 8)}


def _batch(ctx, i, s):
    s_, c, N, pp, pc = ctx.batch_results(i, _n_tpl(s))
    return {"s": s_.cpu().numpy(), "c": c.cpu().numpy(), "N": N.cpu().numpy(),
            "pp": pp.cpu().numpy(), "pc": pc.cpu().numpy()}


def _same(a, b):
    for k in ("s", "c", "N", "pp", "pc"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_batch_equals_single_searches_and_oracle():
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets, searches = _setup(ctx)
    print("case: batch of 5 uneven searches", flush=True)
    top_p, top_c, st = ctx.eval_batch(searches, k=8)
    assert st["graph_replayed"] == 0 and 0 <= st["variant"] <= 3
    assert st["templates"] == sum(_n_tpl(s) for s in searches)
    lat = ctx.batch_latency(len(searches))
    assert np.all(lat > 0) and lat.max() <= st["kernel_ms"] + 1e-6
    batch = [_batch(ctx, i, s) for i, s in enumerate(searches)]
    for i, s in enumerate(searches):
        single = _single(ctx, s)
        _same(batch[i], single)
        assert [t["index"] for t in top_p[i]] == [t["index"] for t in single["top_p"]]
        assert [t["index"] for t in top_c[i]] == [t["index"] for t in single["top_c"]]
    # against the oracle: the two-detector search and the masked one
    for i in (1, 3):
        s = searches[i]
        grid = oracle.Grid(s["f0_min"], s["f0_step"], s["n_f0"], s["tau"], s["brake"], s["sky"], s["t0"])
        ref = oracle.evaluate([dets[d] for d in s["dets"]], grid)
        assert np.array_equal(batch[i]["N"], ref["N"])
        assert np.array_equal(batch[i]["c"], ref["c"])
        assert_sums_close(batch[i]["s"].astype(np.float64), ref["s"])
        assert_topk_count(top_c[i], ref, 8)
    ctx.close()


def test_graph_replay_reads_live_buffers():
    import torch
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets, searches = _setup(ctx)
    ctx.eval_batch(searches, k=5)
    first = [_batch(ctx, i, s) for i, s in enumerate(searches)]
    for rep in range(3):
        _single(ctx, searches[rep])  # eager work between replays
        _, _, st = ctx.eval_batch(searches, k=5)
        assert st["graph_replayed"] == 1
        for i, s in enumerate(searches):
            _same(_batch(ctx, i, s), first[i])
    # new data in slot 0, same shape and weights: the graph is replayed and sees it
    d0 = dets[0]
    rho2 = np.random.default_rng(99).exponential(size=d0.rho.shape).astype(np.float32)
    ctx.load_spectrogram(0, torch.from_numpy(rho2).cuda(), d0.k_lo, d0.t_sft, d0.t_seg, weights=d0.w)
    ctx.set_velocity_table(0, d0.v)
    _, _, st = ctx.eval_batch(searches, k=5)
    assert st["graph_replayed"] == 1
    for i in (0, 4):
        _same(_batch(ctx, i, searches[i]), _single(ctx, searches[i]))
    # new weights change what the graph baked in: rebuilt
    w2 = np.random.default_rng(7).uniform(0.5, 2.0, d0.n_seg).astype(np.float32)
    ctx.load_spectrogram(0, torch.from_numpy(rho2).cuda(), d0.k_lo, d0.t_sft, d0.t_seg, weights=w2)
    ctx.set_velocity_table(0, d0.v)
    _, _, st = ctx.eval_batch(searches, k=5)
    assert st["graph_replayed"] == 0
    _same(_batch(ctx, 0, searches[0]), _single(ctx, searches[0]))
    ctx.close()


def test_tile_shapes_are_bit_identical():
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets, searches = _setup(ctx)
    ref_single, ref_batch = None, None
    for v in range(16):
        print(f"case: tile shape {v}", flush=True)
        ctx.set_tile_shape(v)
        single = _single(ctx, searches[1])
        assert ctx.diagnostics()["tile_shape"] == v
        _, _, st = ctx.eval_batch(searches, k=5)
        assert st["variant"] == v % 4
        batch = [_batch(ctx, i, s) for i, s in enumerate(searches)]
        if ref_single is None:
            ref_single, ref_batch = single, batch
        _same(single, ref_single)
        for a, b in zip(batch, ref_batch):
            _same(a, b)
    ctx.close()


def test_autotune_and_cache_roundtrip(tmp_path):
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets, searches = _setup(ctx)
    s = searches[2]
    best = ctx.autotune(s["f0_min"], s["f0_step"], s["n_f0"], s["tau"], s["brake"], s["sky"], s["t0"],
                        det_mask=1 << s["dets"][0])
    assert 0 <= best <= 15
    _single(ctx, s)
    assert ctx.diagnostics()["tile_shape"] == best
    _, _, st = ctx.eval_batch(searches, k=5)
    path = tmp_path / "tune.json"
    ctx.tune_save(str(path))
    cache = json.loads(path.read_text())["ltgw_tune"]
    assert any(k.startswith("eval/") for k in cache) and any(k.startswith("batch/") for k in cache)
    assert set(cache.values()) <= set(range(16))
    ctx.close()
    # a fresh context takes the shapes from the file
    ctx2 = ltgw.Context(0)
    _setup(ctx2)
    ctx2.tune_load(str(path))
    _single(ctx2, s)
    assert ctx2.diagnostics()["tile_shape"] == best
    _, _, st2 = ctx2.eval_batch(searches, k=5)
    assert st2["variant"] == st["variant"]
    bad = tmp_path / "bad.json"
    bad.write_text('{"ltgw_tune": {"eval/x": 19}}')   # no such variant
    with pytest.raises(ltgw.LtgwError):
        ctx2.tune_load(str(bad))
    with pytest.raises(ltgw.LtgwError):
        ctx2.tune_load(str(tmp_path / "missing.json"))
    ctx2.close()


def test_batch_quantised_store_matches_single():
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets, searches = _setup(ctx, store="bf16")
    ctx.eval_batch(searches, k=5)
    for i, s in enumerate(searches):
        _same(_batch(ctx, i, s), _single(ctx, s))
    ctx.close()


def test_batch_errors():
    import torch
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets, searches = _setup(ctx)
    E = ltgw.LtgwError
    with pytest.raises(E) as ei:
        ctx.eval_batch([dict(searches[0], dets=[9])], k=5)          # slot 9 not loaded
    assert ei.value.code == ltgw.LTGW_E_STATE
    with pytest.raises(E):
        ctx.eval_batch(searches, k=0)
    with pytest.raises(E):
        ctx.eval_batch([dict(searches[0], brake=[1.0])], k=5)
    d = dets[5]
    ctx.load_spectrogram(5, torch.from_numpy(d.rho).cuda(), d.k_lo, d.t_sft, d.t_seg, store="fp8")
    ctx.set_velocity_table(5, d.v)
    with pytest.raises(E) as ei:
        ctx.eval_batch(searches, k=5)                                 # search 3 mixes stores
    assert ei.value.code == ltgw.LTGW_E_UNSUPPORTED
    with pytest.raises(E) as ei:
        ltgw.ltgw_batch_results(ctx.h, 0)                              # the failed batch left none
    assert ei.value.code == ltgw.LTGW_E_STATE
    # still usable
    top_p, top_c, st = ctx.eval_batch(searches[:3], k=5)
    assert len(top_p) == 3 and st["graph_replayed"] == 0
    ctx.close()


def test_slabs_and_generations_are_bit_identical_on_long_searches():
    """Variants that split the statistic launch (generations, segment slabs of
    1024) give the same bits as one launch, here with 2600 segments (three
    slabs, a ragged last one) and uneven weights (moments in the loop)."""
    import torch
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    r = np.random.default_rng(11)
    n_seg, n_bins = 2600, 300
    t_seg = np.arange(n_seg) * 8.0 + 4.0
    v = r.normal(size=(n_seg, 3))
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * 3.0e4
    rho = r.exponential(size=(n_seg, n_bins)).astype(np.float32)
    for weights in (None, r.uniform(0.5, 2.0, n_seg).astype(np.float32),
                    np.exp(r.uniform(-6, 6, n_seg)).astype(np.float32)):
        ctx.load_spectrogram(0, torch.from_numpy(rho).cuda(), 3990, 8.0, t_seg, weights=weights)
        ctx.set_velocity_table(0, v)
        ref = None
        for var in (0, 1, 2, 3, 4, 7, 8, 11, 12, 15):
            print(f"case: slab/generation variant {var}", flush=True)
            ctx.set_tile_shape(var)
            s_, c, N = ctx.eval_templates(500.0, 0.125, 700, [3500.0, 20000.0], [3.0, 5.0],
                                          [[0.6, 0.0, 0.8], [0.0, 1.0, 0.0]], 0.0)
            got = (s_.cpu().numpy(), c.cpu().numpy(), N.cpu().numpy(), ctx.psi("power", s_.numel()).cpu().numpy())
            if ref is None:
                ref = got
            for a, b in zip(got, ref):
                assert np.array_equal(a, b, equal_nan=True), var
    ctx.close()


def test_batch_long_ragged_searches_equal_single_and_oracle():
    """Longer searches with segment counts that are not whole chunks: two
    detectors of 1500 and 1333 segments, one detector of 1100, and a short
    search beside them.  Every search equals its own single search bit for
    bit, and the oracle."""
    import torch
    from paper_2507_07816_amd import ltgw

    ctx = ltgw.Context(0)
    dets = [_det(11, 1500, 200, 1900, "rand", spacing=20.0), _det(12, 1333, 200, 1905, None, spacing=22.0),
            _det(13, 1100, 160, 1910, 0.75, spacing=25.0), _det(14, 90, 128, 1900, None)]
    for d, det in enumerate(dets):
        ctx.load_spectrogram(d, torch.from_numpy(det.rho).cuda(), det.k_lo, det.t_sft, det.t_seg,
                             weights=det.w)
        ctx.set_velocity_table(d, det.v)
    searches = [
        dict(f0_min=476.0, f0_step=0.25, n_f0=160, tau=[3500.0, 20000.0], brake=[3.0, 6.0], sky=SKY[:2],
             t0=0.0, dets=[0, 1]),
        dict(f0_min=478.0, f0_step=0.25, n_f0=130, tau=[9000.0], brake=[5.0], sky=SKY[2:], t0=300.0, dets=[2]),
        dict(f0_min=476.0, f0_step=0.5, n_f0=70, tau=[12000.0], brake=[4.0], sky=SKY[:1], t0=0.0, dets=[3]),
    ]
    print("case: batch of long ragged searches", flush=True)
    top_p, top_c, st = ctx.eval_batch(searches, k=8)
    batch = [_batch(ctx, i, s) for i, s in enumerate(searches)]
    for i, s in enumerate(searches):
        single = _single(ctx, s)
        _same(batch[i], single)
        grid = oracle.Grid(s["f0_min"], s["f0_step"], s["n_f0"], s["tau"], s["brake"], s["sky"], s["t0"])
        ref = oracle.evaluate([dets[d] for d in s["dets"]], grid)
        assert np.array_equal(batch[i]["N"], ref["N"])
        assert np.array_equal(batch[i]["c"], ref["c"])
        assert_sums_close(batch[i]["s"].astype(np.float64), ref["s"])
        assert_topk_count(top_c[i], ref, 8)
    lat = ctx.batch_latency(len(searches))
    assert np.all(lat > 0) and lat.max() <= st["kernel_ms"] + 1e-6
    ctx.close()
