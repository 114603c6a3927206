"""Benchmark: template x segment evaluations per second of the detection statistic.

One step is one pass of the whole search over the resident data:
  load_spectrogram (device FP32 power -> store with the count bit),
  set_velocity_table, eval_templates (Eq. 1 powers, Eq. 2 factors, the
  statistic kernel), and topk_candidates for the power and the count.
Workload (default): the realistic single search -- 10800 segments of 8 s
(24 h), 500-1500 Hz at 0.125 Hz (8000 bins), FP32 Exp(1) power with
U[0.5, 2] per-segment weights and 20 injected tracks; 8000 f0 x 32 tau x 9 n
x 1 sky = 2,304,000 templates, i.e. 2.49e10 template x segment evaluations.

Prints one JSON line.  The roofline object is for the statistic kernel, per
launch: the HBM-side bytes its committed rocprofv3 counter runs measured
(copy-calibrated FETCH_SIZE + WRITE_SIZE) over its average launch duration
from HIP events recorded around its launches on the stream they run on,
against the HBM peak; beside it the algorithmic bytes (in-band evaluations x
stored bytes per element, mostly served by the caches) and the gather-path
unit that binds.  Further legs: the same search with BF16 and FP8 stores,
antenna-pattern weights, the uniform random bank, data preparation, the
sensitivity campaign, the 64-search batch and the learned proposer.  The CPU
baseline is the FP64 oracle timed on this host's cores over a bounded sample
of the same workload (every template when that fits); the stores' errors
against FP64 are taken on that sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("template·segment evals/s, %HBM roofline; learned+BF16 vs plain FP32 at "
          "≥99% recall")
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
BYTES = {"f32": 4, "bf16": 2, "fp8": 1}


# the statistic kernel's code: a change to any of these voids the committed counters
KERNEL_SOURCES = ("paper_2507_07816_amd/csrc/ltgw_kernels.hip", "paper_2507_07816_amd/csrc/ltgw_gather.h",
                  "paper_2507_07816_amd/csrc/ddpow.h", "paper_2507_07816_amd/csrc/ltgw_internal.h",
                  "paper_2507_07816_amd/csrc/exp2_table.h", "paper_2507_07816_amd/csrc/log_table.h")


# the explicit-template kernel's code (its committed FP64 instruction count)
LIST_SOURCES = ("paper_2507_07816_amd/csrc/ltgw_list.hip", "paper_2507_07816_amd/csrc/ltgw_list.h",
                "paper_2507_07816_amd/csrc/ddpow.h", "paper_2507_07816_amd/csrc/pow_enclose.h",
                "paper_2507_07816_amd/csrc/ltgw_gather.h",
                "paper_2507_07816_amd/csrc/ltgw_antenna.h", "paper_2507_07816_amd/csrc/exp2_table.h",
                "paper_2507_07816_amd/csrc/log_table.h")


def kernel_source_hash(sources=KERNEL_SOURCES):
    import hashlib

    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_list_counts():
    """Executed VALU and FP64 lane-instructions per evaluation of the
    explicit-template kernel, from the committed rocprofv3 counter summary
    (SQ_INSTS_VALU and SQ_INSTS_VALU_*_F64 over the launch, times 64 lanes,
    over its evaluations), or None when it is for another kernel source."""
    path = os.path.join(ROOT, "profiles", "list_kernel_fp64.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != kernel_source_hash(LIST_SOURCES):
        return None
    return {"valu": t["valu_lane_instructions_per_eval"], "fp64": t["fp64_lane_instructions_per_eval"]}


def measured_valu(workload, store, variant):
    """VALU lane-instructions per template x segment evaluation of the
    statistic kernel from the committed counter summary (same kernel source,
    workload, store and tile shape), or None."""
    path = os.path.join(ROOT, "profiles", "eval_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if (t.get("source_sha256") != kernel_source_hash() or t.get("workload") != workload
            or t.get("store") != store or t.get("variant") != variant):
        return None
    return t.get("valu_lane_instructions_per_eval")


def cpu_baseline(wl, rho, target_s=20.0, full_factor=1.5):
    """Oracle throughput on this host over a bounded sample of the workload:
    whole (tau, n) groups of all f0, all segments; every template when the
    whole workload fits in full_factor x target_s.  Returns the JSON object
    and the oracle's statistic of the sampled templates (index, s, c, N and
    the critical ratios; with every template also its two top-10 lists), which
    the precision report compares the device's stores against."""
    import oracle

    d = wl.dets[0]
    g = wl.grid
    det = oracle.Detector(rho, d["t_seg"], d["v"], d["k_lo"], d["t_sft"], weights=d["weights"])
    grid = oracle.Grid(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    n_seg = det.n_seg
    # calibrate on 1/4 of one group, then size the sample to ~target_s
    probe = np.arange(0, grid.n_f0 // 4, dtype=np.int64) + grid.n_f0 * 3
    t = time.perf_counter()
    oracle.evaluate_list(det, grid, probe)
    dt = time.perf_counter() - t
    rate = probe.size * n_seg / dt
    n_all = grid.n_templates
    full = n_all * n_seg / rate <= full_factor * target_s
    n_groups_all = n_all // grid.n_f0
    if full:
        t = time.perf_counter()
        res = oracle.evaluate(det, grid)
        dt = time.perf_counter() - t
        idx = np.arange(n_all, dtype=np.int64)
        sample = f"every template: {n_groups_all} (tau, n) groups x {grid.n_f0} f0 x {n_seg} segments"
    else:
        n_tpl = int(min(n_all, max(grid.n_f0, rate * target_s / n_seg)))
        n_groups = max(1, n_tpl // grid.n_f0)
        groups = np.linspace(0, n_groups_all - 1, n_groups).astype(np.int64)
        idx = (groups[:, None] * grid.n_f0 + np.arange(grid.n_f0)[None, :]).ravel()
        t = time.perf_counter()
        res = oracle.evaluate_list(det, grid, idx)
        dt = time.perf_counter() - t
        sample = f"{n_groups} (tau, n) groups x {grid.n_f0} f0 x {n_seg} segments"
    ref = dict(idx=idx, s=res["s"], c=res["c"], N=res["N"], psi_power=oracle.psi_power(res),
               psi_count=oracle.psi_count(res), full=full)
    if full:
        ref["top_power"] = [int(i) for i in oracle.topk(ref["psi_power"], 10)]
        ref["top_count"] = [int(i) for i in oracle.topk(ref["psi_count"], 10)]
        # largest change of a power ratio the float-sum tolerance allows (near-ties may swap)
        with np.errstate(invalid="ignore", divide="ignore"):
            ref["psi_tol"] = 1e-5 * np.abs(res["s"]) / np.sqrt(res["W2"])
    out = {"value": idx.size * n_seg / dt, "unit": "template·segment evals/s",
           "cores": oracle.threads(), "kind": "oracle", "cpu": cpu_model(),
           "sample": f"{sample} ({idx.size * n_seg:.3g} evals, {dt:.1f} s, FP64, incl. its Eq. 1 table)"}
    return out, ref


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def precision_report(ref, runs):
    """Per-result error of each store's statistic against the FP64 oracle of
    the CPU baseline (the same templates), and top-10 agreement.  runs: store
    -> dict of the device's s (FP32 output), c, N over every template and its
    top-10 lists."""
    idx = ref["idx"]
    out = {"reference": "FP64 oracle over " + ("every template" if ref["full"] else f"{idx.size} templates")}
    for store, r in runs.items():
        s = r["s"][idx].astype(np.float64)
        nz = ref["s"] != 0
        rel = np.abs(s[nz] - ref["s"][nz]) / np.abs(ref["s"][nz])
        e = {"max_rel_s": float(rel.max()), "mean_rel_s": float(rel.mean()),
             "n_mismatches": int(np.count_nonzero(r["N"][idx] != ref["N"])),
             "count_mismatches": int(np.count_nonzero(r["c"][idx] != ref["c"]))}
        if ref["full"]:
            e["top10_count_identical"] = r["top_count"] == ref["top_count"]
            e["top10_power_identical"] = r["top_power"] == ref["top_power"]
            e["top10_power_same_set"] = sorted(r["top_power"]) == sorted(ref["top_power"])
            # rank by rank within the ratio tolerance of the float sum
            pp, tol = ref["psi_power"], ref["psi_tol"]
            e["top10_power_within_tolerance"] = bool(all(
                abs(pp[a] - pp[b]) <= 2 * max(tol[a], tol[b]) + 1e-12
                for a, b in zip(r["top_power"], ref["top_power"])))
        out[store] = e
    return out


def proposer_leg(torch, ltgw, realisations=50000, batch=256, epochs=16, eval_signal=4096, eval_noise=1024, seed=7,
                 coarse_segments=8, select2_frac=0.0, block=32, label="near", select_blocks=(8, 10, 11, 12),
                 tier2_quantile=None, counts=True):
    """The learned proposer on the small workload's shape (1024 segments x 800
    bins, 4800 fine templates): trained on `realisations` device-generated
    noise + injection realisations (amplitudes U[0.3, 3]), then recall and
    speed against the plain FP32 exhaustive search at each first-tier budget
    (select_blocks blocks of `block` f0 per realisation: 256, 320, 352 and 384
    of the 4800 cells) and fallback quantile; the point reported is the fastest
    at recall 0.99, else the best recall at 5x or more, and best_at_5x is the
    best recall at 5x or more.  Beside it, the ranking by the coarse power
    ratios alone at the reported budget (the method without the network).
    Returns the JSON object."""
    import synth
    from paper_2507_07816_amd.proposer import Proposer, coarse_grid_for

    wl = synth.tiny(with_noise=False)
    d, g = wl.dets[0], wl.grid
    ctx = ltgw.Context(0)
    dev = torch.device("cuda", 0)
    ctx.load_spectrogram(0, torch.zeros(d["rho"].shape, dtype=torch.float32, device=dev), d["k_lo"],
                         d["t_sft"], d["t_seg"], weights=d["weights"])
    ctx.set_velocity_table(0, d["v"])
    fine = dict(g)
    tau, brake = np.asarray(g["tau"]), np.asarray(g["brake"])
    # 2x coarser in f0, tau and n: pair means (geometric for tau)
    ctau = np.sqrt(tau[0::2] * tau[1::2])
    cbrake = np.array([(brake[0] + brake[1]) / 2, (brake[-2] + brake[-1]) / 2])
    coarse = coarse_grid_for(fine, ctau, cbrake)
    pr = Proposer(ctx, 0, d["rho"].shape, fine, coarse, seed=seed, select_frac=0.05, store="f32",
                  block=block, select2_frac=select2_frac, coarse_segments=coarse_segments, counts=counts)
    steps = max(1, realisations // batch)
    torch.cuda.synchronize()
    t = time.perf_counter()
    losses = pr.train(steps * batch, batch=batch, epochs=epochs, p_signal=0.9, amp_range=(0.3, 3.0), lr=2e-3,
                      label_psi=4.5, label=label)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    ev = pr.evaluate(R_noise=eval_noise, R_signal=eval_signal, amp_range=(0.3, 3.0), fine_store="bf16",
                     coarse_quantiles=(None, 1.0, 0.9, 0.7), tier2_quantile=tier2_quantile,
                     budgets=[k * block for k in select_blocks])
    ctx.close()
    base = ev.pop("coarse_only")
    out = {"workload": "tiny-1024seg-800bin-4800tpl realisations", "train_realisations": steps * batch,
           "epochs": epochs, "label_psi": 4.5, "label": label,
           "train_s": train_s, "loss_first": float(np.mean(losses[:5])), "loss_last": float(np.mean(losses[-5:])),
           "coarse_grid": f"{coarse['n_f0']} f0 x {len(ctau)} tau x {len(cbrake)} n over {coarse_segments} segments",
           "network": f"4-layer CNN, BF16 MFMA, {pr.c_in} input channels (coarse power{' and count' if counts else ''}"
                      " ratios)",
           "speedup_counts": "exhaustive FP32 search / (ltgw_propose + the coarse store's extra ingest time)"}
    out.update(ev)
    fast = [p for p in ev["points"] if p["speedup"] >= 5.0]
    out["best_at_5x"] = None if not fast else {k: v for k, v in max(fast, key=lambda p: p["recall"]).items()
                                               if k in ("n_select", "coarse_quantile", "recall",
                                                        "recall_same_template", "recall_best", "fallback_frac",
                                                        "propose_ms", "speedup")}
    out["coarse_only"] = {k: base[k] for k in ("n_select", "recall", "recall_no_fallback", "recall_same_template",
                                               "recall_best", "fallback_frac", "propose_ms", "speedup",
                                               "coarse_quantile")}
    return out


# vector instruction issue of the chip: 256 CUs x 64 lanes x 2.4 GHz (FP64
# included: the 78.6 TFLOP/s FP64 peak counts each FMA as 2 flops)
FP64_LANE_OPS = 256 * 64 * 2.4e9


def list_leg(torch, ltgw, ctx, wl, n=1000000, reps=3, seed=11, counts=None):
    """The uniform random bank over the loaded search: n templates drawn
    uniformly in f0 (the band), tau and n, at the search's sky point.  Every
    (template, segment) takes its own Eq. 1 power: an FP64 enclosure of the
    correctly rounded value, and that value itself where the enclosure leaves
    the column open (pow_exact_fraction).  The rate is compared with the
    chip's VALU lane-instruction rate given the instructions per evaluation
    counted by rocprofv3 for this kernel source."""
    import synth

    d = wl.dets[0]
    g = wl.grid
    f_hi = g["f0_min"] + (d["rho"].shape[1] - 1) * g["f0_step"]
    params = synth.random_bank(n, (g["f0_min"], f_hi), (float(g["tau"][0]), float(g["tau"][-1])),
                               (float(g["brake"][0]), float(g["brake"][-1])), g["sky"][0], seed)
    ctx.eval_list(params, g["t0"], outputs=False)            # warm-up
    torch.cuda.synchronize()
    dg0 = ctx.diagnostics()
    runs = []
    for _ in range(reps):
        t = time.perf_counter()
        ctx.eval_list(params, g["t0"], outputs=False)
        dg = ctx.diagnostics()                                 # synchronises
        runs.append((time.perf_counter() - t, dg["eval_kernel_ms"]))
    wall = min(r[0] for r in runs)
    kms = float(np.mean([r[1] for r in runs]))
    evals = int(dg["evals"])
    out = {"workload": f"uniform random bank, {n} templates over {wl.name}, seed {seed}",
           "templates": n, "evals": evals, "in_band_fraction": dg["in_band"] / evals,
           "value": evals / wall, "unit": "template·segment evals/s", "wall_ms": wall * 1e3,
           "kernel_ms": kms, "kernel_evals_per_s": evals / (kms * 1e-3),
           "pow_undecided": int(dg["pow_undecided"]),
           "pow_exact_fraction": (dg["pow_exact"] - dg0["pow_exact"]) / (reps * evals),
           "pow_slow_fraction": (dg["pow_slow"] - dg0["pow_slow"]) / (reps * evals)}
    if counts:
        rate = counts["valu"] * evals / (kms * 1e-3)
        out["roofline"] = {"bound": "alu", "achieved": rate / 1e12, "peak": FP64_LANE_OPS / 1e12,
                           "unit": "T VALU lane-instructions/s", "frac": rate / FP64_LANE_OPS,
                           "valu_instructions_per_eval": counts["valu"],
                           "fp64_instructions_per_eval": counts["fp64"],
                           "fp64_frac": counts["fp64"] * evals / (kms * 1e-3) / FP64_LANE_OPS}
    return out


def antenna_leg(torch, ltgw, ctx, wl, power, t_seg, v, w, store, steps=5):
    """The realistic search with antenna-pattern weights on (the H-site arms,
    Earth rotation angles of the segment times): one weight row per sky point,
    W1 and W2 summed by the statistic kernel.  Same step as the headline."""
    import synth

    d = wl.dets[0]
    g = wl.grid
    arms = synth.site_arms(*synth.SITE_H, synth.ARM_AZ_H)
    era = synth.earth_rotation_angle(d["t_seg"])

    def step():
        ctx.load_spectrogram(0, power, d["k_lo"], d["t_sft"], t_seg, weights=w, store=store)
        ctx.set_velocity_table(0, v)
        ctx.set_antenna(0, arms, era)
        ctx.eval_templates(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"],
                           outputs=False)
        ctx.topk("power", 10)
        ctx.topk("count", 10)
        return ctx.diagnostics()

    step()
    # the tile shape for this search with in-kernel moments (the autotuner's cache key includes the mode)
    ctx.autotune(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    step()
    torch.cuda.synchronize()
    t = time.perf_counter()
    kms = []
    for _ in range(steps):
        dg = step()
        kms.append(dg["eval_kernel_ms"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    ctx.set_antenna(0, None)
    kms_mean = float(np.mean(kms))
    launches = max(int(dg["eval_launches"]), 1)
    alg_bytes = dg["in_band"] * BYTES[store] / launches
    achieved = alg_bytes / (kms_mean / launches * 1e-3) / 1e9
    return {"workload": f"{wl.name} with H-site antenna-pattern weights", "steps": steps,
            "value": dg["evals"] * steps / el, "unit": "template·segment evals/s", "ms_per_step": el * 1e3 / steps,
            "eval_kernel_ms": kms_mean, "eval_launches_per_step": launches,
            "tile_shape": int(dg["tile_shape"]),
            "algorithmic": {"gbs": achieved, "x_hbm_peak": achieved / HBM_PEAK_GBS, "bytes_per_launch": alg_bytes,
                            "unit": "one stored element per in-band template x segment evaluation"}}


def campaign_leg(torch, ltgw, R_noise=256, amps=(0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0),
                 per_level=100, seed=2024):
    """The synthetic sensitivity campaign (Sec. 3) on the small workload's
    geometry (1024 segments x 800 bins, U[0.5, 2] weights): thresholds from
    R_noise noise-only full searches, per_level injections (f0 uniform in the
    band, tau = 10000 s, n = 5) at each amplitude, detection near the
    injection, logistic fit and A90 (reported only inside the sampled
    amplitudes), for the power and the count statistic, over the cubic
    lattice (4800 templates; realisations in stacks) and a uniform random
    bank of as many templates (one realisation at a time).  The cubic
    campaign is timed after one untimed run of it."""
    import synth
    from paper_2507_07816_amd.campaign import Campaign

    wl = synth.tiny()
    d = wl.dets[0]
    w = np.random.Generator(np.random.PCG64(55)).uniform(0.5, 2.0, d["rho"].shape[0]).astype(np.float32)
    geo = dict(t_seg=d["t_seg"], v=d["v"], weights=w, k_lo=d["k_lo"], t_sft=d["t_sft"], n_bins=d["rho"].shape[1])
    g = dict(wl.grid)
    out = {"workload": f"{wl.name}: {R_noise} noise-only realisations, {len(amps)} amplitudes x {per_level} "
                       "injections (tau 10000 s, n 5)", "amplitudes": list(amps)}
    ctx = ltgw.Context(0)
    try:
        for bank_name in ("cubic", "random"):
            bank = None if bank_name == "cubic" else synth.random_bank(
                wl.n_templates, (500.0, 600.0), (3500.0, 35000.0), (3.0, 7.0), g["sky"][0], seed=56)
            if bank is None:
                # one untimed run first: the stack path's kernels and buffers are
                # first used here (about 60 ms of one-time cost in a fresh process)
                Campaign(ctx, geo, g, bank=bank, seed=seed).run(list(amps), per_level, R_noise,
                                                                 f0_range=(505.0, 595.0), tau=10000.0, brake=5.0)
            camp = Campaign(ctx, geo, g, bank=bank, seed=seed)
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = camp.run(list(amps), per_level, R_noise, f0_range=(505.0, 595.0), tau=10000.0, brake=5.0)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t
            n_real = R_noise + len(amps) * per_level
            out[bank_name] = {"templates": int(wl.n_templates), "wall_s": wall, "realisations_per_s": n_real / wall,
                              "path": ("stacks of realisations: full searches and near-injection lists per stack"
                                       if bank is None else
                                       "one realisation per search through the C ABI (host-bound)"),
                              **{name: {"threshold": res["threshold"][name],
                                        "efficiency": [float(x) for x in res[name]["efficiency"]],
                                        "a90": res[name]["a90"],
                                        "a90_fitted": res[name]["fit"]["a90"],
                                        "a90_in_sampled_range": res[name]["a90_in_sampled_range"]}
                                 for name in ("power", "count")}}
    finally:
        ctx.close()
    return out


def sft_leg(torch, ltgw, n_seg=10800, n_fft=32768, k_lo=4000, n_bins=8000, window=101, reps=3, seed=17):
    """Data preparation: 24 h of 4096-Hz strain (Gaussian, seeded, generated
    on the device) in 10,800 segments of 8 s -> Hann-windowed FP32 transforms
    -> normalised power over 500-1500 Hz (8000 bins), running median of 101
    bins; the realistic search's input.  Rates are for the whole call."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    strain = torch.randn(n_seg * n_fft, generator=g, device="cuda", dtype=torch.float32)
    out = torch.empty((n_seg, n_bins), dtype=torch.float32, device="cuda")
    ctx = ltgw.Context(0)
    try:
        ltgw.ltgw_sft_normalise(ctx.h, strain, n_seg, n_fft, k_lo, n_bins, window, out)  # plans, warm-up
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            ltgw.ltgw_sft_normalise(ctx.h, strain, n_seg, n_fft, k_lo, n_bins, window, out)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
    finally:
        ctx.close()
    wall = min(ts)
    rho = out[:, ::97].double()
    strain_bytes = n_seg * n_fft * 4
    return {"workload": f"{n_seg} segments x {n_fft} samples (8 s at 4096 Hz), band {k_lo}..{k_lo + n_bins - 1} "
                        f"(500-1500 Hz), running median of {window} bins, seed {seed}",
            "ms": wall * 1e3, "segments_per_s": n_seg / wall, "strain_gb_per_s": strain_bytes / wall / 1e9,
            "bound": "lds (the running-median sort and the median selection take about two thirds of the call)",
            "rho_mean": float(rho.mean()), "rho_tail_1.6": float((rho > 1.6).double().mean())}


def batch_leg(torch, ltgw, reps=2, seed=5):
    """The batch of 64 uneven searches (two detectors each, sky patches of 16 to
    1024 points, 1.76e13 template x segment evaluations) in one persistent,
    graph-captured launch: aggregate evals/s, in-band fraction, the persistent
    statistic launch's time and per-search latency.  Every detector's power is
    cut on the device from one seeded pool of Exp(1) values (synth.pool_rows,
    the input the batch parity tests check against the oracle)."""
    import synth

    searches = synth.batch_searches(seed)
    ctx = ltgw.Context(0)
    dev = torch.device("cuda", 0)
    pool = torch.from_numpy(synth.exp_pool(seed)).to(dev)
    specs = []
    slot = 0
    for i, srch in enumerate(searches):
        dets = []
        for q, d in enumerate(srch["dets"]):
            off = torch.from_numpy(synth.pool_offsets(i, q, d["n_seg"], d["n_bins"], seed)).to(dev)
            p = synth.pool_rows(pool, off, d["n_bins"])
            ctx.load_spectrogram(slot, p, d["k_lo"], d["t_sft"], d["t_seg"], store="f32")
            ctx.set_velocity_table(slot, d["v"])
            del p
            dets.append(slot)
            slot += 1
        specs.append(dict(srch["grid"], dets=dets))
    del pool
    torch.cuda.synchronize()
    t = time.perf_counter()
    top_p, top_c, st0 = ctx.eval_batch(specs, k=10)       # tunes the tile shape, captures the graph
    build_s = time.perf_counter() - t
    runs = []
    for _ in range(reps):
        t = time.perf_counter()
        top_p, top_c, st = ctx.eval_batch(specs, k=10)     # replays the graph
        runs.append((time.perf_counter() - t, st))
    wall, st = min(runs, key=lambda x: x[0])
    lat = ctx.batch_latency(len(specs))
    ctx.close()
    evals = st["evals"]
    alg = st["in_band"] * 4 / (st["kernel_ms"] * 1e-3) / 1e9
    return {"workload": f"{len(specs)} searches, T_obs 2-48 h, bands 100-1000 Hz in 500-3000 Hz, 2 detectors each, "
                        f"sky 16-1024 points, seed {seed}",
            "searches": len(specs), "templates": int(st["templates"]), "evals": int(evals),
            "in_band_fraction": st["in_band"] / evals, "value": evals / wall, "unit": "template·segment evals/s",
            "wall_s": wall, "kernel_ms": st["kernel_ms"], "kernel_evals_per_s": evals / (st["kernel_ms"] * 1e-3),
            "graph_ms": st["total_ms"], "graph_replayed": st["graph_replayed"],
            "first_call_s": build_s, "tile_shape": int(st["variant"]),
            "templates_per_lane": int(st["templates_per_lane"]), "segments_per_batch": int(st["segments_per_batch"]),
            "workgroups": int(st["workgroups"]), "tiles": int(st["tiles"]),
            "algorithmic_gbs": alg, "algorithmic_x_hbm_peak": alg / HBM_PEAK_GBS,
            "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_max": float(lat.max())}


def timed_search(torch, ctx, wl, power, t_seg, v, w, store, steps, warmup, tile_shape=-1):
    """Time `steps` steps of the search (after autotuning and `warmup` steps);
    then one more evaluation with outputs for the error report.  Returns a
    dict of figures, the device results (s, c, N) and the top-10 lists."""
    d = wl.dets[0]
    g = wl.grid

    def step():
        ctx.load_spectrogram(0, power, d["k_lo"], d["t_sft"], t_seg, weights=w, store=store)
        ctx.set_velocity_table(0, v)
        ctx.eval_templates(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"],
                           g["t0"], outputs=False)
        tp = ctx.topk("power", 10)
        tc = ctx.topk("count", 10)
        return tp, tc, ctx.diagnostics()

    # the context's autotuner picks the statistic kernel's tile shape for this
    # search on the device (cached for every later step)
    ctx.load_spectrogram(0, power, d["k_lo"], d["t_sft"], t_seg, weights=w, store=store)
    ctx.set_velocity_table(0, v)
    if tile_shape >= 0:
        ctx.set_tile_shape(tile_shape)
    else:
        ctx.set_tile_shape(-1)
        ctx.autotune(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kern_ms = []
    for _ in range(steps):
        tp, tc, dg = step()
        kern_ms.append(dg["eval_kernel_ms"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    s, c, N = ctx.eval_templates(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"], g["t0"])
    res = {"s": s.cpu().numpy(), "c": c.cpu().numpy(), "N": N.cpu().numpy(),
           "top_power": [t["index"] for t in tp], "top_count": [t["index"] for t in tc]}
    launches = max(int(dg["eval_launches"]), 1)
    kms = float(np.mean(kern_ms))
    fig = {"evals": int(dg["evals"]), "in_band": int(dg["in_band"]), "templates": int(dg["templates"]),
           "ms_per_step": elapsed * 1e3 / steps, "value": dg["evals"] * steps / elapsed,
           "eval_kernel_ms": kms, "eval_launches": launches, "eval_launch_ms": kms / launches,
           "tile_shape": int(dg["tile_shape"]), "pow_undecided": int(dg["pow_undecided"]),
           "pow_slow": int(dg["pow_slow"]), "top_power": tp[0], "top_count": tc[0]}
    return fig, res


def roofline(workload, store, fig):
    """The statistic kernel's roofline, per launch (the step's launches
    averaged): HBM-side bytes measured by the committed counter runs (FETCH_SIZE
    and WRITE_SIZE, copy-calibrated) over the average launch duration from HIP
    events, against the 8 TB/s HBM peak; beside it the algorithmic bytes (one
    stored element per in-band evaluation, served mostly by L1/L2, so above the
    HBM peak) and the unit that binds (the vector-memory gather path, TA/TD
    busy fractions from the counters)."""
    launch_s = fig["eval_launch_ms"] * 1e-3
    alg = fig["in_band"] * BYTES[store] / fig["eval_launches"]
    t = traffic_record(workload, store, fig["tile_shape"])
    traffic = None if t is None else t["bytes_per_launch"]
    achieved = None if traffic is None else traffic / launch_s / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": None if achieved is None else achieved / HBM_PEAK_GBS, "traffic": traffic,
           "launch_us": launch_s * 1e6,
           "algorithmic": {"bytes_per_launch": alg, "gbs": alg / launch_s / 1e9,
                           "x_hbm_peak": alg / launch_s / 1e9 / HBM_PEAK_GBS,
                           "unit": "one stored element per in-band template x segment evaluation"}}
    if t is not None and t.get("binding"):
        out["binding"] = t["binding"]
    return out


def traffic_record(workload, store, variant):
    """The committed counter summary of the statistic kernel (HBM-side bytes per
    launch, gather-path busy fractions) when it was taken for this workload,
    store, tile shape and kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "eval_kernel_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if (t.get("source_sha256") != kernel_source_hash() or t.get("workload") != workload
            or t.get("store") != store or t.get("variant") != variant):
        return None
    per_step = (t["fetch_kib_per_step"] * t["fetch_scale"] + t["write_kib_per_step"] * t["write_scale"]) * 1024.0
    t["bytes_per_launch"] = per_step / t["dispatches_per_step"]
    return t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--store", choices=sorted(BYTES), default="f32")
    ap.add_argument("--workload", choices=["realistic", "tiny"], default="realistic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-precision", action="store_true", help="skip the BF16 and FP8 stores of the same search")
    ap.add_argument("--no-proposer", action="store_true", help="skip the learned-proposer leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-search batch leg")
    ap.add_argument("--no-campaign", action="store_true", help="skip the sensitivity campaign leg")
    ap.add_argument("--no-sft", action="store_true", help="skip the data-preparation leg")
    ap.add_argument("--no-antenna", action="store_true", help="skip the antenna-weights leg")
    ap.add_argument("--list-templates", type=int, default=1000000,
                    help="templates of the uniform random bank leg (0 skips it)")
    ap.add_argument("--tile-shape", type=int, default=-1,
                    help="force the statistic kernel's variant (0..15) instead of autotuning (profiling runs)")
    ap.add_argument("--proposer-realisations", type=int, default=50000)
    ap.add_argument("--proposer-epochs", type=int, default=16)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run three 1 GiB device-to-device copies (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); templates shard across "
              "GPUs with no collective on the hot path, so the one-GPU figure is the unit.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": 4 * n, "dispatches": 3}), flush=True)
        return

    import synth
    from paper_2507_07816_amd import ltgw

    wl = synth.realistic() if args.workload == "realistic" else synth.tiny()
    d = wl.dets[0]
    g = wl.grid
    dev = torch.device("cuda", 0)
    print(f"[bench] workload {wl.name}: {wl.n_templates} templates x {d['rho'].shape[0]} segments, "
          f"store {args.store}", file=sys.stderr, flush=True)
    ctx = ltgw.Context(0)
    power = torch.from_numpy(d["rho"]).to(dev)
    # the spectrogram is resident in HBM; the per-segment geometry (times,
    # velocities, weights: 0.3 MB) is host metadata, as in a search
    t_seg = np.ascontiguousarray(d["t_seg"])
    v = np.ascontiguousarray(d["v"])
    w = None if d["weights"] is None else np.ascontiguousarray(d["weights"])
    # injected tracks, added on the device by the library's own injection call
    ctx.load_spectrogram(0, power, d["k_lo"], d["t_sft"], t_seg, weights=w, store="f32")
    ctx.set_velocity_table(0, v)
    for inj in wl.injections:
        ctx.inject_track(0, power, inj["f0"], inj["tau"], inj["brake"], inj["sky"], g["t0"],
                         inj["amp"])
    torch.cuda.synchronize()

    fig, res = timed_search(torch, ctx, wl, power, t_seg, v, w, args.store, args.steps, args.warmup,
                            args.tile_shape)
    results = {args.store: res}
    evals, in_band = fig["evals"], fig["in_band"]
    print(f"[bench] {fig['ms_per_step']:.3f} ms/step, eval kernel {fig['eval_kernel_ms']:.3f} ms, "
          f"in-band {in_band / evals:.4f}, top power {fig['top_power']['index']} psi {fig['top_power']['psi']:.2f}, "
          f"top count {fig['top_count']['index']} psi {fig['top_count']['psi']:.2f}, "
          f"pow undecided {fig['pow_undecided']}", file=sys.stderr, flush=True)
    rl = roofline(wl.name, args.store, fig)
    out = {
        "metric": METRIC, "value": fig["value"], "unit": "template·segment evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": fig["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.store, "data": "synthetic",
        "config": {"workload": wl.name, "store": args.store, "bin_arithmetic": "f64",
                   "templates": fig["templates"], "segments": int(d["rho"].shape[0]),
                   "bins": int(d["rho"].shape[1]), "evals_per_step": evals,
                   "in_band_fraction": in_band / evals, "eval_kernel_ms": fig["eval_kernel_ms"],
                   "eval_launches_per_step": fig["eval_launches"], "eval_launch_ms": fig["eval_launch_ms"],
                   "tile_shape": fig["tile_shape"]},
        "roofline": rl,
    }
    valu = measured_valu(wl.name, args.store, fig["tile_shape"])
    if valu:
        # the VALU bound at the kernel's counted instructions per evaluation
        kernel_rate = evals / (fig["eval_kernel_ms"] * 1e-3)
        ceiling = FP64_LANE_OPS / valu
        out["second_bound"] = {"bound": "valu", "instructions_per_eval": valu, "achieved_evals_per_s": kernel_rate,
                               "peak_evals_per_s": ceiling, "frac": kernel_rate / ceiling}
    if not args.no_precision and args.workload == "realistic":
        # the same search with the power stored in BF16 and in FP8 (per-segment
        # scale): FP32 accumulation, FP64 track and bins
        prec = {}
        for st in ("bf16", "fp8"):
            if st == args.store:
                continue
            print(f"[bench] store {st}", file=sys.stderr, flush=True)
            f2, r2 = timed_search(torch, ctx, wl, power, t_seg, v, w, st, max(args.steps // 2, 1), 1)
            results[st] = r2
            alg = f2["in_band"] * BYTES[st] / f2["eval_launches"]
            prec[st] = {"value": f2["value"], "unit": "template·segment evals/s", "ms_per_step": f2["ms_per_step"],
                        "eval_kernel_ms": f2["eval_kernel_ms"], "eval_launch_ms": f2["eval_launch_ms"],
                        "tile_shape": f2["tile_shape"],
                        "algorithmic_gbs": alg / (f2["eval_launch_ms"] * 1e-3) / 1e9,
                        "bytes_per_in_band_eval": BYTES[st]}
        out["precision"] = prec
    if not args.no_antenna:
        print("[bench] antenna-pattern weights", file=sys.stderr, flush=True)
        out["antenna"] = antenna_leg(torch, ltgw, ctx, wl, power, t_seg, v, w, args.store)
        print(f"[bench] antenna: {json.dumps(out['antenna'])}", file=sys.stderr, flush=True)
    if args.list_templates > 0:
        print("[bench] uniform random bank", file=sys.stderr, flush=True)
        out["random_bank"] = list_leg(torch, ltgw, ctx, wl, n=args.list_templates,
                                      counts=measured_list_counts())
        print(f"[bench] random bank: {json.dumps(out['random_bank'])}", file=sys.stderr, flush=True)
    ctx.close()
    if not args.no_sft:
        print("[bench] data preparation (strain -> normalised power)", file=sys.stderr, flush=True)
        out["sft"] = sft_leg(torch, ltgw)
        print(f"[bench] sft: {json.dumps(out['sft'])}", file=sys.stderr, flush=True)
    if not args.no_campaign:
        print("[bench] sensitivity campaign", file=sys.stderr, flush=True)
        out["campaign"] = campaign_leg(torch, ltgw)
        print(f"[bench] campaign: {json.dumps(out['campaign'])}", file=sys.stderr, flush=True)
    if not args.no_batch:
        print("[bench] batch of 64 searches", file=sys.stderr, flush=True)
        out["batch"] = batch_leg(torch, ltgw)
        print(f"[bench] batch: {json.dumps(out['batch'])}", file=sys.stderr, flush=True)
    if not args.no_proposer:
        print("[bench] learned proposer: training and evaluation", file=sys.stderr, flush=True)
        out["proposer"] = proposer_leg(torch, ltgw, realisations=args.proposer_realisations,
                                       epochs=args.proposer_epochs)
        print(f"[bench] proposer: {json.dumps(out['proposer'])}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline and args.workload == "realistic":
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"], ref = cpu_baseline(wl, power.cpu().numpy(), args.cpu_seconds)
        if len(results) > 1 or "precision" in out:
            out.setdefault("precision", {})["error_vs_fp64"] = precision_report(ref, results)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
