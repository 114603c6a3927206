"""Learned proposer for the template bank: training on device-generated
realisations and inference, driven over the ltgw C-ABI.

The method evaluates every template of a cubic lattice bank (Sec. 2); its
detection rule flags a template whose critical ratio (Eq. 4) exceeds the
largest value reached on noise alone (Sec. 3).  The proposer is a system
pattern layered on that rule, not part of the paper: a small convolutional
network reads the coarse critical-ratio map of a realisation (2x2-coarsened
BF16 store, a coarse grid with half the f0 points and fewer (tau, n) groups)
and ranks the fine cells; the n_select best are evaluated exactly on the
fine store, and realisations whose coarse map is loud while no selected cell
passes the threshold fall back to the exhaustive fine search.

Every step runs in the library's kernels: noise (Philox4x32-10), injections,
stores, coarse and fine ratios, labels (the exhaustive search's best cell),
the network's passes, the loss and Adam.  This module only draws injection
parameters on the host, keeps the device buffers and orders the calls.
"""
import math

import numpy as np

from . import ltgw

WIDTH, TAPS = 32, 5


def init_params(c_in, c_out, seed):
    """He-uniform weights, zero biases; flat FP32 in the order W1 b1 W2 b2 W3 b3 W4 b4."""
    r = np.random.Generator(np.random.PCG64(seed))
    shapes = [(WIDTH, c_in, TAPS), (WIDTH,), (WIDTH, WIDTH, TAPS), (WIDTH,), (WIDTH, WIDTH, TAPS), (WIDTH,),
              (c_out, WIDTH, 1), (c_out,)]
    parts = []
    for s in shapes:
        if len(s) == 3:
            lim = math.sqrt(6.0 / (s[1] * s[2]))
            parts.append(r.uniform(-lim, lim, s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def coarse_grid_for(fine, tau, brake):
    """Coarse grid over the fine one: positions l cover fine f0 indices 2l, 2l+1
    (centre f0), with its own (tau, n) lists."""
    return dict(f0_min=fine["f0_min"] + 0.5 * fine["f0_step"], f0_step=2.0 * fine["f0_step"],
                n_f0=fine["n_f0"] // 2, tau=np.asarray(tau, np.float64), brake=np.asarray(brake, np.float64),
                sky=np.asarray(fine["sky"], np.float64).reshape(-1, 3), t0=fine.get("t0", 0.0))


def _grid(d):
    return ltgw.make_grid(d["f0_min"], d["f0_step"], d["n_f0"], d["tau"], d["brake"], d["sky"], d.get("t0", 0.0))


def _n_groups(d):
    return len(d["tau"]) * len(d["brake"]) * len(np.asarray(d["sky"]).reshape(-1, 3))


def close_region(fine, inj, df=2, dg=1):
    """Fine templates close to each injection (rows of inj: f0, tau, n): f0
    index within df of the nearest fine f0, tau and n indices within dg of
    the nearest (tau nearest in log, the lattice being geometric).
    [R][(2 df + 1)(2 dg + 1)^2] template indices (order sky, n, tau, f0
    fastest) in ascending order, -1 outside the grid."""
    n_f0 = int(fine["n_f0"])
    tau, brake = np.asarray(fine["tau"], np.float64), np.asarray(fine["brake"], np.float64)
    inj = np.asarray(inj, np.float64)
    i0 = np.rint((inj[:, 0] - fine["f0_min"]) / fine["f0_step"]).astype(np.int64)
    j0 = np.argmin(np.abs(np.log(inj[:, 1])[:, None] - np.log(tau)[None, :]), axis=1)
    k0 = np.argmin(np.abs(inj[:, 2][:, None] - brake[None, :]), axis=1)
    d_g, d_f = np.arange(-dg, dg + 1), np.arange(-df, df + 1)
    K, J, I = (a.ravel() for a in np.meshgrid(d_g, d_g, d_f, indexing="ij"))
    i, j, k = i0[:, None] + I, j0[:, None] + J, k0[:, None] + K
    ok = (i >= 0) & (i < n_f0) & (j >= 0) & (j < len(tau)) & (k >= 0) & (k < len(brake))
    return np.where(ok, (k * len(tau) + j) * n_f0 + i, -1)


def nearest_coarse_groups(fine, coarse):
    """For each fine (sky, n, tau) group, the coarse groups nearest to it in
    tau (by log) and in n, two at most ([n_fine][2] int32, -1 where there is
    one): the cells the coarse map speaks for when no network ranks them."""
    def nearest(v, grid):
        d = np.abs(grid - v)
        return [int(k) for k in np.nonzero(d <= d.min() * (1 + 1e-12) + 1e-300)[0]]
    ft, fb = np.log(np.asarray(fine["tau"], np.float64)), np.asarray(fine["brake"], np.float64)
    ct, cb = np.log(np.asarray(coarse["tau"], np.float64)), np.asarray(coarse["brake"], np.float64)
    n_sky = len(np.asarray(fine["sky"]).reshape(-1, 3))
    out = []
    for s in range(n_sky):
        for i_n in range(len(fb)):
            for i_t in range(len(ft)):
                cand = [(s * len(cb) + kn) * len(ct) + kt for kn in nearest(fb[i_n], cb) for kt in nearest(ft[i_t], ct)]
                cand = sorted(cand)[:2]
                out.append(cand + [-1] * (2 - len(cand)))
    return np.asarray(out, np.int32)


def evaluated(blocks, fallback, tpl, L, block):
    """Whether fine template tpl[r] (fine n_f0 = 2 L) was among the cells that
    realisation r evaluated exactly: its block (group, f0 index // block) in
    the row's tier lists blocks[r] (-1: unused), or the row fell back.
    tpl may also be [R][m] (several templates per realisation)."""
    nbg = -(-2 * L // block)
    tpl = np.asarray(tpl, np.int64)
    blk = (tpl // (2 * L)) * nbg + (tpl % (2 * L)) // block
    fb = np.asarray(fallback) != 0
    b = np.asarray(blocks)
    if tpl.ndim == 1:
        return fb | (b == blk[:, None]).any(axis=1)
    return fb[:, None] | (b[:, None, :] == blk[:, :, None]).any(axis=2)


class Proposer:
    """Training and inference state on one ltgw.Context whose detector slot
    `det` holds the geometry (segment times, weights, velocities)."""

    def __init__(self, ctx, det, shape, fine, coarse, seed=0, select_frac=0.05, store="f32", block=1,
                 select2_frac=0.0, coarse_segments=2, counts=True):
        import torch

        if fine["n_f0"] % 2:
            raise ValueError("the fine grid needs an even number of f0 points")
        if len(np.asarray(fine["sky"]).reshape(-1, 3)) != 1:
            raise ValueError("the proposer serves directed searches (one sky position)")
        self.torch, self.ctx, self.det = torch, ctx, det
        self.n_seg, self.n_bins = shape
        self.fine, self.coarse = fine, coarse
        self.L = fine["n_f0"] // 2
        # input channels: the coarse power ratio of each coarse group, then
        # (counts) its coarse number-count ratio
        self.counts = bool(counts)
        self.c_in = (2 if self.counts else 1) * _n_groups(coarse)
        self.coarse_map = nearest_coarse_groups(fine, coarse)
        self.c_out = 2 * _n_groups(fine)
        self.n_cells = self.c_out * self.L
        self.n_select = max(1, int(round(select_frac * self.n_cells)))
        self.n_select2 = int(round(select2_frac * self.n_cells))
        self.block = int(block)
        self.coarse_segments = int(coarse_segments)
        self.store = store
        self.seed = seed
        self.rng = np.random.Generator(np.random.PCG64(seed))
        dev = ctx.device
        self.params = torch.from_numpy(init_params(self.c_in, self.c_out, seed)).to(dev)
        n = self.params.numel()
        assert n == ltgw.ltgw_cnn_param_count(self.c_in, self.c_out)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grads = torch.zeros(n, dtype=torch.float32, device=dev)
        self.step = 0
        self._bufs = {}
        self._fg, self._fg_keep = _grid(fine)
        self._cg, self._cg_keep = _grid(coarse)

    # -- device buffers, sized once per batch size --------------------------------
    def _buf(self, R):
        T = self.torch
        if R not in self._bufs:
            dev = self.ctx.device
            f32 = dict(dtype=T.float32, device=dev)
            i32 = dict(dtype=T.int32, device=dev)
            self._bufs = {R: dict(
                stack=T.empty((R, self.n_seg, self.n_bins), **f32),
                x=T.empty((R, self.c_in, self.L), **f32),
                act=T.empty((3, R, WIDTH, self.L), **f32),
                logits=T.empty((R, self.c_out, self.L), **f32),
                dlogits=T.empty((R, self.c_out, self.L), **f32),
                loss=T.empty(R, **f32),
                work=T.empty(ltgw.ltgw_cnn_work_floats(R, self.c_in, self.c_out, self.L), **f32),
                best=T.empty(R, **i32),
                best_psi=T.empty(R, dtype=T.float64, device=dev),
                mask=T.empty(R, **i32),
                target=T.empty(R, **i32))}
        return self._bufs[R]

    def draw_injections(self, R, p_signal, amp_range, rng=None):
        """Host draw of (f0, tau, n, amp) per realisation: f0 uniform over the fine
        band, tau log-uniform and n uniform over the fine grid's ranges."""
        f = self.fine
        f_lo = f["f0_min"]
        f_hi = f["f0_min"] + (f["n_f0"] - 1) * f["f0_step"]
        tau, brake = np.asarray(f["tau"]), np.asarray(f["brake"])
        r = self.rng if rng is None else rng
        sig = r.uniform(size=R) < p_signal
        out = np.zeros((R, 4))
        out[:, 0] = r.uniform(f_lo, f_hi, R)
        out[:, 1] = np.exp(r.uniform(math.log(tau.min()), math.log(tau.max()), R))
        out[:, 2] = r.uniform(brake.min(), brake.max(), R)
        out[:, 3] = np.where(sig, r.uniform(amp_range[0], amp_range[1], R), 0.0)
        return out, sig

    def make_batch(self, R, stream, r0, inj, with_labels=True):
        """Noise + injections -> stack stores -> coarse features (and labels)."""
        b = self._buf(R)
        h = self.ctx.h
        ltgw.ltgw_generate_noise(h, self.seed, stream, r0, b["stack"])
        ltgw.ltgw_inject_stack(h, self.det, b["stack"], inj, np.asarray(self.fine["sky"]).reshape(3),
                               self.fine.get("t0", 0.0))
        ltgw.ltgw_load_stack(h, self.det, b["stack"], self.store, coarse=self.coarse_segments)
        ltgw.ltgw_stack_features(h, self._cg, b["x"], counts=self.counts)
        if with_labels:
            ltgw.ltgw_stack_best(h, self._fg, b["best"], b["best_psi"])
        return b

    def near_best(self, inj):
        """The exact ratio's best template close to each injection (close_region)
        on the loaded fine store: (template[R] int32, psi[R]; -1, -inf if none)."""
        T = self.torch
        region = close_region(self.fine, inj)
        R = region.shape[0]
        out = T.empty(region.shape, dtype=T.float64, device=self.ctx.device)
        ltgw.ltgw_stack_psi_list(self.ctx.h, self._fg, T.from_numpy(region.astype(np.int32)).to(self.ctx.device), out)
        vals = out.cpu().numpy()
        vals = np.where((region >= 0) & np.isfinite(vals), vals, -np.inf)
        k = np.argmax(vals, axis=1)                     # first maximum: the lowest index
        tpl = region[np.arange(R), k].astype(np.int32)
        psi = vals[np.arange(R), k]
        return np.where(np.isfinite(psi), tpl, -1).astype(np.int32), psi

    def train_step(self, R, p_signal=0.9, amp_range=(1.0, 3.0), lr=1e-3, stream=1, inj=None, r0=None,
                   label_psi=None, label="best"):
        """One Adam step on a batch of R realisations (fresh ones unless inj and
        r0 name a stored batch).  The label of an injected realisation is the
        exhaustive search's best cell (label="best") or the best cell close to
        the injection (label="near"), dropped when that ratio is not above
        label_psi.  Returns the batch's mean loss (host float)."""
        T = self.torch
        if inj is None:
            inj, _ = self.draw_injections(R, p_signal, amp_range)
        sig = inj[:, 3] > 0
        b = self.make_batch(R, stream, self.step * R if r0 is None else r0, inj, with_labels=(label == "best"))
        h = self.ctx.h
        b["mask"].copy_(T.from_numpy(sig.astype(np.int32)))
        if label == "near":
            tpl, psi = self.near_best(inj)
            b["best"].copy_(T.from_numpy(tpl))
            b["best_psi"].copy_(T.from_numpy(np.where(np.isfinite(psi), psi, -1e300)))
        elif label != "best":
            raise ValueError(f"label must be 'best' or 'near', not {label!r}")
        ltgw.ltgw_cells_from_templates(h, b["best"], self.L, b["target"], mask=b["mask"],
                                       psi=None if label_psi is None else b["best_psi"],
                                       min_psi=0.0 if label_psi is None else label_psi)
        n_valid = int((b["target"].cpu().numpy() >= 0).sum())
        ltgw.ltgw_cnn_forward(h, self.params, b["x"], self.c_out, b["act"], b["logits"])
        ltgw.ltgw_softmax_xent(h, b["logits"], b["target"], max(n_valid, 1), b["loss"], b["dlogits"])
        ltgw.ltgw_cnn_backward(h, self.params, b["x"], self.c_out, b["act"], b["dlogits"], b["work"], self.grads)
        self.step += 1
        ltgw.ltgw_adam_step(h, self.params, self.grads, self.m, self.v, lr, 0.9, 0.999, 1e-8, self.step)
        return float(b["loss"].cpu().numpy().astype(np.float64).sum()) / max(n_valid, 1)

    def train(self, realisations, batch=256, epochs=1, p_signal=0.9, amp_range=(1.0, 3.0), lr=2e-3,
              label_psi=None, stream=1, label="best"):
        """Several passes over one fixed set of `realisations` realisations
        (Philox stream `stream`, realisation indices 0 .. realisations-1; the
        injection parameters are drawn once), batches in a new order each
        epoch, learning rate on a cosine from lr to lr / 20.  Returns the
        per-step losses."""
        steps_per_epoch = max(1, realisations // batch)
        inj, _ = self.draw_injections(steps_per_epoch * batch, p_signal, amp_range)
        total = steps_per_epoch * epochs
        losses = []
        for e in range(epochs):
            for k in self.rng.permutation(steps_per_epoch):
                t = len(losses) / max(total - 1, 1)
                lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * t)))
                sl = slice(int(k) * batch, (int(k) + 1) * batch)
                losses.append(self.train_step(batch, inj=inj[sl], r0=int(k) * batch, lr=lr_t, stream=stream,
                                              label_psi=label_psi, label=label))
        return losses

    def propose(self, psi_threshold, coarse_threshold, R, return_blocks=False, tier2_threshold=-1e300,
                network=True):
        """ltgw_propose on the loaded stack: (best_index, best_psi, fallback[, blocks]).
        network=False ranks the blocks by the coarse power ratios alone (the
        nearest coarse groups of each fine group), the same budget otherwise."""
        return ltgw.ltgw_propose(self.ctx.h, self._fg, self._cg, self.params if network else None, self.c_in,
                                 self.c_out, self.L, self.n_select, psi_threshold, coarse_threshold, R,
                                 block=self.block, n_select2=self.n_select2, return_blocks=return_blocks,
                                 tier2_threshold=tier2_threshold, coarse_map=None if network else self.coarse_map)

    def save(self, path):
        """Write the network (ltgw_proposer_save)."""
        ltgw.ltgw_proposer_save(self.ctx.h, path, self.params, self.c_in, self.c_out)

    def load(self, path):
        """Replace the network by the one in `path` (ltgw_proposer_load); its
        shape must be this proposer's."""
        c_in, c_out = ltgw.ltgw_proposer_load(self.ctx.h, path)
        if (c_in, c_out) != (self.c_in, self.c_out):
            raise ValueError(f"{path} holds a network of {c_in} -> {c_out} channels, this proposer needs "
                             f"{self.c_in} -> {self.c_out}")
        ltgw.ltgw_proposer_load(self.ctx.h, path, self.params)

    def close_region(self, inj, df=2, dg=1):
        return close_region(self.fine, inj, df, dg)

    def evaluated(self, blocks, fallback, tpl):
        return evaluated(blocks, fallback, tpl, self.L, self.block)

    def exhaustive(self, R):
        """Exhaustive fine search of the loaded stack: host (best_index, best_psi)."""
        b = self._buf(R)
        ltgw.ltgw_stack_best(self.ctx.h, self._fg, b["best"], b["best_psi"])
        return b["best"].cpu().numpy().copy(), b["best_psi"].cpu().numpy().copy()

    def _ingest_ms(self, stack, store, coarse, reps):
        """Device time of the store kernels of ltgw_load_stack (best of reps)."""
        t = []
        for _ in range(reps):
            ltgw.ltgw_load_stack(self.ctx.h, self.det, stack, store, coarse=coarse)
            t.append(ltgw.ltgw_diagnostics(self.ctx.h)["ingest_ms"])
        return min(t)

    def evaluate(self, R_noise=256, R_signal=256, amp_range=(1.0, 3.0), fine_store="bf16", reps=3,
                 coarse_quantiles=(1.0,), target_recall=0.99, tier2_quantile=None, baseline=True,
                 target_speedup=5.0, budgets=None, ingest_reps=7):
        """Recall and speed against the exhaustive search, for the network and
        (baseline) for the ranking by the coarse power ratios alone at the
        same budget (blocks, tiers, thresholds, fallback rule).

        Thresholds: psi_threshold is the largest exhaustive fine ratio over
        R_noise noise-only realisations (the detection rule of Sec. 3); for
        each q in coarse_quantiles the fallback's coarse threshold is the q
        quantile of the largest coarse power ratio of each noise realisation
        (1.0: their maximum; None: no fallback); with tier2_quantile, the second tier is taken
        only above that quantile of the same maxima.  Recall follows the
        detection rule of Sec. 3 with "close to the injection" read as the
        neighbourhood of close_region: an injection is detectable when the
        exhaustive FP32 search has a template of that neighbourhood above
        psi_threshold, and recalled when the proposer evaluated a template of
        that neighbourhood exactly whose ratio (on the `fine_store` store)
        passes the threshold.  recall_same_template is the stricter figure
        that asks for the exhaustive search's own best template of the
        neighbourhood; recall_best the looser one over the realisation's
        overall best; recall_no_fallback is recall with the fallback off.
        Times (HIP events on the context's stream, best of `reps`): the
        exhaustive FP32 search (ltgw_stack_best) and ltgw_propose on the same
        realisations; the two ingests below, best of `ingest_reps` each.  The coarse store is written in the same pass as the
        fine store; what it adds to that pass (ingest of the fine store with
        the coarse one, less the ingest of the fine store alone) is charged
        to the proposer: speedup = exhaustive / (propose + coarse_extra).
        The FP32 store the exhaustive search reads costs more to ingest than
        the BF16 one, which is not credited.  The operating point reported is
        the fastest point whose recall reaches target_recall; failing that,
        the best recall among those at least target_speedup times faster;
        failing that, the fastest.  The points are every quantile at every
        budget (first-tier cell counts; None: this proposer's n_select), and
        their figures are under "points".  The coarse-only ranking is
        measured at the chosen point's budget."""
        T = self.torch
        h = self.ctx.h
        zeros = np.zeros((R_noise, 4))
        b = self.make_batch(R_noise, 2, 0, zeros, with_labels=False)
        _, noise_best = self.exhaustive(R_noise)
        psi_thr = float(np.max(noise_best))
        G = _n_groups(self.coarse)
        coarse_max = b["x"][:, :G].cpu().numpy().reshape(R_noise, -1).max(axis=1)
        # the held-out injections come from their own generator, so the
        # evaluation set does not depend on how long the network was trained
        inj, sig = self.draw_injections(R_signal, 1.0, amp_range,
                                        rng=np.random.Generator(np.random.PCG64(self.seed + 7919)))
        b = self.make_batch(R_signal, 3, 0, inj, with_labels=False)
        ev0, ev1 = T.cuda.Event(enable_timing=True), T.cuda.Event(enable_timing=True)
        ingest = dict(f32=self._ingest_ms(b["stack"], "f32", 0, reps))
        t_ex = []
        for _ in range(reps):
            ev0.record()
            ltgw.ltgw_stack_best(h, self._fg, b["best"], b["best_psi"])
            ev1.record()
            ev1.synchronize()
            t_ex.append(ev0.elapsed_time(ev1))
        ex_idx = b["best"].cpu().numpy().copy()
        ex_psi = b["best_psi"].cpu().numpy().copy()
        # the exhaustive search's best template close to each injection (the
        # listed evaluation gives the exhaustive kernel's sums, bit for bit)
        near_tpl, near_psi = self.near_best(inj)
        # the two ingests alternate (best of ingest_reps each), so that drift
        # in the device's clock or load affects both alike; the coarse one
        # runs last and leaves the stores loaded
        t_f, t_c = [], []
        for _ in range(max(1, ingest_reps)):
            t_f.append(self._ingest_ms(b["stack"], fine_store, 0, 1))
            t_c.append(self._ingest_ms(b["stack"], fine_store, self.coarse_segments, 1))
        ingest[fine_store] = min(t_f)
        ingest[fine_store + "+coarse"] = min(t_c)
        coarse_extra = max(0.0, ingest[fine_store + "+coarse"] - ingest[fine_store])
        near_prop = T.empty((R_signal, 1), dtype=T.float64, device=self.ctx.device)
        ltgw.ltgw_stack_psi_list(h, self._fg, T.from_numpy(np.maximum(near_tpl, 0).reshape(-1, 1)).to(self.ctx.device),
                                 near_prop)
        near_prop = np.where(near_tpl >= 0, near_prop.cpu().numpy().ravel(), -np.inf)
        # every template of each injection's neighbourhood on the proposer's store
        region = self.close_region(inj)
        reg_prop = T.empty(region.shape, dtype=T.float64, device=self.ctx.device)
        ltgw.ltgw_stack_psi_list(h, self._fg, T.from_numpy(region.astype(np.int32)).to(self.ctx.device), reg_prop)
        reg_prop = np.where(region >= 0, reg_prop.cpu().numpy(), -np.inf)
        reg_prop = np.where(np.isnan(reg_prop), -np.inf, reg_prop)
        det_near = near_psi > psi_thr
        n_near = int(det_near.sum())
        det_ex = ex_psi > psi_thr
        n_det = int(det_ex.sum())
        frac = lambda hit, of, n: float((of & hit).sum() / n) if n else float("nan")

        def recalls(pp, fb, blocks):
            same = self.evaluated(blocks, fb, near_tpl) & (near_prop > psi_thr)
            ev = self.evaluated(blocks, fb, np.maximum(region, 0)) & (region >= 0)
            hit = (ev & (reg_prop > psi_thr)).any(axis=1)
            return frac(hit, det_near, n_near), frac(pp > psi_thr, det_ex, n_det), frac(same, det_near, n_near)

        t2 = -1e300 if tier2_quantile is None else float(np.quantile(coarse_max, tier2_quantile))

        def budget_points(network, points):
            for q in coarse_quantiles:
                # q None: no fallback
                coarse_thr = 1e300 if q is None else float(np.quantile(coarse_max, q))
                t_pr = []
                for _ in range(reps):
                    ev0.record()
                    self.propose(psi_thr, coarse_thr, R_signal, tier2_threshold=t2, network=network)
                    ev1.record()
                    ev1.synchronize()
                    t_pr.append(ev0.elapsed_time(ev1))
                pi, pp, fb, bl = self.propose(psi_thr, coarse_thr, R_signal, return_blocks=True,
                                              tier2_threshold=t2, network=network)
                rec, rec_best, rec_same = recalls(pp, fb, bl)
                points.append(dict(n_select=self.n_select, coarse_quantile=q, coarse_threshold=coarse_thr,
                                   recall=rec, recall_best=rec_best, recall_same_template=rec_same,
                                   fallback_frac=float(fb.mean()), propose_ms=min(t_pr),
                                   speedup=min(t_ex) / (min(t_pr) + coarse_extra),
                                   speedup_search_only=min(t_ex) / min(t_pr),
                                   same_template=float((pi[det_ex] == ex_idx[det_ex]).mean()) if n_det
                                   else float("nan")))

        def operating_points(network, budgets):
            own = self.n_select
            points = []
            try:
                for n_sel in budgets:
                    self.n_select = own if n_sel is None else int(n_sel)
                    budget_points(network, points)
            finally:
                self.n_select = own
            ok = [p for p in points if p["recall"] >= target_recall]
            fast = [p for p in points if p["speedup"] >= target_speedup]
            if ok:
                best = max(ok, key=lambda p: p["speedup"])
            elif fast:
                best = max(fast, key=lambda p: (p["recall"], p["speedup"]))
            else:
                best = max(points, key=lambda p: p["speedup"])
            # the chosen budget with the fallback never taken
            self.n_select, keep = best["n_select"], self.n_select
            try:
                _, pp_nf, fb_nf, bl_nf = self.propose(psi_thr, 1e300, R_signal, return_blocks=True,
                                                      tier2_threshold=t2, network=network)
            finally:
                self.n_select = keep
            rec_nf, rec_best_nf, rec_same_nf = recalls(pp_nf, fb_nf, bl_nf)
            out = dict(best)
            out.update(recall_no_fallback=rec_nf, recall_best_no_fallback=rec_best_nf,
                       recall_same_template_no_fallback=rec_same_nf, points=points)
            return out

        amp = inj[:, 3]
        out = operating_points(True, budgets if budgets else (None,))
        out.update(detectable=n_near, detectable_best=n_det, realisations=R_signal,
                   detectable_min_amp=float(amp[det_near].min()) if n_near else float("nan"),
                   psi_threshold=psi_thr, tier2_quantile=tier2_quantile, tier2_threshold=t2,
                   exhaustive_ms=min(t_ex), ingest_ms=ingest, coarse_extra_ms=coarse_extra,
                   n_select2=self.n_select2, block=self.block,
                   coarse_segments=self.coarse_segments, input_channels=self.c_in, counts=self.counts,
                   n_cells=self.n_cells, fine_store=fine_store, target_recall=target_recall)
        if baseline:
            out["coarse_only"] = operating_points(False, (out["n_select"],))
        return out
