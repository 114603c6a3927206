"""Synthetic sensitivity campaign (Sec. 3, Figs. 3-4, on synthetic inputs).

The paper measures how far its search reaches: it injects signals at a range
of distances, calls an injection detected when a template close to it has a
critical ratio above the largest one reached on noise alone, fits a sigmoid
to the detection efficiency and quotes the distance at 90% efficiency, for
the power and the number-count statistics and for the cubic and the uniform
random bank.  Here the signal strength is the injected normalised-power
amplitude A (a pixel gains A * w_j along the track); since the power excess
scales as h0^2 and h0 as 1/distance, A ~ 1/d^2 and the 90% point A90 plays
the role of d90.

Every statistic comes from the library's kernels through its C ABI:
- noise realisations: `ltgw_generate_noise` (Philox4x32-10 Exp(1)); each is
  searched in full and its best ratio per statistic kept; the threshold is
  their maximum;
- injected realisations: `ltgw_inject_stack` adds the track; only the
  templates close to the injection decide, so only they are evaluated, and
  the largest ratio among them is compared with the threshold.
Over the lattice, realisations go through in stacks (`ltgw_load_stack`, then
`ltgw_stack_best` for the full searches and `ltgw_stack_psi_list` for the
templates near each injection, power and count); over a random bank, whose
templates share no track tables, one realisation at a time
(`ltgw_eval_list`, `ltgw_topk_candidates` with k = 1, `ltgw_psi`).
The fit is a binomial maximum-likelihood logistic curve in log A (host); its
90% point is reported only where it falls within the sampled amplitudes.
"""
import math

import numpy as np

from . import ltgw
from .proposer import close_region


def lattice_params(grid, idx):
    """(f0, tau, n, sky) rows of lattice templates idx (template order
    ((sky n_brake + i_n) n_tau + i_tau) n_f0 + i_f0)."""
    idx = np.asarray(idx, np.int64)
    n_f0, tau, brake = grid["n_f0"], np.asarray(grid["tau"]), np.asarray(grid["brake"])
    sky = np.asarray(grid["sky"], np.float64).reshape(-1, 3)
    i_f0 = idx % n_f0
    grp = idx // n_f0
    i_tau = grp % len(tau)
    r = grp // len(tau)
    out = np.empty((idx.size, 6))
    out[:, 0] = grid["f0_min"] + i_f0.astype(np.float64) * grid["f0_step"]
    out[:, 1] = tau[i_tau]
    out[:, 2] = brake[r % len(brake)]
    out[:, 3:] = sky[r // len(brake)]
    return out


def random_bank_region(bank, grid, inj, df=2, dg=1):
    """Templates of a random bank close to an injection (f0, tau, n): within df
    lattice f0 steps of it, dg steps of the lattice's tau (in log) and dg steps
    of its n -- the box the lattice's neighbourhood spans, in parameter units."""
    f0, tau, n = inj[:3]
    lt = np.log(np.asarray(grid["tau"], np.float64))
    dlt = (lt[-1] - lt[0]) / max(len(lt) - 1, 1)
    br = np.asarray(grid["brake"], np.float64)
    dn = (br[-1] - br[0]) / max(len(br) - 1, 1)
    ok = ((np.abs(bank[:, 0] - f0) <= df * grid["f0_step"] + 1e-12)
          & (np.abs(np.log(bank[:, 1]) - math.log(tau)) <= dg * dlt + 1e-12)
          & (np.abs(bank[:, 2] - n) <= dg * dn + 1e-12))
    return np.nonzero(ok)[0]


def fit_logistic(amp, k, n, iters=200):
    """Binomial maximum-likelihood fit of eff(A) = 1/(1 + exp(-(ln A - mu)/sigma))
    to k detections out of n at amplitudes amp (Newton's method on the
    log-likelihood in (a, b) with eff = 1/(1 + exp(-(a + b ln A)))).
    Returns dict(mu, sigma, a90 = exp(mu + sigma ln 9), separable, rising);
    a fitted slope that is not positive gives rising = False and a90 = inf."""
    x = np.log(np.asarray(amp, np.float64))
    k = np.asarray(k, np.float64)
    n = np.asarray(n, np.float64)
    # The maximum exists only when the outcomes overlap: some detection at a
    # lower amplitude than some miss.  Otherwise (every miss at or below every
    # detection) the likelihood grows as sigma -> 0; the step is then placed
    # midway in ln A between the largest amplitude with a miss and the
    # smallest with a detection, with sigma = 0.
    miss, hit = x[k < n], x[k > 0]
    if miss.size == 0 or hit.size == 0 or miss.max() <= hit.min():
        lo = miss.max() if miss.size else hit.min()
        hi = hit.min() if hit.size else miss.max()
        mu = 0.5 * (lo + hi)
        return {"mu": mu, "sigma": 0.0, "a90": math.exp(mu), "separable": True, "rising": True}
    def loglik(a, b):
        z = a + b * x
        return float(-np.sum(k * np.logaddexp(0.0, -z) + (n - k) * np.logaddexp(0.0, z)))

    p0 = np.clip((k.sum() + 0.5) / (n.sum() + 1.0), 1e-6, 1 - 1e-6)
    a, b = math.log(p0 / (1 - p0)), 0.0
    ll = loglik(a, b)
    for _ in range(iters):
        z = a + b * x
        p = 1.0 / (1.0 + np.exp(-z))
        wv = n * p * (1.0 - p)
        g = np.array([np.sum(k - n * p), np.sum((k - n * p) * x)])
        H = np.array([[np.sum(wv), np.sum(wv * x)], [np.sum(wv * x), np.sum(wv * x * x)]])
        try:
            step = np.linalg.solve(H, g)
        except np.linalg.LinAlgError:
            break
        # Newton with backtracking: the log-likelihood is concave, so a short
        # enough step along the Newton direction always ascends
        t = 1.0
        while t > 1e-12:
            a2, b2 = a + t * step[0], b + t * step[1]
            ll2 = loglik(a2, b2)
            if ll2 >= ll:
                break
            t *= 0.5
        if t <= 1e-12:
            break
        done = abs(ll2 - ll) <= 1e-15 * max(1.0, abs(ll)) and max(abs(t * step[0]), abs(t * step[1])) < 1e-10
        a, b, ll = a2, b2, ll2
        if done:
            break
    if not b > 0.0:  # efficiency not rising with amplitude: no 90% point
        return {"mu": math.nan, "sigma": math.inf, "a90": math.inf, "separable": False, "rising": False}
    sigma = 1.0 / b
    mu = -a / b
    return {"mu": mu, "sigma": sigma, "a90": math.exp(min(mu + sigma * math.log(9.0), 700.0)),
            "separable": False, "rising": True}


class Campaign:
    """One detector geometry (segment times, velocities, weights, band) and one
    bank: the lattice `grid` (dict of f0_min, f0_step, n_f0, tau, brake, sky,
    t0), or, with `bank` ([n][6] rows), a random bank at the grid's scales."""

    def __init__(self, ctx, geometry, grid, bank=None, seed=2024, store="f32", slot=0, chunk=64, stack_chunk=512):
        import torch

        self.torch = torch
        self.ctx = ctx
        self.geo = geometry
        self.grid = grid
        self.bank = None if bank is None else np.ascontiguousarray(bank, np.float64)
        self.seed = int(seed)
        self.store = store
        self.slot = int(slot)
        self.chunk = int(chunk)
        self.stack_chunk = int(stack_chunk)
        self.n_seg = len(geometry["t_seg"])
        self.n_bins = int(geometry["n_bins"])
        self.sky = np.asarray(grid["sky"], np.float64).reshape(-1, 3)[0]
        self.dev = ctx.device

    def _load(self, power):
        g = self.geo
        self.ctx.load_spectrogram(self.slot, power, g["k_lo"], g["t_sft"], g["t_seg"], weights=g.get("weights"),
                                  store=self.store)
        self.ctx.set_velocity_table(self.slot, g["v"])

    def _stack(self, stream, r0, params):
        """Device stack [R][n_seg][n_bins]: noise realisations r0.. of `stream`
        with injections params[r] = (f0, tau, n, amp) (amp 0: none)."""
        T = self.torch
        R = len(params)
        st = T.empty((R, self.n_seg, self.n_bins), dtype=T.float32, device=self.dev)
        ltgw.ltgw_generate_noise(self.ctx.h, self.seed, stream, r0, st)
        if np.any(np.asarray(params)[:, 3] != 0):
            self._load(st[0])  # the slot's geometry for the injection
            ltgw.ltgw_inject_stack(self.ctx.h, self.slot, st, np.asarray(params, np.float64), self.sky,
                                   float(self.grid.get("t0", 0.0)))
        return st

    def _best_full(self):
        """(power, count) best ratio of the loaded realisation over the bank."""
        g = self.grid
        if self.bank is None:
            self.ctx.eval_templates(g["f0_min"], g["f0_step"], g["n_f0"], g["tau"], g["brake"], g["sky"],
                                    g.get("t0", 0.0), 1 << self.slot, outputs=False)
        else:
            self.ctx.eval_list(self.bank, g.get("t0", 0.0), 1 << self.slot, outputs=False)
        tp, tc = self.ctx.topk("power", 1), self.ctx.topk("count", 1)
        return (tp[0]["psi"] if tp else -math.inf), (tc[0]["psi"] if tc else -math.inf)

    def region(self, inj):
        """Template rows close to an injection (f0, tau, n)."""
        if self.bank is None:
            idx = close_region(self.grid, np.asarray(inj, np.float64)[None, :3])[0]
            return lattice_params(self.grid, idx[idx >= 0])
        return self.bank[random_bank_region(self.bank, self.grid, inj)]

    def _best_region(self, rows):
        if len(rows) == 0:
            return -math.inf, -math.inf
        self.ctx.eval_list(rows, self.grid.get("t0", 0.0), 1 << self.slot, outputs=False)
        m = len(rows)
        pp = self.ctx.psi("power", m).cpu().numpy()
        pc = self.ctx.psi("count", m).cpu().numpy()
        best = lambda a: float(np.nanmax(a)) if np.any(~np.isnan(a)) else -math.inf
        return best(pp), best(pc)

    def _stack_best(self, st):
        """(power[n], count[n]) best ratios of a device stack over the lattice."""
        T = self.torch
        n = st.shape[0]
        self._load(st[0])  # the slot's geometry for the stack
        ltgw.ltgw_load_stack(self.ctx.h, self.slot, st, self.store, coarse=0)
        g, keep = ltgw.make_grid(self.grid["f0_min"], self.grid["f0_step"], self.grid["n_f0"], self.grid["tau"],
                                 self.grid["brake"], self.grid["sky"], self.grid.get("t0", 0.0))
        bi = T.empty(n, dtype=T.int32, device=self.dev)
        out = []
        for stat in ("power", "count"):
            bp = T.empty(n, dtype=T.float64, device=self.dev)
            ltgw.ltgw_stack_best(self.ctx.h, g, bi, bp, stat=stat)
            out.append(bp.cpu().numpy())
        return out[0], out[1]

    def _stack_region(self, st, inj):
        """(power[n], count[n]) largest ratios of each realisation of a device
        stack over the lattice templates close to its injection inj[r]."""
        T = self.torch
        n = st.shape[0]
        self._load(st[0])
        ltgw.ltgw_load_stack(self.ctx.h, self.slot, st, self.store, coarse=0)
        g, keep = ltgw.make_grid(self.grid["f0_min"], self.grid["f0_step"], self.grid["n_f0"], self.grid["tau"],
                                 self.grid["brake"], self.grid["sky"], self.grid.get("t0", 0.0))
        idx = close_region(self.grid, np.asarray(inj, np.float64)[:, :3]).astype(np.int32)  # -1: outside
        idx_d = T.from_numpy(idx).to(self.dev)
        out = []
        for stat in ("power", "count"):
            psi = T.empty(idx.shape, dtype=T.float64, device=self.dev)
            ltgw.ltgw_stack_psi_list(self.ctx.h, g, idx_d, psi, stat=stat)
            p = psi.cpu().numpy()
            ok = ~np.isnan(p)
            out.append(np.where(ok.any(axis=1), np.nanmax(np.where(ok, p, -np.inf), axis=1), -math.inf))
        return out[0], out[1]

    def noise_maxima(self, R, stream=1):
        """Best ratio of each noise-only realisation: arrays (power[R], count[R])."""
        bp, bc = np.empty(R), np.empty(R)
        if self.bank is None:
            for r0 in range(0, R, self.stack_chunk):
                n = min(self.stack_chunk, R - r0)
                bp[r0:r0 + n], bc[r0:r0 + n] = self._stack_best(self._stack(stream, r0, np.zeros((n, 4))))
            return bp, bc
        for r0 in range(0, R, self.chunk):
            n = min(self.chunk, R - r0)
            st = self._stack(stream, r0, np.zeros((n, 4)))
            for i in range(n):
                self._load(st[i])
                bp[r0 + i], bc[r0 + i] = self._best_full()
        return bp, bc

    def injected_maxima(self, inj, stream=2):
        """Largest ratio among the templates close to each injection:
        inj[r] = (f0, tau, n, amp) -> arrays (power[R], count[R])."""
        inj = np.asarray(inj, np.float64)
        R = len(inj)
        bp, bc = np.empty(R), np.empty(R)
        if self.bank is None:
            for r0 in range(0, R, self.stack_chunk):
                n = min(self.stack_chunk, R - r0)
                bp[r0:r0 + n], bc[r0:r0 + n] = self._stack_region(self._stack(stream, r0, inj[r0:r0 + n]),
                                                                  inj[r0:r0 + n])
            return bp, bc
        for r0 in range(0, R, self.chunk):
            n = min(self.chunk, R - r0)
            st = self._stack(stream, r0, inj[r0:r0 + n])
            for i in range(n):
                self._load(st[i])
                bp[r0 + i], bc[r0 + i] = self._best_region(self.region(inj[r0 + i]))
        return bp, bc

    def run(self, amps, per_level, R_noise, f0_range, tau=10000.0, brake=5.0, rng_seed=7):
        """The campaign: thresholds from R_noise realisations, `per_level`
        injections at each amplitude (f0 uniform in f0_range; tau and n fixed,
        as the paper's injections), efficiencies and fits per statistic."""
        noise_p, noise_c = self.noise_maxima(R_noise)
        th = {"power": float(np.max(noise_p)), "count": float(np.max(noise_c))}
        r = np.random.Generator(np.random.PCG64(rng_seed))
        inj = []
        for a in amps:
            for _ in range(per_level):
                inj.append((r.uniform(*f0_range), tau, brake, a))
        inj = np.asarray(inj)
        mp, mc = self.injected_maxima(inj)
        out = {"threshold": th, "noise_max": {"power": noise_p, "count": noise_c},
               "injections": inj, "region_max": {"power": mp, "count": mc}, "amps": list(amps)}
        for name, m in (("power", mp), ("count", mc)):
            det = m > th[name]
            k = det.reshape(len(amps), per_level).sum(axis=1)
            fit = fit_logistic(amps, k, np.full(len(amps), per_level))
            # the 90% point is a result only inside the sampled amplitudes
            inside = fit["rising"] and min(amps) <= fit["a90"] <= max(amps)
            out[name] = {"detected": k, "efficiency": k / per_level, "fit": fit,
                         "a90": fit["a90"] if inside else None, "a90_in_sampled_range": bool(inside)}
        return out
