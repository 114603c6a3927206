"""Helpers shared by the GPU tests: run the HIP path and the oracle on the same inputs."""
import numpy as np

import oracle

REL_TOL = 1e-5  # float-sum form: relative error against the FP64 oracle


def torch_mod():
    import torch

    return torch


def run_gpu(dets, grid, store="f32", k=10, t0=None, det_mask=0, ctx=None):
    """Evaluate on the GPU.  dets: list of oracle.Detector (their FP32 rho and
    weights are what the library loads).  Returns dict of numpy arrays and
    top-k lists."""
    torch = torch_mod()
    from paper_2507_07816_amd import ltgw

    own = ctx is None
    if own:
        ctx = ltgw.Context(0)
    for d, det in enumerate(dets):
        ctx.load_spectrogram(d, torch.from_numpy(det.rho).cuda(), det.k_lo, det.t_sft, det.t_seg,
                             weights=det.w, rho_th=float(det.rho_th), store=store)
        ctx.set_velocity_table(d, det.v)
    s, c, N = ctx.eval_templates(grid.f0_min, grid.f0_step, grid.n_f0, grid.tau, grid.brake,
                                 grid.sky, grid.t0 if t0 is None else t0, det_mask)
    n = grid.n_templates
    out = {"s": s.cpu().numpy().astype(np.float64), "c": c.cpu().numpy(), "N": N.cpu().numpy(),
           "psi_power": ctx.psi("power", n).cpu().numpy(),
           "psi_count": ctx.psi("count", n).cpu().numpy(),
           "top_power": ctx.topk("power", k), "top_count": ctx.topk("count", k),
           "diag": ctx.diagnostics()}
    if own:
        ctx.close()
    return out


def assert_sums_close(gpu_s, ref_s, tol=REL_TOL, what="s"):
    ref_s = np.asarray(ref_s, np.float64)
    err = np.abs(gpu_s - ref_s)
    bound = tol * np.abs(ref_s) + 1e-30
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, (f"{what}: {bad.size} templates beyond rel {tol}; first {bad[:5]} "
                           f"gpu {gpu_s[bad[:5]]} ref {ref_s[bad[:5]]}")
    nz = np.abs(ref_s) > 0
    return float((err[nz] / np.abs(ref_s[nz])).max()) if nz.any() else 0.0


def psi_tolerance(ref, tol=REL_TOL):
    """Largest change of Psi_rho allowed by the float-sum tolerance."""
    with np.errstate(invalid="ignore", divide="ignore"):
        return tol * np.abs(ref["s"]) / np.sqrt(ref["W2"])


def assert_topk_power(top, ref, k):
    """Rank by rank, the GPU's k-th best power template has the oracle's k-th
    best critical ratio up to the float-sum tolerance (near-ties may swap)."""
    psi_o = oracle.psi_power(ref)
    want = oracle.topk(psi_o, k)
    tol = psi_tolerance(ref)
    got = [t["index"] for t in top]
    assert len(got) == len(want)
    assert len(set(got)) == len(got)
    for r, (gi, wi) in enumerate(zip(got, want)):
        slack = 2 * max(tol[gi], tol[wi]) + 1e-12
        assert abs(psi_o[gi] - psi_o[wi]) <= slack, (r, gi, wi, psi_o[gi], psi_o[wi])
    return got, list(want)


def assert_topk_count(top, ref, k):
    want = list(oracle.topk(oracle.psi_count(ref), k))
    got = [t["index"] for t in top]
    assert got == want
    for t in top:
        assert t["stat"] == ref["c"][t["index"]]
        assert t["n_valid"] == ref["N"][t["index"]]
