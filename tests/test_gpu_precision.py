"""Precision of the quantised stores (BF16, OCP FP8 E4M3 with per-segment scale).

Against the FP64 oracle over the FP32 data (what a plain FP32 search would
compute), on the tiny workload (1024 segments, 4800 templates, one injection):
- relative error of the power sum s: max and mean (reported, and bounded by
  the format's rounding: <= 2^-9 per element for BF16, <= 2^-4 for E4M3
  relative to the element, plus the FP32 accumulation);
- bin indices: the storage cannot change them, so N and the count c (decided
  on the FP32 input) stay bit-exact;
- top-k agreement with the FP32 search, for both statistics.
The report is printed, and written to $LTGW_REPORT_DIR/precision_report.json when
that variable names a folder.
"""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_util import run_gpu
from test_gpu_parity import tiny_oracle

pytestmark = pytest.mark.gpu

BOUND = {"bf16": 2.0 ** -8, "fp8": 2.0 ** -3}


def test_quantised_store_precision_report():
    det, grid, _ = tiny_oracle()
    ref = oracle.evaluate(det, grid)              # FP64 over the FP32 data
    top_ref_p = list(oracle.topk(oracle.psi_power(ref), 10))
    top_ref_c = list(oracle.topk(oracle.psi_count(ref), 10))
    report = {"workload": "tiny-1024seg-800bin-4800tpl (one injection)"}
    for store in ("f32", "bf16", "fp8"):
        print(f"case: precision, store {store}", flush=True)
        gpu = run_gpu([det], grid, store=store)
        ok = ref["s"] > 0
        rel = np.abs(gpu["s"][ok] - ref["s"][ok]) / ref["s"][ok]
        top_p = [t["index"] for t in gpu["top_power"]]
        top_c = [t["index"] for t in gpu["top_count"]]
        report[store] = {
            "s_rel_err_max": float(rel.max()), "s_rel_err_mean": float(rel.mean()),
            "N_exact": bool(np.array_equal(gpu["N"], ref["N"])),
            "c_exact": bool(np.array_equal(gpu["c"], ref["c"])),
            "top10_power_overlap": len(set(top_p) & set(top_ref_p)),
            "top10_power_same_order": bool(top_p == [int(i) for i in top_ref_p]),
            "top10_count_identical": bool(top_c == [int(i) for i in top_ref_c]),
            "top1_power_is_injection": bool(top_p[0] == int(top_ref_p[0])),
        }
        r = report[store]
        assert r["N_exact"] and r["c_exact"] and r["top10_count_identical"]
        assert r["top1_power_is_injection"]
        if store == "f32":
            assert r["s_rel_err_max"] < 1e-6
        else:
            assert r["s_rel_err_max"] < BOUND[store]
            assert r["top10_power_overlap"] >= 8
    print(json.dumps(report, indent=1), flush=True)
    out = os.environ.get("LTGW_REPORT_DIR", "")
    if out and os.path.isdir(out):
        with open(os.path.join(out, "precision_report.json"), "w") as fh:
            json.dump(report, fh, indent=1)
