"""The GPU path against the stored oracle cases (``tests/golden/oracle_cases.json``).

The received blocks and transmitted indices are uploaded exactly as stored, so this comparison
depends on neither the seeded generators nor a live oracle run.  Bounds: FP32 direct-difference
path |d| / max(1, |ref|) <= 1e-5, split-FP16 MFMA path <= 1e-4 (M >= 32), GMI and MI within
1e-4 bit, for the multi-SNR entry point with LLRs and for the single-block LLR entry point.
"""
from __future__ import annotations

import json
from pathlib import Path

import numpy as np
import pytest

import paper_2108_07004_amd as dm
import workloads as W
from gpu_helpers import GMI_TOL, LLR_TOL_FP32, rel_err

pytestmark = pytest.mark.gpu

CASES = json.loads((Path(__file__).resolve().parent / "golden" / "oracle_cases.json").read_text())["cases"]
LLR_TOL = {"fp32": LLR_TOL_FP32, "fp16x3": 1e-4}


def _const(name):
    return {"dpqpsk": W.dp_qpsk, "dp16qam": W.dp_16qam, "8qam": lambda: W.qam(8),
            "128qam": lambda: W.qam(128),
            "gauss8d2048": lambda: W.workload("gauss8d2048", N=1).const}[name]()


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_gpu_matches_the_stored_oracle_case(case):
    import torch
    c = _const(case["name"])
    dev = torch.device("cuda:0")
    const = dm.Constellation(c.points, c.labels)
    tx = np.asarray(case["tx"], dtype=np.uint16)
    tx_t = torch.from_numpy(tx.view(np.int16)).to(dev)
    s2 = [p["sigma2"] for p in case["points"]]
    ys = [torch.tensor(p["y"], dtype=torch.float32, device=dev) for p in case["points"]]
    refs = [np.asarray(p["llr"], dtype=np.float64) for p in case["points"]]
    precs = ["fp32"] + (["fp16x3"] if c.M >= 32 else [])
    for prec in precs:
        llrs = [torch.full((len(tx), c.m), float("nan"), dtype=torch.float32, device=dev) for _ in s2]
        gmi, mi = dm.gmi_estimate(const, s2, ys, tx_t, llrs, prec=prec)
        for s, p in enumerate(case["points"]):
            e = rel_err(llrs[s].cpu().numpy(), refs[s])
            print(f"{case['name']} {prec} sigma2={p['sigma2']:.4g}: llr {e:.2e} "
                  f"gmi {gmi[s] - p['gmi']:+.2e} mi {mi[s] - p['mi']:+.2e}", flush=True)
            assert e <= LLR_TOL[prec], (prec, s, e)
            assert abs(gmi[s] - p["gmi"]) <= GMI_TOL, (prec, s)
            assert abs(mi[s] - p["mi"]) <= GMI_TOL, (prec, s)
        one = dm.demap_llr(const, s2[-1], ys[-1], prec=prec)
        assert rel_err(one.cpu().numpy(), refs[-1]) <= LLR_TOL[prec], prec
    torch.cuda.synchronize()
