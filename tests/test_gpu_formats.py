"""The paper's conventional 2D formats through the same API: 4-, 8-, 16-, 32-, 64- and 128-QAM.

For each format, at SNRs spanning its useful range: LLRs element-wise and GMI / MI within the
FP32 bounds against the FP64 oracle (and the fp16x3 MFMA path where M >= 32), NGMI = GMI / m in
[0, 1], and hard decisions bit-exact against the oracle with their error counts.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2108_07004_amd as dm
import workloads as W
from gpu_helpers import GMI_TOL, LLR_TOL_FP32, DeviceBlock, rel_err

pytestmark = pytest.mark.gpu

FORMATS = [4, 8, 16, 32, 64, 128]
LLR_TOL_FP16X3 = 1e-3


@pytest.mark.parametrize("M", FORMATS)
def test_format_parity(M):
    import torch
    c = W.qam(M)
    m = M.bit_length() - 1
    N = 20000 + 37
    tx = W.tx_indices(M, N, 80, M)
    z = W.unit_noise(N, 2, 80, M)
    snr = np.array([0.0, 8.0, 16.0, 24.0])
    blk = DeviceBlock(c, tx, z, W.sigma2_from_snr_db(snr))
    const = dm.Constellation(c.points, c.labels)
    precs = ["fp32"] + (["fp16x3"] if M >= 32 else [])
    for prec in precs:
        llrs = blk.new_llrs()
        gmi, mi = dm.gmi_estimate(const, blk.sigma2, blk.ys, blk.tx_t, llrs, prec=prec)
        for s, s2 in enumerate(blk.sigma2):
            ref = oracle.demap(c.points, c.labels, s2, blk.y_host(s), tx)
            tol = LLR_TOL_FP32 if prec == "fp32" else LLR_TOL_FP16X3
            assert rel_err(llrs[s].cpu().numpy(), ref["llr"]) <= tol, (M, prec, snr[s])
            assert abs(gmi[s] - ref["gmi"]) <= GMI_TOL and abs(mi[s] - ref["mi_mean"]) <= GMI_TOL, (M, prec, snr[s])
        ngmi = gmi / m
        assert np.all(ngmi >= -1e-3) and np.all(ngmi <= 1.0 + 1e-9)
    labels = [torch.empty(N, dtype=torch.int16, device="cuda:0") for _ in snr]
    se, be = dm.hard_decision(const, blk.ys, blk.tx_t, labels)
    for s in range(len(snr)):
        ref = oracle.hard_demap(c.points, c.labels, blk.y_host(s), tx)
        assert np.array_equal(labels[s].cpu().numpy().view(np.uint16), ref["labels"])
        assert se[s] == ref["sym_err"] and be[s] == ref["bit_err"]
