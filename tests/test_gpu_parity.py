"""GPU path vs the FP64 oracle on identical seeded inputs (through the C ABI).

Element-wise LLR parity (|d| / max(1, |ref|) <= 1e-5 for the FP32 path) and GMI / MI
within 1e-4 bit, at sizes the oracle finishes in seconds that span many tiles and a
ragged tail; edge cases (tiny M, odd and padded D, permuted labels, N = 0 and 1,
underflowing far subsets at high SNR); determinism; full-size blocks checked on
sampled symbols and through the FP64 GMI of the GPU's own LLRs.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import paper_2108_07004_amd as dm
import workloads as W
from gpu_helpers import GMI_TOL, LLR_TOL_FP32, DeviceBlock, rel_err

pytestmark = pytest.mark.gpu


def _check_block(w_const, blk, gmi, mi, llrs, tol=LLR_TOL_FP32, gtol=GMI_TOL, label=""):
    for s, s2 in enumerate(blk.sigma2):
        y = blk.y_host(s)
        ref = oracle.demap(w_const.points, w_const.labels, s2, y, blk.tx)
        if llrs is not None:
            e = rel_err(llrs[s].cpu().numpy(), ref["llr"])
            assert e <= tol, f"{label} snr#{s}: LLR rel err {e:.3g}"
        assert abs(gmi[s] - ref["gmi"]) <= gtol, f"{label} snr#{s}: GMI {gmi[s]} vs {ref['gmi']}"
        if mi is not None:
            assert abs(mi[s] - ref["mi_mean"]) <= gtol, f"{label} snr#{s}: MI {mi[s]} vs {ref['mi_mean']}"


def test_awgn_on_device_is_bit_identical_to_host():
    w = W.workload("gauss8d2048", N=5000)
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2[[0, 15]])
    for s, s2 in enumerate(blk.sigma2):
        assert np.array_equal(blk.y_host(s), W.awgn(w.const.points, tx, z, s2))


def test_dpqpsk_full_block_fp32():
    w = W.workload("dpqpsk")
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2)
    c = dm.Constellation(w.const.points, w.const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs)
    _check_block(w.const, blk, gmi, mi, llrs, label="dpqpsk")


def test_dp16qam_prefix_all_snr_fp32():
    w = W.workload("dp16qam", N=(1 << 14) + 123)
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2)
    c = dm.Constellation(w.const.points, w.const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs)
    tot, per = dm.last_fixup_count(len(blk.sigma2))
    assert per[-1] > 0, "20 dB must exercise the far-subset fix-up"
    _check_block(w.const, blk, gmi, mi, llrs, label="dp16qam")


def test_gauss8d_prefix_all_snr_fp32():
    w = W.workload("gauss8d2048", N=2048 + 77)
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2)
    c = dm.Constellation(w.const.points, w.const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs)
    _check_block(w.const, blk, gmi, mi, llrs, label="gauss8d")


@pytest.mark.parametrize("M,D", [(2, 1), (4, 3), (8, 2), (32, 5), (128, 9), (64, 17), (16, 32), (1024, 2)])
def test_shapes_and_permuted_labels(M, D):
    g = W.rng(50, "misc", M, D)
    pts = g.standard_normal((M, D))
    pts *= math.sqrt((D / 2.0) / np.mean(np.sum(pts * pts, axis=1)))
    const = W.Constellation(pts.astype(np.float32), g.permutation(M).astype(np.uint16))
    N = 777
    tx = g.integers(0, M, N).astype(np.uint16)
    z = g.standard_normal((N, D))
    snr = np.array([-3.0, 8.0, 30.0])
    blk = DeviceBlock(const, tx, z, W.sigma2_from_snr_db(snr))
    c = dm.Constellation(const.points, const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs)
    _check_block(const, blk, gmi, mi, llrs, label=f"M{M}D{D}")


def test_empty_and_single_symbol():
    import torch
    w = W.workload("dp16qam", N=1)
    tx, z = W.workload_tx_noise(w)
    c = dm.Constellation(w.const.points, w.const.labels)
    blk = DeviceBlock(w.const, tx, z, w.sigma2[[0, 10]])
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs)
    _check_block(w.const, blk, gmi, mi, llrs, label="N=1")
    e = torch.empty((0, 4), dtype=torch.float32, device="cuda:0")
    gmi0, mi0 = dm.gmi_estimate(c, [0.1], [e], torch.empty(0, dtype=torch.int16, device="cuda:0"))
    assert math.isnan(gmi0[0]) and math.isnan(mi0[0])
    out = dm.demap_llr(c, 0.1, e)
    assert out.shape == (0, 8)


def test_demap_llr_matches_gmi_path_and_gmi_only_mode():
    w = W.workload("dp16qam", N=5000)
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2)
    c = dm.Constellation(w.const.points, w.const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs)
    g2, m2 = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, None)
    assert np.max(np.abs(g2 - gmi)) <= 1e-9 and np.array_equal(m2, mi)
    for s, s2 in enumerate(blk.sigma2):
        l1 = dm.demap_llr(c, s2, blk.ys[s])
        assert np.array_equal(l1.cpu().numpy(), llrs[s].cpu().numpy())


def test_gmi_is_bit_reproducible():
    w = W.workload("gauss8d2048", N=20000)
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2[[3, 9, 15]])
    c = dm.Constellation(w.const.points, w.const.labels)
    a = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, blk.new_llrs())
    b = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, blk.new_llrs())
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rejects_host_pointers_and_bad_sigma():
    import torch
    w = W.workload("dpqpsk", N=16)
    c = dm.Constellation(w.const.points, w.const.labels)
    y = torch.zeros((16, 4), dtype=torch.float32, device="cuda:0")
    with pytest.raises(dm.DemapError):
        dm.demap_llr(c, -1.0, y)
    lib = dm.load_library()
    host = np.zeros((16, 4), np.float32)
    out = torch.empty((16, 4), dtype=torch.float32, device="cuda:0")
    import ctypes
    rc = lib.dm_demap_llr(c.handle, 0.1, host.ctypes.data_as(ctypes.c_void_p), 16,
                          ctypes.c_void_p(out.data_ptr()), 0, None)
    assert rc == -1


def _sampled_full_size(name, snr_idx, prec, tol, n_runs=8, run_len=48):
    """Full-size block in the benchmark's launch configuration; oracle on sampled symbols."""
    w = W.workload(name)
    tx, z = W.workload_tx_noise(w)
    blk = DeviceBlock(w.const, tx, z, w.sigma2)
    c = dm.Constellation(w.const.points, w.const.labels)
    llrs = blk.new_llrs()
    gmi, mi = dm.gmi_estimate(c, blk.sigma2, blk.ys, blk.tx_t, llrs, prec=prec)
    g = W.rng(60, "misc", w.config)
    starts = g.integers(0, w.N - run_len, n_runs)
    idx = np.concatenate([np.arange(s0, s0 + run_len) for s0 in starts])
    for s in snr_idx:
        y = blk.y_host(s, idx)
        assert np.array_equal(y, W.awgn(w.const.points, tx[idx], z[idx], blk.sigma2[s]))
        ref = oracle.demap(w.const.points, w.const.labels, blk.sigma2[s], y, tx[idx])
        got = llrs[s][idx].cpu().numpy()
        e = rel_err(got, ref["llr"])
        assert e <= tol, f"{name} snr#{s}: sampled LLR rel err {e:.3g}"
        # GMI of the GPU's own full-size LLRs, summed in FP64 by the oracle's GMI rule.
        full = llrs[s].cpu().numpy().astype(np.float64)
        g_from_llr = oracle.gmi_from_llr(w.const.m, full, w.const.labels[tx])
        assert abs(g_from_llr - gmi[s]) <= 2e-6, f"{name} snr#{s}: GMI {gmi[s]} vs {g_from_llr}"
        assert np.all(np.isfinite(full))
    return gmi, mi


def test_dp16qam_full_size_sampled():
    _sampled_full_size("dp16qam", [0, 5, 10], "fp32", LLR_TOL_FP32)


@pytest.mark.parametrize("name", ["dp16qam", "128qam"])
def test_row_fixup_with_per_symbol_variance(name):
    # M = 256 and 128 send their underflowed bits to the fix-up's 16-lane rows (four symbols per
    # wavefront); per-symbol variances at 12..26 dB make most symbols' far subsets underflow, and
    # N = 3001 leaves a partial last group of rows.
    import torch
    c = W.dp_16qam() if name == "dp16qam" else W.qam(128)
    const = dm.Constellation(c.points, c.labels)
    N = 3001
    g = W.rng(9, "misc", c.M)
    levels = np.array([12.0, 18.0, 22.0, 26.0])
    pick = g.integers(0, len(levels), N)
    s2 = W.sigma2_from_snr_db(levels)[pick].astype(np.float32)
    tx = g.integers(0, c.M, N).astype(np.uint16)
    z = g.standard_normal((N, c.D))
    y = (c.points.astype(np.float64)[tx] + np.sqrt(s2.astype(np.float64))[:, None] * z).astype(np.float32)
    dev = torch.device("cuda:0")
    got = dm.demap_llr_var(const, torch.from_numpy(s2).to(dev), torch.from_numpy(y).to(dev)).cpu().numpy()
    for k in range(len(levels)):
        idx = np.nonzero(pick == k)[0]
        ref = oracle.demap(c.points, c.labels, float(s2[idx[0]]), y[idx], tx[idx])
        e = rel_err(got[idx], ref["llr"])
        print(f"{name} {levels[k]:.0f} dB: {len(idx)} symbols, LLR rel err {e:.2e}", flush=True)
        assert e <= LLR_TOL_FP32, (name, levels[k], e)
