"""The allocation-free GMI entry point (dm_gmi_estimate_noalloc) against dm_gmi_estimate.

Two calls in a row on one GPU share its static scratch array: the first on DP-16QAM with many
fix-up entries at high SNR, the second with a smaller block and fewer noise levels (the first
call's accumulators and queue counter must not leak into it), then a third on the 8D M = 2048
constellation in another precision.  Each is compared with the allocating entry point on the
same inputs: LLRs bit-identical, GMI and MI equal (the same kernels and fixed-point sums), and
the second call also against the FP64 oracle.  Host-side rejections need no GPU work.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2108_07004_amd as dm
import workloads as W
from gpu_helpers import GMI_TOL, LLR_TOL_FP32, DeviceBlock, rel_err

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _both(const, blk, prec):
    import torch
    l_a, l_b = blk.new_llrs(), blk.new_llrs()
    g_a, m_a = dm.gmi_estimate_noalloc(const, blk.sigma2, blk.ys, blk.tx_t, l_a, prec=prec)
    g_b, m_b = dm.gmi_estimate(const, blk.sigma2, blk.ys, blk.tx_t, l_b, prec=prec)
    torch.cuda.synchronize()
    for s in range(len(blk.sigma2)):
        assert torch.equal(l_a[s], l_b[s]), s
    assert np.array_equal(g_a, g_b), (g_a, g_b)
    assert np.array_equal(m_a, m_b), (m_a, m_b)
    return g_a, m_a, l_a


def test_noalloc_matches_allocating_entry_point_on_consecutive_calls():
    q = W.dp_16qam()
    cq = dm.Constellation(q.points, q.labels)
    _say("call 1: DP-16QAM N=60000 x 4 SNR (4, 12, 18, 20 dB), fp16x3")
    tx = W.tx_indices(q.M, 60000, 71, 0)
    z = W.unit_noise(60000, q.D, 71, 0)
    blk = DeviceBlock(q, tx, z, W.sigma2_from_snr_db(np.array([4.0, 12.0, 18.0, 20.0])))
    g1, m1, _ = _both(cq, blk, "fp16x3")
    _say(f"call 1 GMI {g1}")

    _say("call 2: DP-16QAM N=9001 x 2 SNR (20, 6 dB), fp32, smaller than call 1")
    tx2 = W.tx_indices(q.M, 9001, 71, 1)
    z2 = W.unit_noise(9001, q.D, 71, 1)
    blk2 = DeviceBlock(q, tx2, z2, W.sigma2_from_snr_db(np.array([20.0, 6.0])))
    g2, m2, l2 = _both(cq, blk2, "fp32")
    for s, v in enumerate(blk2.sigma2):
        ref = oracle.demap(q.points, q.labels, v, blk2.y_host(s), tx2)
        assert rel_err(l2[s].cpu().numpy(), ref["llr"]) <= LLR_TOL_FP32, s
        assert abs(g2[s] - ref["gmi"]) <= GMI_TOL and abs(m2[s] - ref["mi_mean"]) <= GMI_TOL, (s, g2[s], ref["gmi"])
    _say(f"call 2 GMI {g2}")

    _say("call 3: 8D M=2048 N=5000 x 3 SNR, fp16x3")
    c = W.gaussian_constellation(2048, 8, 2)
    cc = dm.Constellation(c.points, c.labels)
    tx3 = W.tx_indices(c.M, 5000, 71, 2)
    z3 = W.unit_noise(5000, c.D, 71, 2)
    blk3 = DeviceBlock(c, tx3, z3, W.sigma2_from_snr_db(np.array([0.0, 8.0, 15.0])))
    g3, _, _ = _both(cc, blk3, "fp16x3")
    _say(f"call 3 GMI {g3}")


def test_noalloc_rejects_too_many_noise_levels_and_handles_empty_blocks():
    import torch
    q = W.dp_qpsk()
    cq = dm.Constellation(q.points, q.labels)
    N = 64
    tx = torch.zeros(N, dtype=torch.int16, device="cuda:0")
    ys = [torch.zeros((N, q.D), dtype=torch.float32, device="cuda:0") for _ in range(33)]
    with pytest.raises(dm.DemapError, match="33 exceeds"):
        dm.gmi_estimate_noalloc(cq, np.full(33, 0.1), ys, tx)
    e = torch.empty((0, q.D), dtype=torch.float32, device="cuda:0")
    g, m = dm.gmi_estimate_noalloc(cq, [0.1, 0.2], [e, e], torch.empty(0, dtype=torch.int16, device="cuda:0"))
    assert np.all(np.isnan(g)) and np.all(np.isnan(m))


def test_noalloc_queue_overflow_recomputes_in_place():
    """DP-16QAM at 20 dB flags a far subset for most symbols: 2^21 symbols overflow the static
    fix-up queue (2^20 entries), so the demapping kernel recomputes the rest in place.  LLRs and
    GMI / MI agree with the allocating entry point (whose queue holds them all) and sampled LLRs
    with the oracle.  FP32 operands: that kernel queues every flagged bit (the MFMA kernel for
    these constellations resolves far subsets itself and queues few)."""
    import torch
    q = W.dp_16qam()
    cq = dm.Constellation(q.points, q.labels)
    N = 1 << 21
    _say(f"DP-16QAM N={N} at 20 dB, fp32: fix-up queue overflow")
    tx = W.tx_indices(q.M, N, 71, 3)
    z = W.unit_noise(N, q.D, 71, 3)
    blk = DeviceBlock(q, tx, z, W.sigma2_from_snr_db(np.array([20.0])))
    l_a, l_b = blk.new_llrs(), blk.new_llrs()
    g_a, m_a = dm.gmi_estimate_noalloc(cq, blk.sigma2, blk.ys, blk.tx_t, l_a, prec="fp32")
    g_b, m_b = dm.gmi_estimate(cq, blk.sigma2, blk.ys, blk.tx_t, l_b, prec="fp32")
    n_fix, _ = dm.last_fixup_count(1)
    torch.cuda.synchronize()
    _say(f"GMI {g_a[0]:.9f} / {g_b[0]:.9f}, MI {m_a[0]:.9f} / {m_b[0]:.9f}, fix-up pairs {n_fix}")
    # a symbol is queued when any of its four PAM coordinates was sent on an outer level (the far
    # subset of that coordinate's first label bit then lies two spacings away): 15/16 of the
    # symbols, about 1.97M queue entries for 2^20 places; the pair count checks the flags occurred
    assert n_fix > (1 << 21), n_fix
    a, b = l_a[0].cpu().numpy(), l_b[0].cpu().numpy()
    assert np.all(np.isfinite(a))
    assert rel_err(a, b.astype(np.float64)) <= 1e-4
    assert abs(g_a[0] - g_b[0]) <= 1e-6 and abs(m_a[0] - m_b[0]) <= 1e-6
    idx = np.unique(W.rng(71, "misc", 4).integers(0, N, 2048))
    ref = oracle.demap(q.points, q.labels, blk.sigma2[0], blk.y_host(0, idx), tx[idx])
    assert rel_err(a[idx], ref["llr"]) <= 1e-4
