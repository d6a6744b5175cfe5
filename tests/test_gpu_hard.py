"""Hard-decision demapping on the GPU against the oracle: decided labels bit-exact, error counts equal.

Cases span the three workload constellations (ragged N, several blocks per launch), a padded
dimension (D = 12 -> 16), a table larger than one LDS chunk (M = 4096, D = 8), exact ties and
NaN inputs, the empty block, and a full-size DP-16QAM block checked on a symbol sample plus the
consistency of its counts with its own labels.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2108_07004_amd as dm
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _labels_like(N):
    import torch
    return torch.full((N,), -1, dtype=torch.int16, device=DEV)


def _check(const_np, N, snrs, config, extra=()):
    c = dm.Constellation(const_np.points, const_np.labels)
    M, D = const_np.points.shape
    tx = W.tx_indices(M, N, config, *extra)
    z = W.unit_noise(N, D, config, *extra)
    s2 = W.sigma2_from_snr_db(np.asarray(snrs, dtype=np.float64))
    ys = [W.awgn(const_np.points, tx, z, v) for v in s2]
    outs = [_labels_like(N) for _ in s2]
    se, be = dm.hard_decision(c, [_dev(y) for y in ys], _dev(tx.view(np.int16)), outs)
    for i, y in enumerate(ys):
        ref = oracle.hard_demap(const_np.points, const_np.labels, y, tx)
        got = outs[i].cpu().numpy().view(np.uint16)
        assert np.array_equal(got, ref["labels"]), (i, int(np.sum(got != ref["labels"])))
        assert se[i] == ref["sym_err"] and be[i] == ref["bit_err"], (i, se[i], be[i], ref)


def test_dpqpsk():
    _check(W.dp_qpsk(), 65536 + 77, [0, 2, 4, 6, 8, 10], 0)


def test_dp16qam_prefix():
    _check(W.dp_16qam(), 40000 + 13, [0, 6, 12, 20], 1)


def test_gauss8d2048_prefix():
    _check(W.gaussian_constellation(2048, 8, 2), 5003, [0, 5, 10, 15], 2)


def test_padded_dimension_and_chunked_table():
    _check(W.gaussian_constellation(64, 12, 60), 3001, [3, 12], 60, (1,))
    _check(W.gaussian_constellation(4096, 8, 61), 1500, [8], 61, (1,))


def test_ties_nan_and_empty():
    import torch
    pts = np.array([[1.0], [-1.0], [3.0], [-3.0]], dtype=np.float32)
    lab = np.array([2, 1, 3, 0], dtype=np.uint16)
    c = dm.Constellation(pts, lab)
    y = np.array([[0.0], [2.0], [-2.0], [np.nan], [0.9]], dtype=np.float32)
    out = _labels_like(5)
    se, be = dm.hard_decision(c, [_dev(y)], None, [out], count=False)
    assert se is None and be is None
    assert out.cpu().numpy().tolist() == oracle.hard_demap(pts, lab, y)["labels"].tolist() == [1, 2, 0, 0, 2]
    e = torch.empty((0, 1), dtype=torch.float32, device=DEV)
    se, be = dm.hard_decision(c, [e], torch.empty(0, dtype=torch.int16, device=DEV))
    assert se.tolist() == [0] and be.tolist() == [0]
    with pytest.raises(dm.DemapError):
        dm.hard_decision(c, [_dev(y)], None)  # counting without tx


def test_dp16qam_full_size_sampled():
    w = W.workload("dp16qam")
    tx, z = W.workload_tx_noise(w)
    c = dm.Constellation(w.const.points, w.const.labels)
    tx_t = _dev(tx.view(np.int16))
    z_t = _dev(z)
    ys = [W.awgn_torch(w.const.points, tx_t, z_t, s2) for s2 in w.sigma2[[2, 7]]]
    del z_t
    outs = [_labels_like(w.N) for _ in ys]
    se, be = dm.hard_decision(c, ys, tx_t, outs)
    sent = w.const.labels[tx]
    pick = np.sort(W.rng(1, "misc", 77).choice(w.N, 16384, replace=False))
    for i, y in enumerate(ys):
        got = outs[i].cpu().numpy().view(np.uint16)
        ref = oracle.hard_demap(w.const.points, w.const.labels, y[pick].cpu().numpy())
        assert np.array_equal(got[pick], ref["labels"])
        assert se[i] == int(np.sum(got != sent))
        assert be[i] == int(np.unpackbits((got ^ sent).view(np.uint8)).sum())
