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
    refs = [oracle.hard_demap(const_np.points, const_np.labels, y, tx) for y in ys]
    methods = ["valu", "mfma"] if (M >= 32 and D <= 8) else ["valu"]
    for method in methods:
        outs = [_labels_like(N) for _ in s2]
        se, be, nx = dm.hard_decision(c, [_dev(y) for y in ys], _dev(tx.view(np.int16)), outs, method=method,
                                      return_exact=True)
        if method == "valu":
            assert nx == 0
        for i, ref in enumerate(refs):
            got = outs[i].cpu().numpy().view(np.uint16)
            assert np.array_equal(got, ref["labels"]), (method, i, int(np.sum(got != ref["labels"])))
            assert se[i] == ref["sym_err"] and be[i] == ref["bit_err"], (method, i, se[i], be[i], ref)
        print(f"M={M} D={D} {method}: {nx} of {N * len(s2)} symbols decided by the exact path")


def test_dpqpsk():
    _check(W.dp_qpsk(), 65536 + 77, [0, 2, 4, 6, 8, 10], 0)


def test_dp16qam_prefix():
    _check(W.dp_16qam(), 40000 + 13, [0, 6, 12, 20], 1)


def test_gauss8d2048_prefix():
    _check(W.gaussian_constellation(2048, 8, 2), 5003, [0, 5, 10, 15], 2)


def test_padded_dimension_and_chunked_table():
    _check(W.gaussian_constellation(64, 12, 60), 3001, [3, 12], 60, (1,))
    _check(W.gaussian_constellation(4096, 8, 61), 1500, [8], 61, (1,))


def test_mfma_method_routes_ties_to_the_exact_path():
    # 64-QAM with received points exactly on decision boundaries (midpoints between neighbours)
    c = W.qam(64)
    const = dm.Constellation(c.points, c.labels)
    g = W.rng(62, "misc", 0)
    i = g.integers(0, 64, 4096)
    j = g.integers(0, 64, 4096)
    y = (0.5 * (c.points[i].astype(np.float64) + c.points[j].astype(np.float64))).astype(np.float32)
    y[:16] = np.nan
    out = _labels_like(4096)
    tx = _dev(i.astype(np.uint16).view(np.int16))
    se, be, nx = dm.hard_decision(const, [_dev(y)], tx, [out], method="mfma", return_exact=True)
    ref = oracle.hard_demap(c.points, c.labels, y, i.astype(np.uint16))
    assert np.array_equal(out.cpu().numpy().view(np.uint16), ref["labels"])
    assert se[0] == ref["sym_err"] and be[0] == ref["bit_err"]
    assert nx >= int(np.sum(i != j)) // 2  # exact ties cannot be decided by the MFMA ranking
    with pytest.raises(dm.DemapError):
        dm.hard_decision(dm.Constellation(W.dp_qpsk().points, W.dp_qpsk().labels),
                         [_dev(np.zeros((4, 4), np.float32))], None, None, count=False, method="mfma")


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
