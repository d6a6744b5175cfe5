"""Pins of the hard-decision oracle (minimum-distance decisions, symbol / bit errors), CPU only.

* DP-QPSK: each bit is an independent binary decision, BER = Q(sqrt(SNR)) exactly; the Monte
  Carlo BER must lie within 4 standard errors.
* DP-16QAM: per-dimension 4-PAM with Gray labels; the exact expected bit errors per symbol
  (and their variance) follow from Gaussian interval probabilities; Monte Carlo within 4 SE.
* Brute force in FP64 on small random constellations agrees with every decision (no near ties).
* Exact ties go to the lowest label; NaN inputs decide the lowest label; row order is irrelevant.
* The library's Q-factor helper inverts BER = erfc(q / sqrt 2) / 2 (host function, no GPU).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

import oracle
import workloads as W


def _qfunc(x):
    return 0.5 * erfc(np.asarray(x, dtype=np.float64) / math.sqrt(2.0))


def test_dpqpsk_ber_closed_form():
    c = W.dp_qpsk()
    N = 1 << 16
    tx = W.tx_indices(16, N, 0)
    z = W.unit_noise(N, 4, 0)
    for snr_db in (0.0, 4.0, 8.0):
        s2 = float(W.sigma2_from_snr_db(snr_db))
        r = oracle.hard_demap(c.points, c.labels, W.awgn(c.points, tx, z, s2), tx)
        p = float(_qfunc(math.sqrt(10 ** (snr_db / 10))))
        ber = r["bit_err"] / (4.0 * N)
        se = math.sqrt(p * (1 - p) / (4.0 * N))
        assert abs(ber - p) <= 4 * se, (snr_db, ber, p)
        ser = r["sym_err"] / N
        p_sym = 1 - (1 - p) ** 4
        assert abs(ser - p_sym) <= 4 * math.sqrt(p_sym * (1 - p_sym) / N), (snr_db, ser, p_sym)


def _pam4_bit_error_moments(sigma):
    """Mean and variance of bit errors per dimension for Gray 4-PAM at levels (2i-3)/sqrt(10)."""
    a = 1.0 / math.sqrt(10.0)
    gray = [0, 1, 3, 2]
    edges = [-math.inf, -2 * a, 0.0, 2 * a, math.inf]
    mean = second = 0.0
    for i in range(4):
        mu = (2 * i - 3) * a
        for j in range(4):
            lo, hi = edges[j], edges[j + 1]
            p = float(_qfunc((lo - mu) / sigma) - _qfunc((hi - mu) / sigma))
            h = bin(gray[i] ^ gray[j]).count("1")
            mean += 0.25 * p * h
            second += 0.25 * p * h * h
    return mean, second - mean * mean


def test_dp16qam_bit_errors_exact_expectation():
    c = W.dp_16qam()
    N = 1 << 15
    tx = W.tx_indices(256, N, 1)
    z = W.unit_noise(N, 4, 1)
    for snr_db in (4.0, 10.0, 14.0):
        s2 = float(W.sigma2_from_snr_db(snr_db))
        r = oracle.hard_demap(c.points, c.labels, W.awgn(c.points, tx, z, s2), tx)
        mean, var = _pam4_bit_error_moments(math.sqrt(s2))
        got = r["bit_err"] / N
        assert abs(got - 4 * mean) <= 4 * math.sqrt(4 * var / N) + 1e-12, (snr_db, got, 4 * mean)


def test_brute_force_fp64_decisions():
    g = W.rng(50, "misc", 0)
    for M, D in ((8, 1), (16, 2), (64, 3), (32, 8)):
        pts = g.standard_normal((M, D)).astype(np.float32)
        lab = g.permutation(M).astype(np.uint16)
        y = (pts[g.integers(0, M, 300)] + 0.7 * g.standard_normal((300, D))).astype(np.float32)
        r = oracle.hard_demap(pts, lab, y)
        d = ((y.astype(np.float64)[:, None, :] - pts.astype(np.float64)[None, :, :]) ** 2).sum(-1)
        srt = np.sort(d, axis=1)
        clear = (srt[:, 1] - srt[:, 0]) > 1e-5 * srt[:, 1]  # no near ties
        assert clear.mean() > 0.95
        want = lab[np.argmin(d, axis=1)]
        assert np.array_equal(r["labels"][clear], want[clear]), (M, D)


def test_ties_nan_and_row_order():
    pts = np.array([[1.0], [-1.0], [3.0], [-3.0]], dtype=np.float32)
    lab = np.array([2, 1, 3, 0], dtype=np.uint16)
    y = np.array([[0.0], [2.0], [-2.0], [np.nan], [0.9]], dtype=np.float32)
    r = oracle.hard_demap(pts, lab, y)
    # y=0: rows 0 and 1 tie (labels 2, 1) -> 1; y=2: rows 0, 2 (labels 2, 3) -> 2;
    # y=-2: rows 1, 3 (labels 1, 0) -> 0; NaN -> lowest label 0; 0.9 -> row 0 (label 2)
    assert r["labels"].tolist() == [1, 2, 0, 0, 2]
    perm = np.array([3, 1, 0, 2])
    r2 = oracle.hard_demap(pts[perm], lab[perm], y)
    assert np.array_equal(r["labels"], r2["labels"])
    tx = np.array([1, 0, 1, 0, 0], dtype=np.uint16)  # sent labels 1, 2, 1, 2, 2
    r3 = oracle.hard_demap(pts, lab, y, tx)
    sent = lab[tx]
    assert r3["sym_err"] == int(np.sum(r["labels"] != sent))
    assert r3["bit_err"] == sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(r["labels"], sent))


def test_q_factor_helper_inverts_the_gaussian_ber():
    import paper_2108_07004_amd as dm
    for q in (0.5, 1.0, 2.0, 3.5, 6.0, 7.5):
        ber = float(0.5 * erfc(q / math.sqrt(2.0)))
        assert abs(dm.q_factor_db(ber) - 20 * math.log10(q)) <= 1e-9, q
    assert math.isnan(dm.q_factor_db(0.0)) and math.isnan(dm.q_factor_db(0.5))
