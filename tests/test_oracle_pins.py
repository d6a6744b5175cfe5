"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

The paper prints no soft-demapping values (its GMI use is qualitative, Sec. 5), so
every pin here is mathematical:
* closed-form LLRs of factorising constellations (DP-QPSK, product 4-PAM, M=2);
* Gauss-Hermite GMI/MI of DP-QPSK and DP-16QAM, itself cross-checked by adaptive
  quadrature, hit by the Monte-Carlo oracle within 4 standard errors;
* information-theoretic invariants and the low/high SNR limits;
* metamorphic relations (label complement, bit permutation, row permutation,
  translation, scaling);
* a 50-digit brute force from the definition on tiny constellations.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W
from closed_forms import bpsk_bit_gmi_formula, pam_gmi_mi_gh, pam_gmi_mi_quad, product_se


def _run(c, snr_db, N, config=0, extra=0, llr=True):
    s2 = float(W.sigma2_from_snr_db(snr_db))
    tx = W.tx_indices(c.M, N, config, extra)
    z = W.unit_noise(N, c.D, config, extra)
    y = W.awgn(c.points, tx, z, s2)
    return s2, tx, y, oracle.demap(c.points, c.labels, s2, y, tx, llr=llr)


def _rel_err(a, b):
    return np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b)))


# ---------------------------------------------------------------------------- closed-form LLRs

@pytest.mark.parametrize("snr", [0.0, 6.0, 10.0])
def test_dpqpsk_llr_closed_form(snr):
    c = W.dp_qpsk()
    s2, tx, y, r = _run(c, snr, 4096)
    A = float(np.max(c.points))  # the FP32-rounded amplitude the oracle receives
    assert np.all(np.abs(c.points) == np.float32(A))
    ref = 2.0 * A * y.astype(np.float64) / s2  # LLR index k <-> dimension k (MSB first)
    assert _rel_err(r["llr"], ref) < 1e-12


@pytest.mark.parametrize("snr", [0.0, 10.0, 20.0])
def test_dp16qam_llr_is_1d_pam_llr(snr):
    c = W.dp_16qam()
    s2, tx, y, r = _run(c, snr, 2048)
    amps = np.unique(c.points[:, 0]).astype(np.float64)  # the FP32-rounded 4-PAM levels, ascending
    assert amps.shape == (4,) and np.allclose(amps, np.array([-3, -1, 1, 3]) / math.sqrt(10.0), rtol=1e-7)
    # BRGC 00,01,11,10 on ascending amplitudes: first bit set for {+1,+3}, second for {-1,+1}
    sets = {0: ([2, 3], [0, 1]), 1: ([1, 2], [0, 3])}
    ref = np.empty_like(r["llr"])
    for d in range(4):
        v = -(y[:, d:d + 1].astype(np.float64) - amps[None, :]) ** 2 / (2 * s2)
        for q in range(2):
            one, zero = sets[q]
            ref[:, 2 * d + q] = np.logaddexp(v[:, one[0]], v[:, one[1]]) - np.logaddexp(v[:, zero[0]], v[:, zero[1]])
    assert _rel_err(r["llr"], ref) < 1e-12


def test_two_point_llr_closed_form():
    g = W.rng(99, "misc", 1)
    pts = g.standard_normal((2, 3)).astype(np.float32)
    lab = np.array([1, 0], dtype=np.uint16)  # row 1 carries label 0
    y = (g.standard_normal((500, 3)) * 0.7).astype(np.float32)
    tx = g.integers(0, 2, 500).astype(np.uint16)
    s2 = 0.3
    r = oracle.demap(pts, lab, s2, y, tx)
    y64, p64 = y.astype(np.float64), pts.astype(np.float64)
    d_lab0 = np.sum((y64 - p64[1]) ** 2, axis=1)
    d_lab1 = np.sum((y64 - p64[0]) ** 2, axis=1)
    ref = (d_lab0 - d_lab1) / (2 * s2)
    assert _rel_err(r["llr"][:, 0], ref) < 1e-12


# ---------------------------------------------------------------------------- quadrature pins

@pytest.mark.parametrize("levels", [2, 4])
def test_two_quadratures_agree(levels):
    for snr in (0.0, 8.0, 16.0, 20.0):
        s2 = float(W.sigma2_from_snr_db(snr))
        a = pam_gmi_mi_gh(levels, s2)
        b = pam_gmi_mi_quad(levels, s2)
        assert abs(a[0] - b[0]) < 5e-8 and abs(a[1] - b[1]) < 5e-8


def test_bpsk_formula_matches_pam2():
    for snr in (0.0, 4.0, 10.0):
        s2 = float(W.sigma2_from_snr_db(snr))
        assert abs(bpsk_bit_gmi_formula(10 ** (snr / 10)) - pam_gmi_mi_gh(2, s2)[0]) < 1e-12


def test_dpqpsk_gmi_matches_gauss_hermite():
    w = W.workload("dpqpsk")
    tx, z = W.workload_tx_noise(w)
    for snr, s2 in zip(w.snr_db, w.sigma2):
        y = W.awgn(w.const.points, tx, z, s2)
        r = oracle.demap(w.const.points, w.const.labels, s2, y, tx, llr=False)
        G, MI = (4 * v for v in pam_gmi_mi_gh(2, float(s2)))
        # true standard errors from the quadrature's second moments: at high SNR the
        # sample deviation misses the rare wrong-decision events that set the mean
        se_g, se_m = product_se(2, 4, float(s2), w.N)
        assert abs(r["gmi"] - G) <= 4 * se_g + 1e-12, (snr, r["gmi"], G, se_g)
        assert abs(r["mi_mean"] - MI) <= 4 * se_m + 1e-12, (snr, r["mi_mean"], MI, se_m)


def test_dp16qam_gmi_matches_gauss_hermite():
    w = W.workload("dp16qam", N=1 << 15)
    tx, z = W.workload_tx_noise(w)
    for snr, s2 in zip(w.snr_db, w.sigma2):
        y = W.awgn(w.const.points, tx, z, s2)
        r = oracle.demap(w.const.points, w.const.labels, s2, y, tx, llr=False)
        G, MI = (4 * v for v in pam_gmi_mi_gh(4, float(s2)))
        # true standard errors from the quadrature's second moments: at high SNR the
        # sample deviation misses the rare wrong-decision events that set the mean
        se_g, se_m = product_se(4, 4, float(s2), w.N)
        assert abs(r["gmi"] - G) <= 4 * se_g + 1e-9, (snr, r["gmi"], G, se_g)
        assert abs(r["mi_mean"] - MI) <= 4 * se_m + 1e-9, (snr, r["mi_mean"], MI, se_m)


# ---------------------------------------------------------------------------- invariants

@pytest.mark.parametrize("snr", [0.0, 7.0, 15.0])
def test_gmi_le_mi_le_log2m(snr):
    c = W.gaussian_constellation(2048, 8, 2)
    s2, tx, y, r = _run(c, snr, 1024, config=2, llr=False)
    se = max(np.std(r["g"]), np.std(r["mi"])) / math.sqrt(1024)
    assert np.all(r["mi"] <= c.m + 1e-12)  # per symbol: the tx term alone makes the sum >= 1
    assert np.all(r["g"] <= c.m + 1e-12)   # each bit term is at most 1
    assert -4 * se <= r["gmi"] <= r["mi_mean"] + 4 * se
    assert r["mi_mean"] <= c.m


def test_snr_limits():
    for c in (W.dp_qpsk(), W.dp_16qam(), W.gaussian_constellation(64, 4, 3)):
        _, _, _, lo = _run(c, -30.0, 4096, llr=False)
        assert abs(lo["gmi"]) <= 0.01 and abs(lo["mi_mean"]) <= 0.01
    for c in (W.dp_qpsk(), W.dp_16qam()):
        _, _, _, hi = _run(c, 40.0, 4096, llr=False)
        assert hi["gmi"] >= c.m - 1e-6 and hi["mi_mean"] >= c.m - 1e-6


# ---------------------------------------------------------------------------- metamorphic relations

def _gauss_case(M=32, D=3, N=600, seed=5, grid=None):
    g = W.rng(98, "misc", seed)
    pts = g.standard_normal((M, D))
    lab = g.permutation(M).astype(np.uint16)
    tx = g.integers(0, M, N).astype(np.uint16)
    y = pts[tx] + 0.5 * g.standard_normal((N, D))
    if grid:
        pts, y = np.round(pts * grid) / grid, np.round(y * grid) / grid
    return pts.astype(np.float32), lab, y.astype(np.float32), tx


def test_label_bit_complement_negates_llr():
    pts, lab, y, tx = _gauss_case()
    m = 5
    base = oracle.demap(pts, lab, 0.4, y, tx)
    for k in range(m):
        r = oracle.demap(pts, lab ^ np.uint16(1 << (m - 1 - k)), 0.4, y, tx)
        expect = base["llr"].copy()
        expect[:, k] *= -1
        assert _rel_err(r["llr"], expect) < 1e-12
        assert abs(r["gmi"] - base["gmi"]) < 1e-12


def test_label_bit_permutation_permutes_llr():
    pts, lab, y, tx = _gauss_case()
    m = 5
    perm = [3, 0, 4, 1, 2]  # new bit k takes old bit perm[k] (MSB-first indices)
    new = np.zeros_like(lab)
    for k in range(m):
        new |= (((lab >> (m - 1 - perm[k])) & 1) << (m - 1 - k)).astype(np.uint16)
    base = oracle.demap(pts, lab, 0.4, y, tx)
    r = oracle.demap(pts, new, 0.4, y, tx)
    assert _rel_err(r["llr"], base["llr"][:, perm]) < 1e-12
    assert abs(r["gmi"] - base["gmi"]) < 1e-12


def test_row_permutation_is_invisible():
    pts, lab, y, tx = _gauss_case()
    g = W.rng(98, "misc", 77)
    p = g.permutation(pts.shape[0])
    inv = np.argsort(p)
    base = oracle.demap(pts, lab, 0.4, y, tx)
    r = oracle.demap(pts[p], lab[p], 0.4, y, inv[tx].astype(np.uint16))
    assert _rel_err(r["llr"], base["llr"]) < 1e-12
    assert abs(r["gmi"] - base["gmi"]) < 1e-12 and abs(r["mi_mean"] - base["mi_mean"]) < 1e-12


def test_translation_and_scaling():
    pts, lab, y, tx = _gauss_case(grid=1024)
    base = oracle.demap(pts, lab, 0.4, y, tx)
    v = np.array([0.25, -1.5, 3.0], dtype=np.float32)  # dyadic grid: sums stay exact in FP32
    r = oracle.demap(pts + v, lab, 0.4, y + v, tx)
    assert _rel_err(r["llr"], base["llr"]) < 1e-11
    assert abs(r["gmi"] - base["gmi"]) < 1e-11
    r = oracle.demap(pts * 2, lab, 1.6, y * 2, tx)
    assert _rel_err(r["llr"], base["llr"]) < 1e-12
    assert abs(r["mi_mean"] - base["mi_mean"]) < 1e-12


def test_gmi_from_llr_agrees():
    pts, lab, y, tx = _gauss_case()
    r = oracle.demap(pts, lab, 0.4, y, tx)
    assert abs(oracle.gmi_from_llr(5, r["llr"], lab[tx]) - r["gmi"]) < 1e-13


# ---------------------------------------------------------------------------- brute force

def _brute(pts, lab, s2, y, tx):
    mpmath.mp.dps = 50
    M, D = pts.shape
    m = int(M).bit_length() - 1
    P = [[mpmath.mpf(float(v)) for v in row] for row in pts]
    L = np.empty((len(y), m))
    g = np.empty(len(y))
    mi = np.empty(len(y))
    ln2 = mpmath.log(2)
    for n, yn in enumerate(y):
        Y = [mpmath.mpf(float(v)) for v in yn]
        e = [mpmath.exp(-sum((Y[d] - P[j][d]) ** 2 for d in range(D)) / (2 * mpmath.mpf(s2))) for j in range(M)]
        gn = mpmath.mpf(0)
        b_tx = int(lab[tx[n]])
        for k in range(m):
            sel = lambda j, b: ((int(lab[j]) >> (m - 1 - k)) & 1) == b
            lam = mpmath.log(sum(e[j] for j in range(M) if sel(j, 1))) - mpmath.log(sum(e[j] for j in range(M) if sel(j, 0)))
            L[n, k] = float(lam)
            s = lam if ((b_tx >> (m - 1 - k)) & 1) == 0 else -lam
            gn += 1 - mpmath.log(1 + mpmath.exp(s)) / ln2
        g[n] = float(gn)
        mi[n] = float(m - mpmath.log(sum(e) / e[tx[n]]) / ln2)
    return L, g, mi


@pytest.mark.parametrize("M,D", [(2, 1), (4, 1), (4, 2), (8, 2)])
def test_brute_force_tiny(M, D):
    g = W.rng(97, "misc", M * 10 + D)
    pts = g.standard_normal((M, D)).astype(np.float32)
    lab = g.permutation(M).astype(np.uint16)
    N = 150
    tx = g.integers(0, M, N).astype(np.uint16)
    s2 = 0.05 if M == 8 else 0.2
    y = (pts[tx].astype(np.float64) + math.sqrt(s2) * g.standard_normal((N, D))).astype(np.float32)
    L, gb, mib = _brute(pts, lab, s2, y, tx)
    r = oracle.demap(pts, lab, s2, y, tx)
    assert _rel_err(r["llr"], L) < 1e-12
    assert np.max(np.abs(r["g"] - gb)) < 1e-11
    assert np.max(np.abs(r["mi"] - mib)) < 1e-11
    assert abs(r["gmi"] - float(np.mean(gb))) < 1e-12


# ---------------------------------------------------------------------------- edge cases

def test_empty_block_and_bad_arguments():
    c = W.dp_qpsk()
    r = oracle.demap(c.points, c.labels, 0.1, np.zeros((0, 4), np.float32), np.zeros(0, np.uint16))
    assert math.isnan(r["gmi"]) and r["llr"].shape == (0, 4)
    bad = c.labels.copy()
    bad[1] = bad[0]
    with pytest.raises(ValueError):
        oracle.demap(c.points, bad, 0.1, np.zeros((1, 4), np.float32), np.zeros(1, np.uint16))
    with pytest.raises(ValueError):
        oracle.demap(c.points, c.labels, 0.0, np.zeros((1, 4), np.float32), np.zeros(1, np.uint16))
