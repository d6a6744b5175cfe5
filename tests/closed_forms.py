"""Closed-form GMI / MI of product-labelled AWGN constellations (test pins).

Independent of the oracle: these integrate the bit-metric definitions over the
1D noise density with two separate quadrature rules (Gauss-Hermite and adaptive
``scipy.integrate.quad``).  They apply where the likelihood factorises over
dimensions and each label bit belongs to one dimension (DP-QPSK, products of
BRGC 4-PAM), so a D-dimensional GMI/MI is D times a 1D integral.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def _pam(levels):
    idx = np.arange(levels)
    amps = (2 * idx - (levels - 1)).astype(np.float64)
    amps = amps * math.sqrt(1.0 / (2.0 * np.mean(amps * amps)))
    return amps, idx ^ (idx >> 1)


def _logsumexp(v):
    mx = max(v)
    return mx + math.log(sum(math.exp(t - mx) for t in v))


def _bit_terms_1d(levels, sigma2, i, y):
    """For tx level i and received y: (sum over bits of the GMI term, MI term)."""
    amps, lab = _pam(levels)
    q = int(round(math.log2(levels)))
    v = [-(y - a) ** 2 / (2 * sigma2) for a in amps]
    g = 0.0
    for k in range(q):
        bit = lambda j: (int(lab[j]) >> (q - 1 - k)) & 1
        l1 = _logsumexp([v[j] for j in range(levels) if bit(j) == 1])
        l0 = _logsumexp([v[j] for j in range(levels) if bit(j) == 0])
        lam = l1 - l0
        s = lam if bit(i) == 0 else -lam
        g += 1.0 - (max(s, 0.0) + math.log1p(math.exp(-abs(s)))) / math.log(2.0)
    mi = q - (_logsumexp(v) - v[i]) / math.log(2.0)
    return g, mi


def pam_gmi_mi_gh(levels: int, sigma2: float, nodes: int = 160):
    """1D GMI and MI (bits per real dimension) by Gauss-Hermite quadrature."""
    x, w = np.polynomial.hermite.hermgauss(nodes)
    amps, _ = _pam(levels)
    s = math.sqrt(sigma2)
    G = MI = 0.0
    for i in range(levels):
        for xn, wn in zip(x, w):
            y = amps[i] + s * math.sqrt(2.0) * xn
            g, mi = _bit_terms_1d(levels, sigma2, i, y)
            G += wn * g
            MI += wn * mi
    norm = levels * math.sqrt(math.pi)
    return G / norm, MI / norm


def pam_second_moments_gh(levels: int, sigma2: float, nodes: int = 160):
    """E[g^2] and E[mi^2] of the 1D per-symbol terms (for the true Monte-Carlo standard error)."""
    x, w = np.polynomial.hermite.hermgauss(nodes)
    amps, _ = _pam(levels)
    s = math.sqrt(sigma2)
    G2 = M2 = 0.0
    for i in range(levels):
        for xn, wn in zip(x, w):
            g, mi = _bit_terms_1d(levels, sigma2, i, amps[i] + s * math.sqrt(2.0) * xn)
            G2 += wn * g * g
            M2 += wn * mi * mi
    norm = levels * math.sqrt(math.pi)
    return G2 / norm, M2 / norm


def product_se(levels: int, dims: int, sigma2: float, N: int):
    """Standard errors of the N-symbol GMI/MI means of a dims-fold product PAM."""
    g1, mi1 = pam_gmi_mi_gh(levels, sigma2)
    g2, mi2 = pam_second_moments_gh(levels, sigma2)
    return (math.sqrt(max(dims * (g2 - g1 * g1), 0.0) / N),
            math.sqrt(max(dims * (mi2 - mi1 * mi1), 0.0) / N))


def pam_gmi_mi_quad(levels: int, sigma2: float):
    """1D GMI and MI by adaptive quadrature over the Gaussian noise density."""
    amps, _ = _pam(levels)
    s = math.sqrt(sigma2)
    pdf = lambda z: math.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)
    G = MI = 0.0
    for i in range(levels):
        G += integrate.quad(lambda z: pdf(z) * _bit_terms_1d(levels, sigma2, i, amps[i] + s * z)[0],
                            -12, 12, epsabs=1e-13, epsrel=1e-12, limit=400)[0]
        MI += integrate.quad(lambda z: pdf(z) * _bit_terms_1d(levels, sigma2, i, amps[i] + s * z)[1],
                             -12, 12, epsabs=1e-13, epsrel=1e-12, limit=400)[0]
    return G / levels, MI / levels


def bpsk_bit_gmi_formula(rho: float, nodes: int = 160) -> float:
    """Per-bit GMI of BPSK at amplitude 1/sqrt2: 1 - E log2(1 + exp(-2 rho - 2 sqrt(rho) z))."""
    x, w = np.polynomial.hermite.hermgauss(nodes)
    z = math.sqrt(2.0) * x
    a = -2 * rho - 2 * math.sqrt(rho) * z
    sp = np.maximum(a, 0) + np.log1p(np.exp(-np.abs(a)))
    return 1.0 - float(np.sum(w * sp) / math.sqrt(math.pi)) / math.log(2.0)
