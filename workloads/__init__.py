"""Seeded synthetic inputs for the soft demapper and its oracle.

This module is the only code shared by the GPU path and the FP64 oracle, and it
holds none of the demapping arithmetic: it draws constellations (point table +
binary labelling), transmitted point indices, unit-variance Gaussian noise and
forms the AWGN channel output y = fl32(x + sigma * z).

Conventions (the paper gives none of them; these are the readings used
throughout the project):

* Random numbers come from NumPy's PCG64 generator, as the paper's transmitter
  does for its symbol sequences (Sec. 3, experimental setup).  Each purpose
  draws from its own stream, derived with ``SeedSequence(BASE_SEED,
  spawn_key=(config, purpose, ...))``.
* Constellations are normalised to unit energy per two real dimensions, so
  E||x||^2 = D/2.  The SNR is Es(2D)/N0 with N0 = 2 sigma^2, hence
  sigma^2 = 1 / (2 * 10^(SNR_dB/10)) for every dimensionality D.
* A constellation is given as the paper's receiver receives it (Sec. 2): an
  arbitrary point table and its bit mapping, uploaded as-is.  Rows need not be
  in label order; the labelling is a bijection onto [0, M).
* One noise draw z is shared by all SNR points of a configuration (common
  random numbers); y_s = fl32(x_tx + sigma_s * z) with the product and the sum
  each rounded in FP64 (no fused multiply-add), then rounded once to FP32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 210807004

_PURPOSES = {
    "constellation": 0,
    "tx": 1,
    "noise": 2,
    "snr": 3,
    "instances": 4,
    "mlp_init": 5,
    "mlp_train": 6,
    "mlp_eval": 7,
    "misc": 8,
}


def rng(config: int, purpose: str, *extra: int) -> np.random.Generator:
    """PCG64 stream for (config, purpose, *extra) under the project base seed."""
    key = (int(config), _PURPOSES[purpose]) + tuple(int(e) for e in extra)
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(BASE_SEED, spawn_key=key)))


def sigma2_from_snr_db(snr_db) -> np.ndarray:
    """Noise variance per real dimension for unit energy per 2D: 1/(2*10^(SNR/10))."""
    s = np.asarray(snr_db, dtype=np.float64)
    return 1.0 / (2.0 * np.power(10.0, s / 10.0))


@dataclass(frozen=True)
class Constellation:
    """Point table (M x D, float32, arbitrary row order) and labels (M, uint16)."""

    points: np.ndarray
    labels: np.ndarray
    name: str = ""

    @property
    def M(self) -> int:
        return int(self.points.shape[0])

    @property
    def D(self) -> int:
        return int(self.points.shape[1])

    @property
    def m(self) -> int:
        return int(round(math.log2(self.M)))


def _gray(i: np.ndarray) -> np.ndarray:
    return i ^ (i >> 1)


def pam_brgc(levels: int) -> tuple[np.ndarray, np.ndarray]:
    """Equally spaced PAM amplitudes (ascending, unnormalised odd integers) and their BRGC labels."""
    idx = np.arange(levels, dtype=np.int64)
    amps = (2 * idx - (levels - 1)).astype(np.float64)
    return amps, _gray(idx)


def product_pam(levels: int, D: int, name: str) -> Constellation:
    """D-fold product of a BRGC-labelled PAM, unit energy per 2D.

    Row r enumerates amplitude indices (a_0, ..., a_{D-1}) in ascending
    lexicographic order of the amplitudes; the label concatenates the per-
    dimension BRGC labels with dimension 0 in the most significant position.
    """
    amps, glab = pam_brgc(levels)
    q = int(round(math.log2(levels)))
    scale = math.sqrt(1.0 / (2.0 * float(np.mean(amps * amps))))  # E x_d^2 = 1/2
    grids = np.stack(np.meshgrid(*([np.arange(levels)] * D), indexing="ij"), axis=-1).reshape(-1, D)
    pts = (amps[grids] * scale).astype(np.float32)
    lab = np.zeros(grids.shape[0], dtype=np.int64)
    for d in range(D):
        lab = (lab << q) | glab[grids[:, d]]
    return Constellation(pts, lab.astype(np.uint16), name)


def product_pam_mixed(levels: list, name: str = "") -> Constellation:
    """Product of BRGC-labelled PAMs with levels[d] points in dimension d, each scaled so that
    E x_d^2 = 1/2 (unit energy per 2D); rows in ascending lexicographic amplitude order, label =
    concatenated per-dimension BRGC labels, dimension 0 most significant.  With levels
    (4, 4, 4, 2, 2, 2, 2, 2) it is an 8D, M = 2048 constellation whose bit LLRs each depend on one
    coordinate (a structured counterpart of the random 8D constellation)."""
    D = len(levels)
    per = [pam_brgc(L) for L in levels]
    qs = [int(round(math.log2(L))) for L in levels]
    grids = np.stack(np.meshgrid(*[np.arange(L) for L in levels], indexing="ij"), axis=-1).reshape(-1, D)
    pts = np.empty(grids.shape, dtype=np.float64)
    lab = np.zeros(grids.shape[0], dtype=np.int64)
    for d, (amps, glab) in enumerate(per):
        scale = math.sqrt(1.0 / (2.0 * float(np.mean(amps * amps))))
        pts[:, d] = amps[grids[:, d]] * scale
        lab = (lab << qs[d]) | glab[grids[:, d]]
    return Constellation(pts.astype(np.float32), lab.astype(np.uint16), name)


def dp_qpsk() -> Constellation:
    """DP-QPSK: 4D, M=16, per-quadrature BRGC (bit 0 -> -A, 1 -> +A, A=1/sqrt2)."""
    return product_pam(2, 4, "dp-qpsk")


def dp_16qam() -> Constellation:
    """Product of two Gray 16QAM: 4D, M=256, per-dimension 4-PAM with BRGC {00,01,11,10}."""
    return product_pam(4, 4, "dp-16qam")


def rect_qam(levels_i: int, levels_q: int, name: str = "") -> Constellation:
    """Rectangular QAM: BRGC PAM in each of two dimensions (I bits most significant), unit
    energy per 2D.  rect_qam(4, 2) is the rectangular 8-QAM."""
    ai, gi = pam_brgc(levels_i)
    aq, gq = pam_brgc(levels_q)
    qb = int(round(math.log2(levels_q)))
    pts, lab = [], []
    for i in range(levels_i):
        for q in range(levels_q):
            pts.append((ai[i], aq[q]))
            lab.append((int(gi[i]) << qb) | int(gq[q]))
    p = np.asarray(pts, dtype=np.float64)
    p *= math.sqrt(1.0 / float(np.mean(np.sum(p * p, axis=1))))
    return Constellation(p.astype(np.float32), np.asarray(lab, dtype=np.uint16),
                         name or f"{levels_i * levels_q}-qam-rect")


def cross_qam(M: int, name: str = "") -> Constellation:
    """Cross QAM (M = 32 or 128): a square grid of odd integer amplitudes with the four corner
    blocks removed (6 x 6 minus 4 corners for 32, 12 x 12 minus four 2 x 2 corners for
    128), unit energy per 2D.  Labels are the raster index of the kept points (the paper's own
    mappings are not published; any bijection is a valid labelling)."""
    side, cut = {32: (6, 1), 128: (12, 2)}[M]
    amps = 2 * np.arange(side) - (side - 1)
    pts = []
    for i in range(side):
        for q in range(side):
            corner = (i < cut or i >= side - cut) and (q < cut or q >= side - cut)
            if not corner:
                pts.append((amps[i], amps[q]))
    p = np.asarray(pts, dtype=np.float64)
    p *= math.sqrt(1.0 / float(np.mean(np.sum(p * p, axis=1))))
    return Constellation(p.astype(np.float32), np.arange(M, dtype=np.uint16), name or f"{M}-qam-cross")


def qam(M: int) -> Constellation:
    """The paper's conventional 2D formats: 4-, 16-, 64-QAM square Gray, 8-QAM rectangular,
    32- and 128-QAM cross."""
    if M in (4, 16, 64, 256):
        k = int(round(math.sqrt(M)))
        return product_pam(k, 2, f"{M}-qam")
    if M == 8:
        return rect_qam(4, 2, "8-qam")
    if M in (32, 128):
        return cross_qam(M)
    raise KeyError(M)


def pam(levels: int) -> Constellation:
    """1D BRGC PAM (used by closed-form checks)."""
    return product_pam(levels, 1, f"{levels}-pam")


def gaussian_constellation(M: int, D: int, config: int, *extra: int) -> Constellation:
    """Random constellation: i.i.d. N(0,1) points rescaled to unit energy per 2D; label j = j."""
    g = rng(config, "constellation", *extra)
    X = g.standard_normal((M, D))
    X *= math.sqrt((D / 2.0) / float(np.mean(np.sum(X * X, axis=1))))
    return Constellation(X.astype(np.float32), np.arange(M, dtype=np.uint16), f"gauss-{D}d-{M}")


def tx_indices(M: int, N: int, config: int, *extra: int) -> np.ndarray:
    """Transmitted point (row) indices, uniform i.i.d. on [0, M)."""
    return rng(config, "tx", *extra).integers(0, M, size=N, dtype=np.int64).astype(np.uint16)


def unit_noise(N: int, D: int, config: int, *extra: int) -> np.ndarray:
    """Unit-variance real Gaussian noise, FP64, N x D (shared by all SNR points)."""
    return rng(config, "noise", *extra).standard_normal((N, D))


def awgn(points: np.ndarray, tx: np.ndarray, z: np.ndarray, sigma2: float) -> np.ndarray:
    """Channel output fl32(x_tx + sigma*z): FP64 product, FP64 sum, one FP32 rounding."""
    x = points.astype(np.float64)[tx.astype(np.int64)]
    s = math.sqrt(float(sigma2))
    return (x + s * z).astype(np.float32)


# --------------------------------------------------------------------------------------------
# Workload recipes (sizes and SNR grids of the measured configurations)
# --------------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    config: int
    const: Constellation
    N: int
    snr_db: np.ndarray

    @property
    def sigma2(self) -> np.ndarray:
        return sigma2_from_snr_db(self.snr_db)


def workload(name: str, N: int | None = None) -> Workload:
    """Named workloads; ``N`` overrides the symbol count (a prefix of the same streams)."""
    if name == "dpqpsk":
        c, n, snr, cfg = dp_qpsk(), 65536, np.arange(0, 11, 2, dtype=np.float64), 0
    elif name == "dp16qam":
        c, n, snr, cfg = dp_16qam(), 1 << 22, np.arange(0, 21, 2, dtype=np.float64), 1
    elif name == "gauss8d2048":
        c, n, snr, cfg = gaussian_constellation(2048, 8, 2), 1 << 24, np.arange(0, 16, 1, dtype=np.float64), 2
    else:
        raise KeyError(name)
    return Workload(name, cfg, c, int(n if N is None else N), snr)


def workload_tx_noise(w: Workload) -> tuple[np.ndarray, np.ndarray]:
    """tx indices and unit noise of a workload; a smaller N is a prefix of the full draw."""
    full = {"dpqpsk": 65536, "dp16qam": 1 << 22, "gauss8d2048": 1 << 24}[w.name]
    if w.N > full:
        raise ValueError("N larger than the workload's full size")
    # Draw in fixed-size chunks so any prefix is reproducible without drawing the whole block.
    tx = _chunked_tx(w.const.M, w.N, w.config)
    z = _chunked_noise(w.N, w.const.D, w.config)
    return tx, z


_CHUNK = 1 << 16


def _chunked_tx(M: int, N: int, config: int) -> np.ndarray:
    out = np.empty(N, dtype=np.uint16)
    for c0 in range(0, N, _CHUNK):
        c1 = min(N, c0 + _CHUNK)
        out[c0:c1] = tx_indices(M, _CHUNK, config, c0 // _CHUNK)[: c1 - c0]
    return out


def _chunked_noise(N: int, D: int, config: int) -> np.ndarray:
    out = np.empty((N, D), dtype=np.float64)
    for c0 in range(0, N, _CHUNK):
        c1 = min(N, c0 + _CHUNK)
        out[c0:c1] = unit_noise(_CHUNK, D, config, c0 // _CHUNK)[: c1 - c0]
    return out


def chunk_tx_noise(M: int, D: int, config: int, first: int, count: int) -> tuple[np.ndarray, np.ndarray]:
    """tx and z for symbols [first, first+count) of a chunked workload stream."""
    tx = np.empty(count, dtype=np.uint16)
    z = np.empty((count, D), dtype=np.float64)
    pos = 0
    while pos < count:
        n = first + pos
        ci, off = divmod(n, _CHUNK)
        take = min(_CHUNK - off, count - pos)
        tx[pos:pos + take] = tx_indices(M, _CHUNK, config, ci)[off:off + take]
        z[pos:pos + take] = unit_noise(_CHUNK, D, config, ci)[off:off + take]
        pos += take
    return tx, z


def awgn_torch(points, tx, z, sigma2):
    """GPU twin of ``awgn``: same FP64 product and sum, one FP32 rounding (bit-identical).

    points: (M, D) float32 array or tensor; tx: (N,) integer tensor; z: (N, D) float64 tensor.
    """
    import torch
    dev = z.device
    p64 = torch.as_tensor(np.asarray(points), dtype=torch.float32).to(dev).to(torch.float64)
    x = p64[tx.to(torch.int64)]
    s = math.sqrt(float(sigma2))
    return (x + (z * s)).to(torch.float32)


def mlp_init_weights(D: int, H: int, m: int, config: int = 4) -> dict:
    """Seeded initial weights of the learned demapper's MLP (FP32 master copies).

    Uniform(-b, b) with b = 0.5 sqrt(6 / fan_in); zero biases.  Row-major W (fan_in, fan_out).
    """
    g = rng(config, "mlp_init", D, H, m)
    w = {}
    for name, fi, fo in (("1", D + 1, H), ("2", H, H), ("3", H, m)):
        b = 0.5 * math.sqrt(6.0 / fi)
        w["W" + name] = g.uniform(-b, b, (fi, fo)).astype(np.float32)
        w["b" + name] = np.zeros(fo, dtype=np.float32)
    return w


@dataclass(frozen=True)
class Instance:
    """One batched instance: constellation, SNR, block size and its own tx / noise streams."""
    index: int
    const: Constellation
    N: int
    snr_db: float

    @property
    def sigma2(self) -> float:
        return float(sigma2_from_snr_db(self.snr_db))

    def tx_noise(self, N: int | None = None):
        n = self.N if N is None else N
        return tx_indices(self.const.M, n, 3, self.index), unit_noise(n, self.const.D, 3, self.index)


def batched_instances(count: int = 64, n_lo: int = 14, n_hi: int = 22) -> list:
    """Uneven instances: M in {16,64,256,1024,2048}, D in {2,4,8}, N log-uniform in
    [2^n_lo, 2^n_hi], SNR uniform in [0, 20] dB; Gaussian constellations as the 8D recipe,
    except (M, D) = (16, 4) -> DP-QPSK and (256, 4) -> DP-16QAM."""
    g = rng(3, "instances")
    out = []
    for i in range(count):
        M = int(g.choice([16, 64, 256, 1024, 2048]))
        D = int(g.choice([2, 4, 8]))
        N = int(round(2.0 ** g.uniform(n_lo, n_hi)))
        snr = float(g.uniform(0.0, 20.0))
        if (M, D) == (16, 4):
            c = dp_qpsk()
        elif (M, D) == (256, 4):
            c = dp_16qam()
        else:
            c = gaussian_constellation(M, D, 3, i)
        out.append(Instance(i, c, N, snr))
    return out


def mlp_samples(const: Constellation, N: int, snr_lo: float = 0.0, snr_hi: float = 15.0, config: int = 4,
                purpose: str = "mlp_train", *extra: int):
    """Training / evaluation samples of the learned demapper: uniform transmitted rows, an SNR per
    sample drawn uniformly (continuous, dB) from [snr_lo, snr_hi], y = fl32(x + sigma z).

    Returns (y float32 (N, D), sigma2 float32 (N,), tx uint16 (N,), snr_db float64 (N,)).
    """
    g = rng(config, purpose, *extra)
    M, D = const.points.shape
    tx = g.integers(0, M, size=N, dtype=np.int64)
    snr = g.uniform(snr_lo, snr_hi, size=N)
    z = g.standard_normal((N, D))
    s2 = sigma2_from_snr_db(snr)
    y = (const.points.astype(np.float64)[tx] + np.sqrt(s2)[:, None] * z).astype(np.float32)
    return y, s2.astype(np.float32), tx.astype(np.uint16), snr


def mlp_samples_torch(points, N: int, snr_lo: float, snr_hi: float, device, config: int = 4, *extra: int):
    """Device-side twin of ``mlp_samples`` for large N (torch's seeded generator on the GPU; the
    stream differs from NumPy's).  Returns (y float32 (N, D), sigma2 float32 (N,)) tensors."""
    import torch
    seed = int(np.random.SeedSequence(BASE_SEED, spawn_key=(int(config), _PURPOSES["mlp_train"]) +
                                      tuple(int(e) for e in extra)).generate_state(1, np.uint64)[0] >> 1)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    pts = torch.as_tensor(np.asarray(points), dtype=torch.float32).to(device)
    M, D = pts.shape
    tx = torch.randint(0, M, (N,), generator=g, device=device)
    snr = torch.rand(N, generator=g, device=device, dtype=torch.float64) * (snr_hi - snr_lo) + snr_lo
    s2 = 1.0 / (2.0 * torch.pow(10.0, snr / 10.0))
    y = torch.empty((N, D), dtype=torch.float32, device=device)
    step = 1 << 22
    for a in range(0, N, step):
        b = min(N, a + step)
        z = torch.randn((b - a, D), generator=g, device=device, dtype=torch.float64)
        y[a:b] = (pts[tx[a:b]].to(torch.float64) + torch.sqrt(s2[a:b])[:, None] * z).to(torch.float32)
    return y, s2.to(torch.float32)
