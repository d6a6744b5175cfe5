"""Shared helpers of the GPU parity tests: seeded inputs on the device, comparisons."""
from __future__ import annotations

import numpy as np

import workloads as W

LLR_TOL_FP32 = 1e-5  # max |llr_gpu - llr_ref| / max(1, |llr_ref|)
GMI_TOL = 1e-4       # bits per symbol


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    if got.size == 0:
        return 0.0
    return float(np.max(np.abs(got - ref) / np.maximum(1.0, np.abs(ref))))


class DeviceBlock:
    """tx, unit noise and per-SNR received blocks of a constellation, resident on the GPU."""

    def __init__(self, const, tx, z, sigma2, device="cuda:0"):
        import torch
        self.const = const
        self.tx = tx
        self.sigma2 = np.asarray(sigma2, dtype=np.float64)
        self.dev = torch.device(device)
        self.tx_t = torch.from_numpy(tx.view(np.int16)).to(self.dev)
        z_t = torch.from_numpy(np.ascontiguousarray(z)).to(self.dev)
        self.ys = [W.awgn_torch(const.points, self.tx_t, z_t, v) for v in self.sigma2]
        del z_t
        self.N = int(tx.shape[0])

    def y_host(self, s, idx=None):
        y = self.ys[s] if idx is None else self.ys[s][idx]
        return y.cpu().numpy()

    def new_llrs(self):
        import torch
        return [torch.full((self.N, self.const.m), float("nan"), dtype=torch.float32, device=self.dev)
                for _ in self.sigma2]
