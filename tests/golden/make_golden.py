"""Writes ``oracle_cases.json``: small seeded demapping cases with the FP64 oracle's results.

Run from the repository root: ``python tests/golden/make_golden.py``.  Every input comes from
the seeded generators in ``workloads`` and every expected value from ``oracle.demap``; nothing
here touches the GPU library.  The stored received blocks make the GPU comparison independent
of the generators, and the constellation hashes let the CPU test detect a changed generator.

Cases (the formats of Sec. 2 and Sec. 4 of the paper plus the random 8D constellation):
DP-QPSK, DP-16QAM, rectangular 8-QAM, cross 128-QAM and the random 8D M = 2048 set, each
at a few SNR points with N = 40 symbols (one full 32-symbol batch and a ragged tail).
SNR is Es per 2D over N0 = 2 sigma^2 with unit energy per 2D.
"""
from __future__ import annotations

import hashlib
import json
import sys
from pathlib import Path

import numpy as np

_ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(_ROOT))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = Path(__file__).resolve().parent / "oracle_cases.json"


def const_hash(c) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(c.points, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(c.labels, dtype=np.uint16).tobytes())
    return h.hexdigest()


def case_inputs(name: str):
    """(constellation, tx, unit noise, SNR grid in dB) of one stored case."""
    if name in ("dpqpsk", "dp16qam", "gauss8d2048"):
        N, snr = {"dpqpsk": (40, [0.0, 6.0, 10.0]), "dp16qam": (40, [0.0, 10.0, 20.0]),
                  "gauss8d2048": (40, [0.0, 15.0])}[name]
        w = W.workload(name, N=N)
        tx, z = W.workload_tx_noise(w)
        return w.const, tx, z, snr
    M, N, snr = {"8qam": (8, 40, [14.0]), "128qam": (128, 40, [20.0, 26.0])}[name]
    c = W.qam(M)
    return c, W.tx_indices(M, N, 8, M), W.unit_noise(N, 2, 8, M), snr


CASES = ("dpqpsk", "dp16qam", "8qam", "128qam", "gauss8d2048")


def build_case(name: str) -> dict:
    c, tx, z, snr = case_inputs(name)
    out = {"name": name, "M": int(c.M), "D": int(c.D), "const_sha256": const_hash(c),
           "tx": [int(v) for v in tx], "snr_db": snr, "points": []}
    for s_db in snr:
        s2 = float(W.sigma2_from_snr_db(s_db))
        y = W.awgn(c.points, tx, z, s2)
        ref = oracle.demap(c.points, c.labels, s2, y, tx)
        out["points"].append({
            "sigma2": s2,
            # FP32 inputs in their shortest round-trip form, FP64 results to 17 digits.
            "y": [[json.loads(np.format_float_positional(v, unique=True, trim="-")) for v in row]
                  for row in y],
            "llr": [[float("%.17g" % v) for v in row] for row in ref["llr"]],
            "gmi": ref["gmi"],
            "mi": ref["mi_mean"],
        })
    return out


def main():
    doc = {
        "about": ("Seeded demapping cases and FP64 oracle results (LLR in nats, index k = label "
                  "bit m-1-k; GMI and MI in bits per D-dimensional symbol). Written by "
                  "tests/golden/make_golden.py from oracle.demap; inputs from workloads."),
        "cases": [build_case(n) for n in CASES],
    }
    OUT.write_text(json.dumps(doc, separators=(",", ":")) + "\n")
    print(f"wrote {OUT} ({OUT.stat().st_size} bytes)")


if __name__ == "__main__":
    main()
