"""FP64 CPU oracle for the soft demapper — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2108_07004_amd``) and neither imports the other; the seeded inputs
both consume come from ``workloads``.

Contents:
* ``demap``: exact LLRs / GMI / MI terms from the plain C implementation in
  ``demap_oracle.c`` (bit-metric decoding definitions, FP64, subset-wise
  log-sum-exp).  Pinned by closed forms, invariants, metamorphic relations and
  a 50-digit brute force in ``tests/test_oracle_pins.py``.
* ``mlp``: FP64 NumPy forward/backward/Adam of the learned demapper network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "demap_oracle.c"
_LIB = _HERE / "liboracle.so"

_lib = None


def build(force: bool = False) -> Path:
    """Compile the C oracle with gcc (IEEE FP64, no contraction, OpenMP over symbols)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", str(_SRC), "-o", str(tmp), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(str(_LIB))
        P = ctypes.c_void_p
        lib.oracle_demap.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_double, P, P,
                                     ctypes.c_int64, P, P, P, P, P, ctypes.c_int]
        lib.oracle_demap.restype = ctypes.c_int
        lib.oracle_gmi_from_llr.argtypes = [ctypes.c_int, P, P, ctypes.c_int64, P]
        lib.oracle_gmi_from_llr.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_hard_demap.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int64, P, P, P]
        lib.oracle_hard_demap.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def demap(points, labels, sigma2, y, tx, *, llr=True, nthreads=0):
    """Exact FP64 demapping of N symbols.

    Returns dict(llr=(N, m) float64 or None, g=(N,), mi=(N,), gmi=float, mi_mean=float).
    LLR index k is label bit (m-1-k); LLRs are ln P(b=1|y)/P(b=0|y) in nats.
    """
    lib = _load()
    points = np.ascontiguousarray(points, dtype=np.float32)
    labels = np.ascontiguousarray(labels, dtype=np.uint16)
    y = np.ascontiguousarray(y, dtype=np.float32)
    tx = np.ascontiguousarray(tx, dtype=np.uint16)
    M, D = points.shape
    m = int(M).bit_length() - 1
    N = int(y.shape[0])
    if y.ndim != 2 or y.shape[1] != D or tx.shape != (N,):
        raise ValueError("shape mismatch")
    L = np.empty((N, m), dtype=np.float64) if llr else None
    g = np.empty(N, dtype=np.float64)
    mi = np.empty(N, dtype=np.float64)
    gmi = np.empty(1, dtype=np.float64)
    mim = np.empty(1, dtype=np.float64)
    rc = lib.oracle_demap(M, D, _ptr(points), _ptr(labels), float(sigma2), _ptr(y), _ptr(tx), N,
                          _ptr(L), _ptr(g), _ptr(mi), _ptr(gmi), _ptr(mim), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_demap rejected its arguments (rc={rc})")
    return {"llr": L, "g": g, "mi": mi, "gmi": float(gmi[0]), "mi_mean": float(mim[0])}


def gmi_from_llr(m, llr, tx_label):
    """GMI (bits/symbol) of arbitrary LLRs (nats) against transmitted labels."""
    lib = _load()
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    tx_label = np.ascontiguousarray(tx_label, dtype=np.uint16)
    out = np.empty(1, dtype=np.float64)
    rc = lib.oracle_gmi_from_llr(int(m), _ptr(llr), _ptr(tx_label), int(llr.shape[0]), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_gmi_from_llr rejected its arguments")
    return float(out[0])


def hard_demap(points, labels, y, tx=None):
    """Minimum-distance decisions (FP32 fused distance, ties to the lowest label) and, with tx,
    the symbol and bit error counts.  Returns dict(labels=(N,) uint16, sym_err=int, bit_err=int)."""
    lib = _load()
    points = np.ascontiguousarray(points, dtype=np.float32)
    labels = np.ascontiguousarray(labels, dtype=np.uint16)
    y = np.ascontiguousarray(y, dtype=np.float32)
    M, D = points.shape
    N = int(y.shape[0])
    if y.ndim != 2 or y.shape[1] != D:
        raise ValueError("shape mismatch")
    out = np.empty(N, dtype=np.uint16)
    txa = None if tx is None else np.ascontiguousarray(tx, dtype=np.uint16)
    se = np.zeros(1, dtype=np.int64)
    be = np.zeros(1, dtype=np.int64)
    rc = lib.oracle_hard_demap(M, D, _ptr(points), _ptr(labels), _ptr(y), _ptr(txa), N, _ptr(out), _ptr(se), _ptr(be))
    if rc != 0:
        raise ValueError(f"oracle_hard_demap rejected its arguments (rc={rc})")
    return {"labels": out, "sym_err": int(se[0]), "bit_err": int(be[0])}
