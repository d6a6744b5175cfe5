"""C-ABI library checks that need no GPU: it loads, exports every declared symbol,
and its host-side validation rejects bad arguments before touching the device."""
from __future__ import annotations

import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

import paper_2108_07004_amd as dm
import workloads as W

ROOT = Path(__file__).resolve().parent.parent


def _declared_symbols():
    names = set()
    for h in (ROOT / "include").glob("*.h"):
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names |= set(re.findall(r"\b(dm_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = dm.load_library()
    syms = _declared_symbols()
    assert "dm_demap_llr" in syms and "dm_gmi_estimate" in syms
    for s in syms:
        assert hasattr(lib, s), f"{s} declared in include/ but not exported"


def test_version_and_error_strings():
    lib = dm.load_library()
    assert b"gfx950" in lib.dm_version()
    assert isinstance(lib.dm_last_error(), bytes)


def _create(points, labels):
    lib = dm.load_library()
    h = ctypes.c_void_p()
    rc = lib.dm_constellation_create(points.ctypes.data_as(ctypes.c_void_p), labels.ctypes.data_as(ctypes.c_void_p),
                                     points.shape[0], points.shape[1], ctypes.byref(h))
    return rc, lib.dm_last_error().decode()


def test_constellation_validation_on_host():
    c = W.dp_qpsk()
    bad = c.labels.copy()
    bad[3] = bad[2]
    rc, msg = _create(c.points, bad)
    assert rc == -1 and "bijection" in msg
    rc, msg = _create(c.points[:12].copy(), c.labels[:12].copy())
    assert rc == -1 and "power of two" in msg
    pts = c.points.copy()
    pts[0, 0] = np.nan
    rc, msg = _create(pts, c.labels)
    assert rc == -1 and "finite" in msg
    big = np.zeros((2, 33), np.float32)
    rc, msg = _create(big, np.array([0, 1], np.uint16))
    assert rc == -2


def test_null_arguments_rejected():
    lib = dm.load_library()
    assert lib.dm_demap_llr(None, 1.0, None, 0, None, 0, None) == -1
    assert lib.dm_gmi_estimate(None, 1, None, None, None, 0, None, None, None, 0, None) == -1
    assert lib.dm_last_fixup_count(None, 0) in (-1,) or lib.dm_last_fixup_count(None, 0) >= 0


def test_python_binding_has_no_cpu_path():
    src = (ROOT / "paper_2108_07004_amd" / "__init__.py").read_text()
    assert "import oracle" not in src and "from oracle" not in src
    for p in (ROOT / "paper_2108_07004_amd").rglob("*"):
        if p.suffix in (".py", ".hip", ".hpp", ".cpp", ".h"):
            t = p.read_text()
            assert "oracle" not in t.replace("no oracle", ""), f"{p} mentions the oracle"
