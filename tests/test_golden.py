"""Stored oracle cases (``tests/golden/oracle_cases.json``): the seeded generators and the FP64
oracle must still reproduce them.

The fixture is written by ``tests/golden/make_golden.py`` from ``oracle.demap`` alone; this test
guards it against drift of the input generators (constellation hash, tx, received blocks
bit-exact) and of the oracle's arithmetic (LLRs within 1e-12 relative, GMI / MI within 1e-12
bit).  The GPU comparison against the same file is in ``test_gpu_golden.py``.
"""
from __future__ import annotations

import json
import sys
from pathlib import Path

import numpy as np
import pytest

import oracle
import workloads as W

_GOLDEN = Path(__file__).resolve().parent / "golden"
sys.path.insert(0, str(_GOLDEN))
import make_golden  # noqa: E402

CASES = json.loads((_GOLDEN / "oracle_cases.json").read_text())["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_generators_and_oracle_reproduce_the_stored_case(case):
    c, tx, z, snr = make_golden.case_inputs(case["name"])
    assert make_golden.const_hash(c) == case["const_sha256"]
    assert (c.M, c.D) == (case["M"], case["D"])
    assert np.array_equal(tx, np.asarray(case["tx"], dtype=np.uint16))
    assert list(snr) == case["snr_db"]
    for s_db, p in zip(snr, case["points"]):
        assert p["sigma2"] == float(W.sigma2_from_snr_db(s_db))
        y = np.asarray(p["y"], dtype=np.float32)
        assert np.array_equal(y, W.awgn(c.points, tx, z, p["sigma2"]))
        ref = oracle.demap(c.points, c.labels, p["sigma2"], y, tx)
        want = np.asarray(p["llr"], dtype=np.float64)
        assert want.shape == (len(tx), c.m)
        err = np.max(np.abs(ref["llr"] - want) / np.maximum(1.0, np.abs(want)))
        assert err <= 1e-12, (case["name"], s_db, err)
        assert abs(ref["gmi"] - p["gmi"]) <= 1e-12
        assert abs(ref["mi_mean"] - p["mi"]) <= 1e-12

