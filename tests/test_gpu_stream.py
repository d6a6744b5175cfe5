"""Streamed demapping of host arrays: LLRs identical to the one-shot device call for every buffer
size and ring depth (ragged last buffer, a single short buffer, the empty block), and equal to
the oracle within the FP32 bound."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import paper_2108_07004_amd as dm
import workloads as W
from gpu_helpers import LLR_TOL_FP32, rel_err

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "fp16x3"])
def test_streamed_llrs_equal_one_shot(prec):
    import torch
    w = W.workload("dp16qam", N=100_003)
    tx, z = W.workload_tx_noise(w)
    s2 = float(W.sigma2_from_snr_db(12.0))
    y = W.awgn(w.const.points, tx, z, s2)
    const = dm.Constellation(w.const.points, w.const.labels)
    ref = dm.demap_llr(const, s2, torch.from_numpy(y).cuda(), prec=prec).cpu().numpy()
    for B, nb in ((4096, 2), (30_000, 3), (1 << 20, 4)):
        st = dm.Streamer(const, buffer_symbols=B, n_buffers=nb, prec=prec)
        llr, sec = st.run(s2, y)
        assert np.array_equal(llr, ref), (B, nb)
        assert sec > 0.0
        st.close()
    # page-locked caller arrays are transferred directly (no staging copies)
    y_pin = torch.from_numpy(y).pin_memory()
    l_pin = torch.empty((y.shape[0], 8), dtype=torch.float32).pin_memory()
    st = dm.Streamer(const, buffer_symbols=30_000, n_buffers=3, prec=prec)
    st.run(s2, y_pin, l_pin)
    st.close()
    assert np.array_equal(l_pin.numpy(), ref)
    if prec == "fp32":
        o = oracle.demap(w.const.points, w.const.labels, s2, y[:5000], tx[:5000])
        assert rel_err(ref[:5000], o["llr"]) <= LLR_TOL_FP32


def test_streamer_edge_cases():
    c = W.dp_qpsk()
    const = dm.Constellation(c.points, c.labels)
    st = dm.Streamer(const, buffer_symbols=1000, n_buffers=2)
    llr, _ = st.run(0.1, np.zeros((0, 4), dtype=np.float32))
    assert llr.shape == (0, 4)
    y = W.awgn(c.points, W.tx_indices(16, 7, 0), W.unit_noise(7, 4, 0), 0.1)
    llr, _ = st.run(0.1, y)
    o = oracle.demap(c.points, c.labels, 0.1, y, W.tx_indices(16, 7, 0))
    assert rel_err(llr, o["llr"]) <= LLR_TOL_FP32
    with pytest.raises(dm.DemapError):
        dm.Streamer(const, buffer_symbols=0)
    with pytest.raises(dm.DemapError):
        dm.Streamer(const, n_buffers=1)
