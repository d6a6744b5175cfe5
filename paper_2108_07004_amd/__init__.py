"""MI355X soft demapper: exact bit-wise LLRs and Monte-Carlo GMI/MI (HIP, gfx950).

Thin ctypes binding over ``libdemap.so`` (C ABI declared in ``include/demap.h``).
Every computation runs in the library's HIP kernels; this module only checks and
marshals arguments.  PyTorch supplies device memory and the current stream.
If the library is not built the functions raise: there is no CPU fallback.

Python names follow the C entry points without their ``dm_`` prefix:
``demap_llr`` -> ``dm_demap_llr``, ``gmi_estimate`` -> ``dm_gmi_estimate``, ...
"""
from __future__ import annotations

import ctypes
from pathlib import Path
from typing import Sequence

import numpy as np

__all__ = ["Constellation", "DemapError", "MLP", "PREC", "Plan", "demap_batched", "demap_learned", "demap_llr",
           "demap_llr_var", "gmi_estimate", "gs_optimize", "hard_decision", "q_factor_db", "Streamer", "last_fixup_count", "library_path", "load_library", "mlp_param_count",
           "probe_valu_rates", "probe_atomic_rates", "probe_gelu", "profile_enable", "profile_read"]

_LIB_PATH = Path(__file__).resolve().with_name("libdemap.so")
PREC = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x3": 3, "fp16x3": 4}
_ERRORS = {-1: "DM_EINVAL", -2: "DM_EUNSUPPORTED", -3: "DM_EHIP", -4: "DM_ENOMEM"}

_lib = None


class DemapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


def library_path() -> Path:
    return _LIB_PATH


def load_library():
    """Load libdemap.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not _LIB_PATH.exists():
        raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(str(_LIB_PATH))
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.dm_constellation_create.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P)]
    lib.dm_constellation_create.restype = I
    lib.dm_constellation_destroy.argtypes = [P]
    lib.dm_constellation_destroy.restype = None
    lib.dm_demap_llr.argtypes = [P, D, P, I64, P, I, P]
    lib.dm_demap_llr.restype = I
    lib.dm_gmi_estimate.argtypes = [P, I, P, P, P, I64, P, P, P, I, P]
    lib.dm_gmi_estimate.restype = I
    lib.dm_gmi_estimate_noalloc.argtypes = [P, I, P, P, P, I64, P, P, P, I, P]
    lib.dm_gmi_estimate_noalloc.restype = I
    lib.dm_last_fixup_count.argtypes = [P, I]
    lib.dm_last_fixup_count.restype = I64
    lib.dm_probe_valu_rates.argtypes = [P, P]
    lib.dm_probe_valu_rates.restype = I
    lib.dm_probe_atomic_rates.argtypes = [P, P]
    lib.dm_probe_atomic_rates.restype = I
    lib.dm_probe_gelu.argtypes = [P, P, ctypes.c_int64]
    lib.dm_probe_gelu.restype = I
    lib.dm_profile_enable.argtypes = [I]
    lib.dm_profile_enable.restype = I
    lib.dm_profile_read.argtypes = [P, P, P, I]
    lib.dm_profile_read.restype = I
    lib.dm_plan_create.argtypes = [P, I, I, I, ctypes.POINTER(P)]
    lib.dm_plan_create.restype = I
    lib.dm_plan_launch.argtypes = [P, P]
    lib.dm_plan_launch.restype = I
    lib.dm_plan_results.argtypes = [P, P, P, P, P]
    lib.dm_plan_results.restype = I
    lib.dm_plan_info.argtypes = [P, P, P, P]
    lib.dm_plan_info.restype = I
    lib.dm_plan_stats.argtypes = [P, P, P, P]
    lib.dm_plan_stats.restype = I
    lib.dm_plan_destroy.argtypes = [P]
    lib.dm_plan_destroy.restype = None
    lib.dm_demap_batched.argtypes = [P, I, I, I, P, P, P]
    lib.dm_demap_batched.restype = I
    lib.dm_demap_llr_var.argtypes = [P, P, P, I64, P, I, P]
    lib.dm_demap_llr_var.restype = I
    lib.dm_mlp_param_count.argtypes = [ctypes.c_int32, ctypes.c_int32]
    lib.dm_mlp_param_count.restype = I64
    lib.dm_mlp_create.argtypes = [P, P, ctypes.POINTER(P)]
    lib.dm_mlp_create.restype = I
    lib.dm_mlp_destroy.argtypes = [P]
    lib.dm_mlp_destroy.restype = None
    lib.dm_mlp_get_weights.argtypes = [P, P]
    lib.dm_mlp_get_weights.restype = I
    lib.dm_mlp_set_weights.argtypes = [P, P]
    lib.dm_mlp_set_weights.restype = I
    lib.dm_mlp_info.argtypes = [P, P, P, P]
    lib.dm_mlp_info.restype = I
    lib.dm_mlp_train.argtypes = [P, P, P, P, P, I64, P, P]
    lib.dm_mlp_train.restype = I
    lib.dm_mlp_gradients.argtypes = [P, P, P, P, ctypes.c_int32, P, P, P]
    lib.dm_mlp_gradients.restype = I
    lib.dm_demap_learned.argtypes = [P, P, I, P, P, P, I64, P, P, P, P, P, P]
    lib.dm_demap_learned.restype = I
    lib.dm_mlp_save.argtypes = [P, ctypes.c_char_p]
    lib.dm_mlp_save.restype = I
    lib.dm_mlp_load.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(P)]
    lib.dm_mlp_load.restype = I
    lib.dm_hard_decision.argtypes = [P, I, P, P, I64, P, P, P, ctypes.c_int32, P, P]
    lib.dm_hard_decision.restype = I
    lib.dm_q_factor_db.argtypes = [D]
    lib.dm_q_factor_db.restype = D
    lib.dm_gs_optimize.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, P, P, I64, P, P, P, P]
    lib.dm_gs_optimize.restype = I
    lib.dm_streamer_create.argtypes = [P, I64, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(P)]
    lib.dm_streamer_create.restype = I
    lib.dm_streamer_run.argtypes = [P, D, P, I64, P, P]
    lib.dm_streamer_run.restype = I
    lib.dm_streamer_destroy.argtypes = [P]
    lib.dm_streamer_destroy.restype = None
    lib.dm_last_error.restype = ctypes.c_char_p
    lib.dm_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise DemapError(rc, load_library().dm_last_error().decode())


def _stream_handle(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_tensor(t, dtype_names, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if str(t.dtype).replace("torch.", "") not in dtype_names:
        raise TypeError(f"{name} must have dtype in {dtype_names}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Constellation:
    """A point table (M x D) and bit mapping uploaded to the current GPU."""

    def __init__(self, points, labels):
        lib = load_library()
        pts = np.ascontiguousarray(points, dtype=np.float32)
        lab = np.ascontiguousarray(labels, dtype=np.uint16)
        if pts.ndim != 2 or lab.shape != (pts.shape[0],):
            raise ValueError("points must be M x D and labels length M")
        self.M, self.D = int(pts.shape[0]), int(pts.shape[1])
        self.m = self.M.bit_length() - 1
        h = ctypes.c_void_p()
        _check(lib.dm_constellation_create(pts.ctypes.data_as(ctypes.c_void_p), lab.ctypes.data_as(ctypes.c_void_p),
                                           self.M, self.D, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def stats(self):
        """(work items, items per claim, workgroups) of the plan's launch."""
        n = ctypes.c_int64()
        grab = ctypes.c_int32()
        grid = ctypes.c_int32()
        _check(load_library().dm_plan_stats(self._h, ctypes.byref(n), ctypes.byref(grab), ctypes.byref(grid)))
        return int(n.value), int(grab.value), int(grid.value)

    def work_items(self):
        return self.stats()[0]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().dm_constellation_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def demap_llr(const: Constellation, sigma2: float, y, llr=None, prec: str = "fp32", stream=None):
    """Exact LLRs (nats, N x m FP32) of the received block y (N x D FP32 on the GPU)."""
    import torch
    N = int(y.shape[0])
    yp = _dev_tensor(y, ("float32",), (N, const.D), "y")
    if llr is None:
        llr = torch.empty((N, const.m), dtype=torch.float32, device=y.device)
    lp = _dev_tensor(llr, ("float32",), (N, const.m), "llr")
    _check(load_library().dm_demap_llr(const.handle, float(sigma2), yp, N, lp, PREC[prec], _stream_handle(stream)))
    return llr


def gmi_estimate(const: Constellation, sigma2: Sequence[float], ys, tx, llrs=None, prec: str = "fp32",
                 stream=None, want_mi: bool = True, _entry: str = "dm_gmi_estimate"):
    """Monte-Carlo GMI (and MI) in bits/symbol at each noise variance.

    ys: list of n_snr tensors (N x D FP32) or one (n_snr, N, D) tensor.
    tx: (N,) int16/uint16 tensor of transmitted row indices.
    llrs: None, or a list / (n_snr, N, m) tensor receiving the LLRs.
    Returns (gmi, mi) as float64 NumPy arrays (mi is None if want_mi is False).
    """
    s2 = np.ascontiguousarray(np.asarray(sigma2, dtype=np.float64).reshape(-1))
    ns = int(s2.shape[0])
    ylist = [ys[i] for i in range(ns)]
    if len(ylist) != ns:
        raise ValueError("need one received block per SNR point")
    N = int(ylist[0].shape[0])
    yptr = (ctypes.c_void_p * ns)(*[_dev_tensor(t, ("float32",), (N, const.D), "y[s]").value for t in ylist])
    txp = _dev_tensor(tx, ("int16", "uint16"), (N,), "tx")
    lptr = None
    if llrs is not None:
        llist = [llrs[i] for i in range(ns)]
        lptr = (ctypes.c_void_p * ns)(*[_dev_tensor(t, ("float32",), (N, const.m), "llr[s]").value for t in llist])
    gmi = np.empty(ns, dtype=np.float64)
    mi = np.empty(ns, dtype=np.float64) if want_mi else None
    _check(getattr(load_library(), _entry)(
        const.handle, ns, s2.ctypes.data_as(ctypes.c_void_p), ctypes.cast(yptr, ctypes.c_void_p), txp, N,
        None if lptr is None else ctypes.cast(lptr, ctypes.c_void_p), gmi.ctypes.data_as(ctypes.c_void_p),
        None if mi is None else mi.ctypes.data_as(ctypes.c_void_p), PREC[prec], _stream_handle(stream)))
    return gmi, mi


def gmi_estimate_noalloc(const: Constellation, sigma2: Sequence[float], ys, tx, llrs=None, prec: str = "fp32",
                         stream=None, want_mi: bool = True):
    """gmi_estimate through dm_gmi_estimate_noalloc: no device allocation (static scratch),
    at most 32 noise levels per call."""
    return gmi_estimate(const, sigma2, ys, tx, llrs, prec, stream, want_mi, _entry="dm_gmi_estimate_noalloc")


def last_fixup_count(n_snr: int):
    """(total, per-SNR) (symbol, bit) pairs the last gmi_estimate on this thread sent to the fix-up."""
    per = np.zeros(max(1, n_snr), dtype=np.int64)
    tot = load_library().dm_last_fixup_count(per.ctypes.data_as(ctypes.c_void_p), n_snr)
    if tot < 0:
        _check(int(tot))
    return int(tot), per[:n_snr]


def probe_valu_rates(stream=None) -> dict:
    """Measured exp2, FMA and (exp2 + 2 add) rates of the current GPU (dm_probe_valu_rates)."""
    r = np.zeros(4, dtype=np.float64)
    rc = load_library().dm_probe_valu_rates(r.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))
    if rc != 0:
        raise DemapError(rc, "dm_probe_valu_rates failed")
    return {"exp2_per_s": r[0], "fma_per_s": r[1], "exp2_add2_per_s": r[2], "cus": int(r[3])}


def probe_atomic_rates(stream=None) -> dict:
    """Measured device-scope atomic rates on one address and over 64 (dm_probe_atomic_rates)."""
    r = np.zeros(3, dtype=np.float64)
    rc = load_library().dm_probe_atomic_rates(r.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream))
    if rc != 0:
        raise DemapError(rc, "dm_probe_atomic_rates failed")
    return {"one_address_per_s": r[0], "spread_per_s": r[1], "spread_addresses": int(r[2])}


def probe_gelu(x) -> np.ndarray:
    """The inference kernel's packed-FP16 GELU on host values x (dm_probe_gelu): FP16 results
    widened to FP32."""
    xs = np.ascontiguousarray(x, dtype=np.float32).ravel()
    out = np.empty_like(xs)
    rc = load_library().dm_probe_gelu(xs.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p),
                                      xs.size)
    if rc != 0:
        raise DemapError(rc, "dm_probe_gelu failed")
    return out.reshape(np.shape(x))


def profile_enable(on: bool = True):
    """Start (and clear) or stop HIP-event timing of the library's kernels on this thread."""
    _check(load_library().dm_profile_enable(1 if on else 0))


def profile_read(reset: bool = False):
    """(main_ms, fixup_ms, launches) summed over the recorded launches (dm_profile_read)."""
    a = ctypes.c_double()
    b = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load_library().dm_profile_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(n), 1 if reset else 0))
    return a.value, b.value, n.value


PLAN_AUTOTUNE, PLAN_FORCE_VALU, PLAN_FORCE_MFMA = 1, 2, 4


class _Instance(ctypes.Structure):
    _fields_ = [("c", ctypes.c_void_p), ("sigma2", ctypes.c_double), ("y", ctypes.c_void_p),
                ("tx", ctypes.c_void_p), ("N", ctypes.c_int64), ("llr", ctypes.c_void_p)]


def _instances(items):
    """items: sequence of (Constellation, sigma2, y, tx or None, llr or None) -> ctypes array."""
    arr = (_Instance * len(items))()
    for i, (c, s2, y, tx, llr) in enumerate(items):
        N = int(y.shape[0])
        arr[i].c = c.handle
        arr[i].sigma2 = float(s2)
        arr[i].y = _dev_tensor(y, ("float32",), (N, c.D), "y").value
        arr[i].tx = None if tx is None else _dev_tensor(tx, ("int16", "uint16"), (N,), "tx").value
        arr[i].N = N
        arr[i].llr = None if llr is None else _dev_tensor(llr, ("float32",), (N, c.m), "llr").value
    return arr


class Plan:
    """Batched plan over instances (Constellation, sigma2, y, tx, llr) — dm_plan_create.

    The plan keeps references to every tensor it was built with (their memory must stay valid).
    """

    def __init__(self, items, prec: str = "fp16x3", autotune: bool = True, force: str | None = None,
                 item_tiles: int | None = None, claim: int | None = None):
        """force: None / "valu" / "mfma" (kernel body); item_tiles: None or 1, 2, 4 (symbol tiles
        per work item); claim: None or 1, 2, 4, 8 (work items per claim).  With autotune the
        unforced parts of the shape are timed, else a fixed rule fills them."""
        self._items = list(items)
        flags = PLAN_AUTOTUNE if autotune else 0
        if force == "valu":
            flags |= PLAN_FORCE_VALU
        elif force == "mfma":
            flags |= PLAN_FORCE_MFMA
        if item_tiles is not None:
            flags |= {1: 1, 2: 2, 4: 3}[item_tiles] << 8
        if claim is not None:
            flags |= {1: 1, 2: 2, 4: 3, 8: 4}[claim] << 12
        self._arr = _instances(self._items)
        h = ctypes.c_void_p()
        _check(load_library().dm_plan_create(ctypes.cast(self._arr, ctypes.c_void_p), len(self._items), PREC[prec],
                                             flags, ctypes.byref(h)))
        self._h = h
        self.n = len(self._items)

    def launch(self, stream=None):
        _check(load_library().dm_plan_launch(self._h, _stream_handle(stream)))

    def results(self, stream=None):
        g = np.empty(self.n, dtype=np.float64)
        mi = np.empty(self.n, dtype=np.float64)
        fx = np.empty(self.n, dtype=np.int64)
        _check(load_library().dm_plan_results(self._h, g.ctypes.data_as(ctypes.c_void_p),
                                              mi.ctypes.data_as(ctypes.c_void_p), fx.ctypes.data_as(ctypes.c_void_p),
                                              _stream_handle(stream)))
        return g, mi, fx

    def info(self):
        """(kernel body per instance: 0 FP32 / 1 MFMA, ns per pair, symbols per work item)."""
        kinds = np.empty(self.n, dtype=np.int32)
        ns = np.empty(self.n, dtype=np.float64)
        sym = np.empty(self.n, dtype=np.int32)
        _check(load_library().dm_plan_info(self._h, kinds.ctypes.data_as(ctypes.c_void_p),
                                           ns.ctypes.data_as(ctypes.c_void_p), sym.ctypes.data_as(ctypes.c_void_p)))
        return kinds, ns, sym

    def stats(self):
        """(work items, items per claim, workgroups) of the plan's launch."""
        n = ctypes.c_int64()
        grab = ctypes.c_int32()
        grid = ctypes.c_int32()
        _check(load_library().dm_plan_stats(self._h, ctypes.byref(n), ctypes.byref(grab), ctypes.byref(grid)))
        return int(n.value), int(grab.value), int(grid.value)

    def work_items(self):
        return self.stats()[0]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().dm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def demap_batched(items, prec: str = "fp16x3", autotune: bool = False, stream=None):
    """One-shot batched GMI/MI (dm_demap_batched); returns (gmi, mi) NumPy arrays."""
    arr = _instances(list(items))
    n = len(arr)
    g = np.empty(n, dtype=np.float64)
    mi = np.empty(n, dtype=np.float64)
    _check(load_library().dm_demap_batched(ctypes.cast(arr, ctypes.c_void_p), n, PREC[prec],
                                           PLAN_AUTOTUNE if autotune else 0, g.ctypes.data_as(ctypes.c_void_p),
                                           mi.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)))
    return g, mi


def demap_llr_var(const: Constellation, sigma2, y, llr=None, prec: str = "fp32", stream=None):
    """Exact LLRs with one noise variance per symbol (sigma2: (N,) FP32 tensor) — dm_demap_llr_var."""
    import torch
    N = int(y.shape[0])
    yp = _dev_tensor(y, ("float32",), (N, const.D), "y")
    sp = _dev_tensor(sigma2, ("float32",), (N,), "sigma2")
    if llr is None:
        llr = torch.empty((N, const.m), dtype=torch.float32, device=y.device)
    lp = _dev_tensor(llr, ("float32",), (N, const.m), "llr")
    _check(load_library().dm_demap_llr_var(const.handle, sp, yp, N, lp, PREC[prec], _stream_handle(stream)))
    return llr


_MLP_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")
MLP_HIDDEN = 256

FALLBACK = {0: "learned", 1: "audit", 2: "snr_range", 3: "constellation"}


def mlp_param_count(D: int, m: int) -> int:
    n = int(load_library().dm_mlp_param_count(D, m))
    if n < 0:
        _check(n)
    return n


def _mlp_shapes(D: int, m: int):
    H = MLP_HIDDEN
    return {"W1": (D + 1, H), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H, m), "b3": (m,)}


def _flatten(w: dict, D: int, m: int) -> np.ndarray:
    parts = []
    for k, shp in _mlp_shapes(D, m).items():
        a = np.asarray(w[k], dtype=np.float32)
        if a.shape != shp:
            raise ValueError(f"{k} has shape {a.shape}, expected {shp}")
        parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def _unflatten(flat: np.ndarray, D: int, m: int) -> dict:
    out, o = {}, 0
    for k, shp in _mlp_shapes(D, m).items():
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp).copy()
        o += n
    return out


class _TrainConfig(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("epochs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("target_prec", ctypes.c_int32), ("snr_lo_db", ctypes.c_double),
                ("snr_hi_db", ctypes.c_double)]


class _LearnedOpts(ctypes.Structure):
    _fields_ = [("max_gmi_loss", ctypes.c_double), ("audit_log2", ctypes.c_int32), ("exact_prec", ctypes.c_int32)]


class MLP:
    """Learned demapper network bound to one constellation (dm_mlp_*).

    Weights are dicts of FP32 arrays W1 (D+1, 256), b1, W2 (256, 256), b2, W3 (256, m), b3 with
    out = x @ W + b.
    """

    def __init__(self, const: Constellation, weights: dict | None = None, _handle=None):
        self.D, self.m = const.D, const.m
        if _handle is not None:
            self._h = _handle
            return
        flat = _flatten(weights, self.D, self.m)
        h = ctypes.c_void_p()
        _check(load_library().dm_mlp_create(const.handle, flat.ctypes.data_as(ctypes.c_void_p), ctypes.byref(h)))
        self._h = h

    @classmethod
    def load(cls, const: Constellation, path: str) -> "MLP":
        h = ctypes.c_void_p()
        _check(load_library().dm_mlp_load(const.handle, str(path).encode(), ctypes.byref(h)))
        return cls(const, _handle=h)

    def save(self, path: str):
        _check(load_library().dm_mlp_save(self._h, str(path).encode()))

    def get_weights(self) -> dict:
        flat = np.empty(mlp_param_count(self.D, self.m), dtype=np.float32)
        _check(load_library().dm_mlp_get_weights(self._h, flat.ctypes.data_as(ctypes.c_void_p)))
        return _unflatten(flat, self.D, self.m)

    def set_weights(self, weights: dict):
        flat = _flatten(weights, self.D, self.m)
        _check(load_library().dm_mlp_set_weights(self._h, flat.ctypes.data_as(ctypes.c_void_p)))

    def info(self):
        st = ctypes.c_int64()
        lo = ctypes.c_double()
        hi = ctypes.c_double()
        _check(load_library().dm_mlp_info(self._h, ctypes.byref(st), ctypes.byref(lo), ctypes.byref(hi)))
        return {"steps": st.value, "snr_lo_db": lo.value, "snr_hi_db": hi.value}

    def train(self, const: Constellation, y, sigma2, batch: int = 4096, epochs: int = 1, lr: float = 1e-3,
              lr_final: float = 1e-5, target_prec: str = "fp32", snr_range=(0.0, 15.0), beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, stream=None) -> float:
        """Train on y (N x D) with per-sample noise variances sigma2 (N,) FP32; returns the final mean loss."""
        N = int(y.shape[0])
        yp = _dev_tensor(y, ("float32",), (N, self.D), "y")
        sp = _dev_tensor(sigma2, ("float32",), (N,), "sigma2")
        cfg = _TrainConfig(batch, epochs, lr, lr_final, beta1, beta2, eps, PREC[target_prec], float(snr_range[0]),
                           float(snr_range[1]))
        loss = ctypes.c_double()
        _check(load_library().dm_mlp_train(self._h, const.handle, ctypes.byref(cfg), yp, sp, N, ctypes.byref(loss),
                                           _stream_handle(stream)))
        return loss.value

    def gradients(self, y, sigma2, target, stream=None):
        """(gradients dict, loss) of one batch at the current weights (dm_mlp_gradients)."""
        B = int(y.shape[0])
        yp = _dev_tensor(y, ("float32",), (B, self.D), "y")
        sp = _dev_tensor(sigma2, ("float32",), (B,), "sigma2")
        tp = _dev_tensor(target, ("float32",), (B, self.m), "target")
        flat = np.empty(mlp_param_count(self.D, self.m), dtype=np.float32)
        loss = ctypes.c_double()
        _check(load_library().dm_mlp_gradients(self._h, yp, sp, tp, B, flat.ctypes.data_as(ctypes.c_void_p),
                                               ctypes.byref(loss), _stream_handle(stream)))
        return _unflatten(flat, self.D, self.m), loss.value

    def stats(self):
        """(work items, items per claim, workgroups) of the plan's launch."""
        n = ctypes.c_int64()
        grab = ctypes.c_int32()
        grid = ctypes.c_int32()
        _check(load_library().dm_plan_stats(self._h, ctypes.byref(n), ctypes.byref(grab), ctypes.byref(grid)))
        return int(n.value), int(grab.value), int(grid.value)

    def work_items(self):
        return self.stats()[0]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().dm_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def demap_learned(net: MLP, const: Constellation, sigma2: Sequence[float], ys, tx=None, llrs=None,
                  max_gmi_loss: float = 0.01, audit_log2: int = 6, exact_prec: str = "fp32", stream=None):
    """Learned demapping with exact audit / fallback (dm_demap_learned).

    Returns (gmi, gmi_loss, used_fallback) NumPy arrays; used_fallback codes are in FALLBACK.
    """
    s2 = np.ascontiguousarray(np.asarray(sigma2, dtype=np.float64).reshape(-1))
    ns = int(s2.shape[0])
    ylist = [ys[i] for i in range(ns)]
    N = int(ylist[0].shape[0])
    yptr = (ctypes.c_void_p * ns)(*[_dev_tensor(t, ("float32",), (N, const.D), "y[s]").value for t in ylist])
    txp = None if tx is None else _dev_tensor(tx, ("int16", "uint16"), (N,), "tx")
    lptr = None
    if llrs is not None:
        lptr = (ctypes.c_void_p * ns)(*[_dev_tensor(llrs[i], ("float32",), (N, const.m), "llr[s]").value
                                        for i in range(ns)])
    gmi = np.full(ns, np.nan)
    loss = np.full(ns, np.nan)
    fb = np.zeros(ns, dtype=np.int32)
    opts = _LearnedOpts(max_gmi_loss, audit_log2, PREC[exact_prec])
    _check(load_library().dm_demap_learned(
        net._h, const.handle, ns, s2.ctypes.data_as(ctypes.c_void_p), ctypes.cast(yptr, ctypes.c_void_p), txp, N,
        None if lptr is None else ctypes.cast(lptr, ctypes.c_void_p), ctypes.byref(opts),
        gmi.ctypes.data_as(ctypes.c_void_p), loss.ctypes.data_as(ctypes.c_void_p), fb.ctypes.data_as(ctypes.c_void_p),
        _stream_handle(stream)))
    return gmi, loss, fb


HARD_METHOD = {"auto": 0, "valu": 1, "mfma": 2}


def hard_decision(const: Constellation, ys, tx=None, labels=None, count: bool = True, method: str = "auto",
                  return_exact: bool = False, stream=None):
    """Minimum-distance decisions of n_blk received blocks (dm_hard_decision).

    ys: list of (N, D) FP32 tensors; tx: (N,) int16/uint16 rows (needed for counting);
    labels: None or a list of (N,) int16/uint16 tensors receiving the decided labels;
    method: "auto", "valu" or "mfma" (same decisions).
    Returns (symbol_errors, bit_errors) int64 NumPy arrays, or (None, None) without counting;
    with return_exact, also the number of symbols the MFMA method sent to the exact path.
    """
    nb = len(ys)
    N = int(ys[0].shape[0])
    yptr = (ctypes.c_void_p * nb)(*[_dev_tensor(t, ("float32",), (N, const.D), "y[s]").value for t in ys])
    txp = None if tx is None else _dev_tensor(tx, ("int16", "uint16"), (N,), "tx")
    lptr = None
    if labels is not None:
        lptr = (ctypes.c_void_p * nb)(*[_dev_tensor(t, ("int16", "uint16"), (N,), "labels[s]").value for t in labels])
    se = np.zeros(nb, dtype=np.int64) if count else None
    be = np.zeros(nb, dtype=np.int64) if count else None
    nx = ctypes.c_int64(0)
    _check(load_library().dm_hard_decision(
        const.handle, nb, ctypes.cast(yptr, ctypes.c_void_p), txp, N,
        None if lptr is None else ctypes.cast(lptr, ctypes.c_void_p),
        None if se is None else se.ctypes.data_as(ctypes.c_void_p),
        None if be is None else be.ctypes.data_as(ctypes.c_void_p), HARD_METHOD[method],
        ctypes.byref(nx) if return_exact else None, _stream_handle(stream)))
    return (se, be, int(nx.value)) if return_exact else (se, be)


def q_factor_db(ber: float) -> float:
    """20 log10(sqrt(2) erfcinv(2 BER)) (dm_q_factor_db); NaN outside 0 < BER < 0.5."""
    return float(load_library().dm_q_factor_db(float(ber)))


class _GsConfig(ctypes.Structure):
    _fields_ = [("snr_db", ctypes.c_double), ("iters", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("perturb_sd", ctypes.c_double), ("swap_prob", ctypes.c_double), ("seed", ctypes.c_uint64)]


def gs_optimize(points, labels, snr_db: float, tx, z, iters: int = 200, candidates: int = 32,
                perturb_sd: float = 0.05, swap_prob: float = 0.3, seed: int = 1, stream=None):
    """GMI-driven geometric-shaping search (dm_gs_optimize).

    tx: (N,) int16/uint16 tensor of transmitted LABELS; z: (N, D) FP32 unit-noise tensor.
    Returns (points (M, D) float32 in label order, labels = arange(M), gmi_trace (iters+1,), accepted).
    """
    pts = np.ascontiguousarray(points, dtype=np.float32)
    lab = np.ascontiguousarray(labels, dtype=np.uint16)
    M, D = pts.shape
    N = int(tx.shape[0])
    txp = _dev_tensor(tx, ("int16", "uint16"), (N,), "tx")
    zp = _dev_tensor(z, ("float32",), (N, D), "z")
    out = np.empty((M, D), dtype=np.float32)
    trace = np.empty(iters + 1, dtype=np.float64)
    acc = ctypes.c_int32()
    cfg = _GsConfig(float(snr_db), int(iters), int(candidates), float(perturb_sd), float(swap_prob), int(seed))
    _check(load_library().dm_gs_optimize(pts.ctypes.data_as(ctypes.c_void_p), lab.ctypes.data_as(ctypes.c_void_p),
                                         M, D, ctypes.byref(cfg), txp, zp, N, out.ctypes.data_as(ctypes.c_void_p),
                                         trace.ctypes.data_as(ctypes.c_void_p), ctypes.byref(acc),
                                         _stream_handle(stream)))
    return out, np.arange(M, dtype=np.uint16), trace, int(acc.value)


class Streamer:
    """Streamed demapping of host arrays in fixed-size buffers (dm_streamer_*)."""

    def __init__(self, const: Constellation, buffer_symbols: int = 1 << 20, n_buffers: int = 3, prec: str = "fp32"):
        self.D, self.m = const.D, const.m
        self._const = const
        h = ctypes.c_void_p()
        _check(load_library().dm_streamer_create(const.handle, int(buffer_symbols), int(n_buffers), PREC[prec],
                                                 ctypes.byref(h)))
        self._h = h

    def run(self, sigma2: float, y, llr=None):
        """Demap host y (N, D) FP32 into host llr (N, m) FP32; returns (llr, seconds).

        y / llr may be NumPy arrays or CPU torch tensors (pinned tensors are transferred directly).
        """
        import torch
        if isinstance(y, torch.Tensor) or isinstance(llr, torch.Tensor):
            N = int(y.shape[0])
            if llr is None:
                llr = torch.empty((N, self.m), dtype=torch.float32, pin_memory=y.is_pinned())
            for t, shp, nm in ((y, (N, self.D), "y"), (llr, (N, self.m), "llr")):
                if t.is_cuda or t.dtype != torch.float32 or tuple(t.shape) != shp or not t.is_contiguous():
                    raise ValueError(f"{nm} must be a contiguous float32 CPU tensor of shape {shp}")
            sec = ctypes.c_double()
            _check(load_library().dm_streamer_run(self._h, float(sigma2), ctypes.c_void_p(y.data_ptr()), N,
                                                  ctypes.c_void_p(llr.data_ptr()), ctypes.byref(sec)))
            return llr, sec.value
        y = np.ascontiguousarray(y, dtype=np.float32)
        N = int(y.shape[0])
        if y.shape != (N, self.D):
            raise ValueError("y must be N x D")
        if llr is None:
            llr = np.empty((N, self.m), dtype=np.float32)
        if llr.shape != (N, self.m) or llr.dtype != np.float32 or not llr.flags["C_CONTIGUOUS"]:
            raise ValueError("llr must be a C-contiguous float32 N x m array")
        sec = ctypes.c_double()
        _check(load_library().dm_streamer_run(self._h, float(sigma2), y.ctypes.data_as(ctypes.c_void_p), N,
                                              llr.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sec)))
        return llr, sec.value

    def stats(self):
        """(work items, items per claim, workgroups) of the plan's launch."""
        n = ctypes.c_int64()
        grab = ctypes.c_int32()
        grid = ctypes.c_int32()
        _check(load_library().dm_plan_stats(self._h, ctypes.byref(n), ctypes.byref(grab), ctypes.byref(grid)))
        return int(n.value), int(grab.value), int(grid.value)

    def work_items(self):
        return self.stats()[0]

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().dm_streamer_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
