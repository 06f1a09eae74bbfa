"""Python binding of the ERX gfx950 library (include/erx.h).

Argument marshalling only: every step of the detector runs in the HIP kernels
of liberx.so.  PyTorch is used for device memory and streams.  There is no
fallback: if the library is missing or cannot be loaded, every entry point
raises ErxError.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liberx.so")

ERX_OK, ERX_EINVAL, ERX_ENOMEM, ERX_EDEVICE, ERX_ENOTPD, ERX_ESTATE = 0, -1, -2, -3, -4, -5
DTYPES = {"f32": 0, "f16": 1, "u16": 2}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2, "split16": 3}
SCORE_ARITH = {"split16": 0, "fp32": 1}
BACKGROUNDS = {"ema": 0, "imc": 1}
FLAG_NEED_FP64, FLAG_FP64_DONE, FLAG_NOTPD, FLAG_SCORE32 = 1, 2, 4, 8
MAX_BANDS = 304

# every entry point declared in include/erx.h
EXPORTS = (
    "erx_config_default", "erx_create", "erx_create_ex", "erx_set_stream", "erx_push_lines",
    "erx_push_lines_ex", "erx_scores", "erx_scores_device", "erx_scores_normalised", "erx_labels",
    "erx_get_state", "erx_set_state", "erx_stats", "erx_line_info", "erx_profile_enable",
    "erx_profile_read", "erx_batch_create", "erx_batch_set_stream", "erx_batch_push",
    "erx_batch_scores", "erx_batch_get_state", "erx_batch_stats", "erx_batch_use_graphs", "erx_batch_small_path",
    "erx_batch_synchronize", "erx_batch_destroy", "erx_synchronize", "erx_destroy", "erx_last_error",
    "erx_surrogate_create", "erx_surrogate_num_params", "erx_surrogate_set_params",
    "erx_surrogate_get_params", "erx_surrogate_scores", "erx_surrogate_train_step",
    "erx_surrogate_grads", "erx_surrogate_destroy", "erx_surrogate_detector_create",
    "erx_surrogate_detector_push", "erx_surrogate_detector_scores", "erx_surrogate_detector_status",
    "erx_surrogate_detector_drift_stats", "erx_surrogate_detector_destroy", "erx_autotune", "erx_tune_lookup", "erx_push_lines_noalloc",
    "erx_detection_metrics", "erx_srp_matrix", "erx_rxb_create", "erx_rxb_push", "erx_rxb_scores",
    "erx_rxb_destroy",
)
SURR_K, SURR_HIDDEN = 16, 64


class ErxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Config(C.Structure):
    _fields_ = [("bands", C.c_int), ("pixels", C.c_int), ("momentum", C.c_float),
                ("ridge", C.c_float), ("warmup", C.c_int), ("dtype", C.c_int),
                ("precision", C.c_int), ("fp64_cond_threshold", C.c_double),
                ("normalise", C.c_int), ("block_lines", C.c_int), ("scan_lines", C.c_int),
                ("cond_estimate", C.c_int), ("score_arith", C.c_int), ("srp_dims", C.c_int),
                ("srp_seed", C.c_ulonglong), ("background", C.c_int), ("state_fp32", C.c_int),
                ("score_tiles", C.c_int), ("gram_macro", C.c_int)]


class DetectionMetrics(C.Structure):
    _fields_ = [("auc", C.c_double), ("auc_tpr_tau", C.c_double), ("auc_fpr_tau", C.c_double),
                ("auc_td", C.c_double), ("auc_bs", C.c_double), ("positives", C.c_longlong),
                ("negatives", C.c_longlong), ("excluded", C.c_longlong)]


class TuneResult(C.Structure):
    _fields_ = [("block_lines", C.c_int), ("scan_lines", C.c_int), ("small_path", C.c_int),
                ("candidates", C.c_int), ("us_per_line", C.c_double), ("score_tiles", C.c_int),
                ("gram_macro", C.c_int)]


class KernelTime(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_longlong), ("total_ms", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("lines", C.c_longlong), ("fp64_refactors", C.c_longlong),
                ("notpd", C.c_longlong), ("max_cond", C.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load liberx.so and declare its signatures (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ErxError(ERX_EDEVICE, f"{path} is not built; run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, ip = C.c_void_p, C.c_int
    sig = {
        "erx_config_default": (None, [C.POINTER(Config), ip, ip, C.c_float]),
        "erx_create": (vp, [ip, ip, C.c_float]),
        "erx_create_ex": (vp, [C.POINTER(Config)]),
        "erx_set_stream": (ip, [vp, vp]),
        "erx_push_lines": (ip, [vp, vp, ip]),
        "erx_push_lines_ex": (ip, [vp, vp, ip]),
        "erx_scores": (ip, [vp, vp]),
        "erx_scores_device": (ip, [vp, vp]),
        "erx_scores_normalised": (ip, [vp, vp]),
        "erx_labels": (ip, [vp, C.c_float, vp]),
        "erx_get_state": (ip, [vp, C.POINTER(C.c_longlong), vp, vp]),
        "erx_set_state": (ip, [vp, C.c_longlong, vp, vp]),
        "erx_stats": (ip, [vp, C.POINTER(Stats)]),
        "erx_line_info": (ip, [vp, vp, vp]),
        "erx_profile_enable": (ip, [vp, ip]),
        "erx_profile_read": (ip, [vp, C.POINTER(KernelTime), ip]),
        "erx_batch_create": (vp, [ip, vp, vp, vp, C.POINTER(Config)]),
        "erx_batch_set_stream": (ip, [vp, vp]),
        "erx_batch_push": (ip, [vp, vp, vp]),
        "erx_batch_scores": (ip, [vp, vp]),
        "erx_batch_get_state": (ip, [vp, ip, C.POINTER(C.c_longlong), vp, vp]),
        "erx_batch_stats": (ip, [vp, C.POINTER(Stats)]),
        "erx_batch_use_graphs": (ip, [vp, ip]),
        "erx_batch_small_path": (ip, [vp, ip]),
        "erx_batch_synchronize": (ip, [vp]),
        "erx_batch_destroy": (None, [vp]),
        "erx_synchronize": (ip, [vp]),
        "erx_destroy": (None, [vp]),
        "erx_last_error": (C.c_char_p, []),
        "erx_surrogate_create": (vp, [ip, C.c_ulonglong]),
        "erx_surrogate_num_params": (ip, [vp]),
        "erx_surrogate_set_params": (ip, [vp, vp]),
        "erx_surrogate_get_params": (ip, [vp, vp]),
        "erx_surrogate_scores": (ip, [vp, vp, ip, ip, C.c_float, vp]),
        "erx_surrogate_train_step": (ip, [vp, vp, vp, ip, ip, C.c_float, C.c_float, C.POINTER(C.c_float)]),
        "erx_surrogate_grads": (ip, [vp, vp]),
        "erx_surrogate_destroy": (None, [vp]),
        "erx_surrogate_detector_create": (vp, [vp, ip, C.c_float, C.c_float, ip]),
        "erx_surrogate_detector_push": (ip, [vp, vp, ip]),
        "erx_surrogate_detector_scores": (ip, [vp, vp]),
        "erx_surrogate_detector_status": (ip, [vp, C.POINTER(C.c_int), C.POINTER(C.c_longlong),
                                                C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]),
        "erx_surrogate_detector_drift_stats": (ip, [vp, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                                    C.POINTER(C.c_float)]),
        "erx_surrogate_detector_destroy": (None, [vp]),
        "erx_autotune": (ip, [C.POINTER(Config), ip, C.c_char_p, C.POINTER(TuneResult)]),
        "erx_tune_lookup": (ip, [C.POINTER(Config), ip, C.c_char_p, C.POINTER(TuneResult)]),
        "erx_push_lines_noalloc": (ip, [C.POINTER(Config), vp, C.c_longlong, vp, ip, vp, vp]),
        "erx_detection_metrics": (ip, [vp, vp, C.c_longlong, vp, C.POINTER(DetectionMetrics)]),
        "erx_srp_matrix": (ip, [ip, ip, C.c_ulonglong, vp]),
        "erx_rxb_create": (vp, [C.POINTER(Config), ip]),
        "erx_rxb_push": (ip, [vp, vp, ip]),
        "erx_rxb_scores": (ip, [vp, vp, C.POINTER(C.c_longlong), C.POINTER(C.c_int)]),
        "erx_rxb_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().erx_last_error().decode()


def _check(rc: int, allow=()):
    if rc != ERX_OK and rc not in allow:
        raise ErxError(rc, last_error())
    return rc


def _ptr(x) -> int:
    """Data pointer of a contiguous torch tensor or numpy array."""
    if hasattr(x, "data_ptr"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    raise TypeError(type(x))


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return None


class Detector:
    """One ERX stream on the current GPU (a handle of the C library)."""

    def __init__(self, bands: int, pixels: int, momentum: float = 0.1, ridge: float = 1e-5,
                 dtype: str = "f32", precision: str = "split16", fp64_cond_threshold: float = 0.0,
                 normalise: bool = False, warmup: int = 0, block_lines: int = 2048,
                 scan_lines: int = 64, cond_estimate: int = -1, stream: Optional[int] = -1,
                 score_arith: str = "split16", srp_dims: int = 0, srp_seed: int = 0,
                 background: str = "ema", state_fp32: bool = False, score_tiles: int = 0,
                 gram_macro: int = 0):
        """stream: hipStream_t handle to run on; -1 (default) = torch's current
        stream, None = a stream owned by the handle.  srp_dims > 0: project every line
        to that many dimensions first (Sec. III-B, weights from srp_matrix).
        state_fp32: keep the moving-average state and per-line statistics in FP32."""
        lib = load()
        cfg = Config()
        lib.erx_config_default(C.byref(cfg), int(bands), int(pixels), float(momentum))
        cfg.ridge = float(ridge)
        cfg.dtype = DTYPES[dtype]
        cfg.precision = PRECISIONS[precision]
        cfg.fp64_cond_threshold = float(fp64_cond_threshold)
        cfg.normalise = 1 if normalise else 0
        cfg.warmup = int(warmup)
        cfg.block_lines = int(block_lines)
        cfg.scan_lines = int(scan_lines)
        cfg.cond_estimate = int(cond_estimate)
        cfg.score_arith = SCORE_ARITH[score_arith]
        cfg.srp_dims = int(srp_dims)
        cfg.srp_seed = int(srp_seed)
        cfg.background = BACKGROUNDS[background]
        cfg.state_fp32 = 1 if state_fp32 else 0
        cfg.score_tiles = int(score_tiles)
        cfg.gram_macro = int(gram_macro)
        self.cfg = cfg
        self.bands, self.pixels, self.dtype = int(bands), int(pixels), dtype
        self.work_bands = int(srp_dims) if srp_dims else int(bands)
        self._lib = lib
        self._h = lib.erx_create_ex(C.byref(cfg))
        if not self._h:
            raise ErxError(ERX_EINVAL, last_error())
        self.last_n = 0
        if stream == -1:
            stream = _torch_stream()
        if stream is not None:
            _check(lib.erx_set_stream(self._h, C.c_void_p(stream)))

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            self._lib.erx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    # -- work
    def push(self, lines) -> "Detector":
        """Absorb and score lines [n, pixels, bands] (torch tensor or numpy array)."""
        shape = tuple(lines.shape)
        if len(shape) == 2:
            shape = (1,) + shape
        if shape[1:] != (self.pixels, self.bands):
            raise ValueError(f"lines must be [n, {self.pixels}, {self.bands}], got {tuple(lines.shape)}")
        _check(self._lib.erx_push_lines_ex(self._h, C.c_void_p(_ptr(lines)), int(shape[0])))
        self.last_n = int(shape[0])
        return self

    def scores(self, out=None, allow_notpd: bool = True):
        """Scores of the last push as a [n, pixels] float32 torch tensor on the GPU."""
        import torch
        if out is None:
            out = torch.empty((self.last_n, self.pixels), dtype=torch.float32, device="cuda")
        _check(self._lib.erx_scores_device(self._h, C.c_void_p(_ptr(out))))
        return out

    def scores_host(self, allow_notpd: bool = True) -> np.ndarray:
        out = np.empty((self.last_n, self.pixels), np.float32)
        _check(self._lib.erx_scores(self._h, C.c_void_p(out.ctypes.data)),
               allow=(ERX_ENOTPD,) if allow_notpd else ())
        return out

    def scores_normalised(self, allow_notpd: bool = True) -> np.ndarray:
        out = np.empty((self.last_n, self.pixels), np.float32)
        _check(self._lib.erx_scores_normalised(self._h, C.c_void_p(out.ctypes.data)),
               allow=(ERX_ENOTPD,) if allow_notpd else ())
        return out

    def labels(self, tau: float) -> np.ndarray:
        out = np.empty((self.last_n, self.pixels), np.uint8)
        _check(self._lib.erx_labels(self._h, C.c_float(tau), C.c_void_p(out.ctypes.data)))
        return out

    def synchronize(self):
        _check(self._lib.erx_synchronize(self._h))

    # -- state and diagnostics
    def state(self):
        t = C.c_longlong(0)
        mu = np.empty(self.work_bands)
        K = np.empty((self.work_bands, self.work_bands))
        _check(self._lib.erx_get_state(self._h, C.byref(t), C.c_void_p(mu.ctypes.data),
                                       C.c_void_p(K.ctypes.data)))
        return int(t.value), mu, K

    def set_state(self, t: int, mu=None, K=None):
        mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
        K = None if K is None else np.ascontiguousarray(K, dtype=np.float64)
        _check(self._lib.erx_set_state(self._h, int(t),
                                       None if mu is None else C.c_void_p(mu.ctypes.data),
                                       None if K is None else C.c_void_p(K.ctypes.data)))

    def stats(self) -> dict:
        s = Stats()
        _check(self._lib.erx_stats(self._h, C.byref(s)))
        return dict(lines=s.lines, fp64_refactors=s.fp64_refactors, notpd=s.notpd,
                    max_cond=s.max_cond)

    def profile(self, on: bool = True):
        """Bracket every kernel launch with HIP events on the handle's stream."""
        _check(self._lib.erx_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel: (launches, total_ms)} since the last read (waits for the stream)."""
        buf = (KernelTime * 16)()
        k = self._lib.erx_profile_read(self._h, buf, 16)
        if k < 0:
            raise ErxError(k, last_error())
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(k)}

    def line_info(self):
        cond = np.empty(self.last_n, np.float32)
        flags = np.empty(self.last_n, np.int32)
        _check(self._lib.erx_line_info(self._h, C.c_void_p(cond.ctypes.data),
                                       C.c_void_p(flags.ctypes.data)))
        return cond, flags


class Batch:
    """Many independent streams (one detector each) processed in shared device passes."""

    def __init__(self, bands, pixels, momentum, ridge: float = 1e-5, dtype: str = "f32",
                 precision: str = "split16",
                 fp64_cond_threshold: float = 0.0, normalise: bool = False, block_lines: int = 8192,
                 scan_lines: int = 64, cond_estimate: int = -1, graphs: bool = True, score_arith: str = "split16",
                 stream: Optional[int] = -1, small_path: int = -1, state_fp32: bool = False,
                 score_tiles: int = 0, gram_macro: int = 0):
        lib = load()
        self.bands = [int(x) for x in bands]
        self.pixels = [int(x) for x in pixels]
        ns = len(self.bands)
        if len(self.pixels) != ns or len(momentum) != ns:
            raise ValueError("bands, pixels and momentum need one entry per stream")
        cfg = Config()
        lib.erx_config_default(C.byref(cfg), 1, 2, 0.1)
        cfg.ridge = float(ridge)
        cfg.dtype = DTYPES[dtype]
        cfg.precision = PRECISIONS[precision]
        cfg.fp64_cond_threshold = float(fp64_cond_threshold)
        cfg.normalise = 1 if normalise else 0
        cfg.block_lines = int(block_lines)
        cfg.scan_lines = int(scan_lines)
        cfg.cond_estimate = int(cond_estimate)
        cfg.score_arith = SCORE_ARITH[score_arith]
        cfg.state_fp32 = 1 if state_fp32 else 0
        cfg.score_tiles = int(score_tiles)
        cfg.gram_macro = int(gram_macro)
        b = (C.c_int * ns)(*self.bands)
        p = (C.c_int * ns)(*self.pixels)
        m = (C.c_float * ns)(*[float(x) for x in momentum])
        self._lib = lib
        self._h = lib.erx_batch_create(ns, b, p, m, C.byref(cfg))
        if not self._h:
            raise ErxError(ERX_EINVAL, last_error())
        self.nstreams = ns
        self.dtype = dtype
        self.last_n = [0] * ns
        if stream == -1:
            stream = _torch_stream()
        if stream is not None:
            _check(lib.erx_batch_set_stream(self._h, C.c_void_p(stream)))
        _check(lib.erx_batch_use_graphs(self._h, 1 if graphs else 0))
        _check(lib.erx_batch_small_path(self._h, int(small_path)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.erx_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, lines):
        """lines[s]: device tensor [n_s, pixels_s, bands_s] or None (no lines)."""
        ns = self.nstreams
        ptrs = (C.c_void_p * ns)()
        cnt = (C.c_int * ns)()
        for s, x in enumerate(lines):
            if x is None or x.shape[0] == 0:
                ptrs[s], cnt[s] = None, 0
                continue
            if tuple(x.shape[1:]) != (self.pixels[s], self.bands[s]):
                raise ValueError(f"stream {s}: lines must be [n, {self.pixels[s]}, {self.bands[s]}]")
            ptrs[s], cnt[s] = _ptr(x), int(x.shape[0])
        _check(self._lib.erx_batch_push(self._h, ptrs, cnt))
        self.last_n = [int(cnt[s]) for s in range(ns)]

    def scores(self, allow_notpd: bool = True, streams=None):
        """Scores of the last push: one float32 CUDA tensor [n_s, pixels_s] per stream (None if 0,
        or if streams is given and does not list s)."""
        import torch
        want = None if streams is None else set(int(s) for s in streams)
        outs = [torch.empty((n, p), dtype=torch.float32, device="cuda") if n and (want is None or s in want) else None
                for s, (n, p) in enumerate(zip(self.last_n, self.pixels))]
        arr = (C.c_void_p * self.nstreams)(*[(o.data_ptr() if o is not None else None) for o in outs])
        torch.cuda.synchronize()
        _check(self._lib.erx_batch_scores(self._h, arr), allow=(ERX_ENOTPD,) if allow_notpd else ())
        return outs

    def state(self, s: int):
        t = C.c_longlong(0)
        b = self.bands[s]
        mu = np.empty(b)
        K = np.empty((b, b))
        _check(self._lib.erx_batch_get_state(self._h, int(s), C.byref(t), C.c_void_p(mu.ctypes.data),
                                             C.c_void_p(K.ctypes.data)))
        return int(t.value), mu, K

    def stats(self) -> dict:
        st = Stats()
        _check(self._lib.erx_batch_stats(self._h, C.byref(st)))
        return dict(lines=st.lines, fp64_refactors=st.fp64_refactors, notpd=st.notpd,
                    max_cond=st.max_cond)

    def use_graphs(self, on: bool):
        _check(self._lib.erx_batch_use_graphs(self._h, 1 if on else 0))

    def synchronize(self):
        _check(self._lib.erx_batch_synchronize(self._h))


NOALLOC_SCRATCH_BYTES = 48 << 20


def noalloc_state_entries(bands: int) -> int:
    """Doubles of the caller-owned stream state of push_lines_noalloc."""
    nt = (int(bands) + 15) // 16
    return 256 * nt * (nt + 1) // 2 + 16 * nt


def push_lines_noalloc(lines, out, state, t0: int, momentum: float = 0.1, ridge: float = 1e-5,
                       dtype: str = "f32", precision: str = "split16", fp64_cond_threshold: float = 0.0,
                       block_lines: int = 2048, scan_lines: int = 64, cond_estimate: int = -1,
                       stream: Optional[int] = -1, score_arith: str = "split16") -> int:
    """erx_push_lines_noalloc: score lines [n, pixels, bands] (device tensor) into out
    [n, pixels] (device float32) with the caller-owned FP64 state (device tensor of
    noalloc_state_entries(bands) doubles); t0 = lines the stream absorbed before.
    Returns t0 + n.  stream: hipStream_t, -1 = torch's current stream."""
    lib = load()
    n, p, b = (int(v) for v in lines.shape)
    cfg = Config()
    lib.erx_config_default(C.byref(cfg), b, p, float(momentum))
    cfg.ridge = float(ridge)
    cfg.dtype = DTYPES[dtype]
    cfg.precision = PRECISIONS[precision]
    cfg.fp64_cond_threshold = float(fp64_cond_threshold)
    cfg.block_lines = int(block_lines)
    cfg.scan_lines = int(scan_lines)
    cfg.cond_estimate = int(cond_estimate)
    cfg.score_arith = SCORE_ARITH[score_arith]
    if stream == -1:
        stream = _torch_stream()
    _check(lib.erx_push_lines_noalloc(C.byref(cfg), C.c_void_p(_ptr(state)), int(t0), C.c_void_p(_ptr(lines)),
                                      n, C.c_void_p(_ptr(out)), C.c_void_p(stream)))
    return int(t0) + n


class RXBaseline:
    """RX Baseline (rolling window of `window` lines scoring its centre line) on the GPU."""

    def __init__(self, bands: int, pixels: int, window: int = 99, ridge: float = 0.0, dtype: str = "f32",
                 precision: str = "split16", fp64_cond_threshold: float = 0.0, block_lines: int = 2048,
                 scan_lines: int = 64, score_arith: str = "split16"):
        lib = load()
        cfg = Config()
        lib.erx_config_default(C.byref(cfg), int(bands), int(pixels), 0.1)
        cfg.ridge = float(ridge)
        cfg.dtype = DTYPES[dtype]
        cfg.precision = PRECISIONS[precision]
        cfg.fp64_cond_threshold = float(fp64_cond_threshold)
        cfg.block_lines = int(block_lines)
        cfg.scan_lines = int(scan_lines)
        cfg.score_arith = SCORE_ARITH[score_arith]
        self._lib = lib
        self.pixels = int(pixels)
        self._h = lib.erx_rxb_create(C.byref(cfg), int(window))
        if not self._h:
            raise ErxError(ERX_EINVAL, last_error())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.erx_rxb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, lines):
        _check(self._lib.erx_rxb_push(self._h, C.c_void_p(_ptr(lines)), int(lines.shape[0])))
        return self

    def scores(self):
        """(first scored stream line, float32 array [m, pixels]) of the last push."""
        first, m = C.c_longlong(0), C.c_int(0)
        _check(self._lib.erx_rxb_scores(self._h, None, C.byref(first), C.byref(m)))
        out = np.empty((m.value, self.pixels), np.float32)
        if m.value:
            _check(self._lib.erx_rxb_scores(self._h, C.c_void_p(out.ctypes.data), C.byref(first), C.byref(m)))
        return int(first.value), out


def srp_matrix(bands: int, dims: int, seed: int) -> np.ndarray:
    """erx_srp_matrix: the projection weights W [bands][dims] a detector with srp_dims =
    dims and srp_seed = seed uses (host computation, no GPU needed)."""
    W = np.empty((int(bands), int(dims)), np.float32)
    _check(load().erx_srp_matrix(int(bands), int(dims), C.c_ulonglong(int(seed)), C.c_void_p(W.ctypes.data)))
    return W


def detection_metrics(scores, truth, stream: Optional[int] = -1) -> dict:
    """erx_detection_metrics on device tensors: scores (float32) and truth (uint8 / bool,
    non-zero = anomaly) of the same number of pixels."""
    lib = load()
    n = int(scores.numel())
    if int(truth.numel()) != n:
        raise ValueError("scores and truth need the same number of elements")
    if truth.dtype != __import__("torch").uint8:
        truth = truth.to(__import__("torch").uint8)
    truth = truth.contiguous()
    if stream == -1:
        stream = _torch_stream()
    m = DetectionMetrics()
    _check(lib.erx_detection_metrics(C.c_void_p(_ptr(scores.contiguous())), C.c_void_p(_ptr(truth)), n,
                                     C.c_void_p(stream), C.byref(m)))
    return {k: getattr(m, k) for k, _ in DetectionMetrics._fields_}


__all__ = ["Detector", "Batch", "RXBaseline", "detection_metrics", "srp_matrix", "ErxError", "load", "last_error", "EXPORTS", "DTYPES", "PRECISIONS",
           "FLAG_NEED_FP64", "FLAG_FP64_DONE", "FLAG_NOTPD", "FLAG_SCORE32", "MAX_BANDS", "SCORE_ARITH", "push_lines_noalloc",
           "noalloc_state_entries", "NOALLOC_SCRATCH_BYTES"]


# ---------------------------------------------------------------------------
# learned projection surrogate
# ---------------------------------------------------------------------------
PARAM_ORDER = ("W", "c", "A1", "a1", "w2", "c2")


def _tune_config(bands, pixels, momentum, dtype, precision, fp64_cond_threshold, normalise,
                 score_arith="split16", state_fp32=False):
    cfg = Config()
    load().erx_config_default(C.byref(cfg), int(bands), int(pixels), float(momentum))
    cfg.dtype = DTYPES[dtype]
    cfg.precision = PRECISIONS[precision]
    cfg.fp64_cond_threshold = float(fp64_cond_threshold)
    cfg.normalise = 1 if normalise else 0
    cfg.score_arith = SCORE_ARITH[score_arith]
    cfg.state_fp32 = 1 if state_fp32 else 0
    return cfg


def _tune_dict(r):
    return {"block_lines": r.block_lines, "scan_lines": r.scan_lines, "small_path": r.small_path,
            "score_tiles": r.score_tiles, "gram_macro": r.gram_macro, "candidates": r.candidates,
            "us_per_line": r.us_per_line}


def autotune(bands: int, pixels: int, momentum: float = 0.1, dtype: str = "f32", precision: str = "split16",
             fp64_cond_threshold: float = 0.0, normalise: bool = False, nstreams: int = 1,
             cache: Optional[str] = None, score_arith: str = "split16", state_fp32: bool = False) -> dict:
    """Fastest launch setting for a workload shape (erx_autotune): block_lines, scan_lines,
    small_path (batch mode, -1 for one stream), score_tiles (the score kernel's tile shape),
    gram_macro (the split-FP16 Gram's macro tile),
    candidates timed, us_per_line."""
    lib = load()
    cfg = _tune_config(bands, pixels, momentum, dtype, precision, fp64_cond_threshold, normalise, score_arith,
                       state_fp32)
    r = TuneResult()
    _check(lib.erx_autotune(C.byref(cfg), int(nstreams), cache.encode() if cache else None, C.byref(r)))
    return _tune_dict(r)


def tune_lookup(bands: int, pixels: int, cache: str, momentum: float = 0.1, dtype: str = "f32",
                precision: str = "split16", fp64_cond_threshold: float = 0.0, normalise: bool = False,
                nstreams: int = 1, score_arith: str = "split16", state_fp32: bool = False) -> Optional[dict]:
    """Cached setting for a workload shape (erx_tune_lookup), or None when the cache has none."""
    lib = load()
    cfg = _tune_config(bands, pixels, momentum, dtype, precision, fp64_cond_threshold, normalise, score_arith,
                       state_fp32)
    r = TuneResult()
    rc = _check(lib.erx_tune_lookup(C.byref(cfg), int(nstreams), cache.encode(), C.byref(r)), allow=(ERX_ESTATE,))
    return None if rc == ERX_ESTATE else _tune_dict(r)


def _param_shapes(bands):
    return {"W": (SURR_K, bands), "c": (SURR_K,), "A1": (SURR_HIDDEN, SURR_K), "a1": (SURR_HIDDEN,),
            "w2": (SURR_HIDDEN,), "c2": (1,)}


class Surrogate:
    """Learned band projection + small network (a handle of the C library)."""

    def __init__(self, bands: int, seed: int = 0):
        lib = load()
        self._lib = lib
        self.bands = int(bands)
        self._h = lib.erx_surrogate_create(self.bands, C.c_ulonglong(seed))
        if not self._h:
            raise ErxError(ERX_EINVAL, last_error())
        self.nparams = lib.erx_surrogate_num_params(self._h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.erx_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _unflat(self, flat):
        out, k = {}, 0
        for name in PARAM_ORDER:
            shp = _param_shapes(self.bands)[name]
            n = int(np.prod(shp))
            out[name] = flat[k:k + n].reshape(shp).copy()
            k += n
        return out

    def params(self) -> dict:
        flat = np.empty(self.nparams, np.float32)
        _check(self._lib.erx_surrogate_get_params(self._h, C.c_void_p(flat.ctypes.data)))
        return self._unflat(flat)

    def set_params(self, params: dict):
        flat = np.concatenate([np.asarray(params[n], np.float32).reshape(-1) for n in PARAM_ORDER])
        if flat.size != self.nparams:
            raise ValueError("parameter sizes do not match the band count")
        flat = np.ascontiguousarray(flat)
        _check(self._lib.erx_surrogate_set_params(self._h, C.c_void_p(flat.ctypes.data)))

    def grads(self) -> dict:
        flat = np.empty(self.nparams, np.float32)
        _check(self._lib.erx_surrogate_grads(self._h, C.c_void_p(flat.ctypes.data)))
        return self._unflat(flat)

    def scores(self, lines, momentum: float):
        """Scores of lines [n, pixels, bands] (float32 CUDA tensor) of a stream from its first line."""
        import torch
        n, p, b = lines.shape
        out = torch.empty((n, p), dtype=torch.float32, device=lines.device)
        torch.cuda.synchronize()
        _check(self._lib.erx_surrogate_scores(self._h, C.c_void_p(_ptr(lines)), n, p, C.c_float(momentum),
                                              C.c_void_p(out.data_ptr())))
        return out

    def train_step(self, lines, targets, momentum: float, lr: float) -> float:
        import torch
        n, p, b = lines.shape
        loss = C.c_float()
        torch.cuda.synchronize()
        _check(self._lib.erx_surrogate_train_step(self._h, C.c_void_p(_ptr(lines)), C.c_void_p(_ptr(targets)), n, p,
                                                  C.c_float(momentum), C.c_float(lr), C.byref(loss)))
        return float(loss.value)


class SurrogateDetector:
    """A stream scored by a Surrogate, checked against plain ERX every check_every lines."""

    def __init__(self, net: Surrogate, pixels: int, momentum: float, drift_threshold: float = 0.05,
                 check_every: int = 32):
        self._lib = net._lib
        self.net = net  # keeps the network alive
        self.pixels = int(pixels)
        self._h = self._lib.erx_surrogate_detector_create(net._h, self.pixels, C.c_float(momentum),
                                                          C.c_float(drift_threshold), int(check_every))
        if not self._h:
            raise ErxError(ERX_EINVAL, last_error())
        self.last_n = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.erx_surrogate_detector_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, lines):
        import torch
        torch.cuda.synchronize()
        _check(self._lib.erx_surrogate_detector_push(self._h, C.c_void_p(_ptr(lines)), int(lines.shape[0])))
        self.last_n = int(lines.shape[0])
        return self

    def scores(self):
        import torch
        out = torch.empty((self.last_n, self.pixels), dtype=torch.float32, device="cuda")
        _check(self._lib.erx_surrogate_detector_scores(self._h, C.c_void_p(out.data_ptr())))
        return out

    def drift_stats(self) -> dict:
        """Drift of the last check and the mean / largest drift over the checks so far."""
        last, mean, mx = C.c_float(), C.c_float(), C.c_float()
        _check(self._lib.erx_surrogate_detector_drift_stats(self._h, C.byref(last), C.byref(mean), C.byref(mx)))
        return dict(last=last.value, mean=mean.value, max=mx.value)

    def status(self) -> dict:
        a = C.c_int()
        ch, dr, sw = C.c_longlong(), C.c_longlong(), C.c_longlong()
        _check(self._lib.erx_surrogate_detector_status(self._h, C.byref(a), C.byref(ch), C.byref(dr), C.byref(sw)))
        return {"active": bool(a.value), "checks": ch.value, "drifts": dr.value, "switched_at": sw.value}
