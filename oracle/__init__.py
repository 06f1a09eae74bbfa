"""FP64 CPU oracle of the ERX detector (ctypes wrapper around erx_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark.  The GPU library never imports, links or
calls anything here, and nothing here imports the GPU library.

Every input is promoted exactly to float64 before it reaches the C code, so the
oracle consumes precisely the values the GPU path consumed.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "erx_oracle.c")
_LIB = os.path.join(_HERE, "liberx_oracle.so")
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_llp = C.POINTER(C.c_longlong)


def build(src: str = _SRC, out: str = _LIB, extra=()) -> str:
    """Compile the oracle with gcc (plain C, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fvisibility=hidden",
           *extra, src, "-o", out, "-lm"]
    subprocess.check_call(cmd)
    return out


def load(path: str = _LIB):
    """Load a built oracle library (building it if it is absent)."""
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        build(out=path)
    lib = C.CDLL(path)
    lib.ero_line_mean.argtypes = [C.c_int, C.c_int, _dp, _dp]
    lib.ero_line_cov.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, C.c_int]
    lib.ero_cholesky.argtypes = [C.c_int, _dp, _dp]
    lib.ero_cholesky.restype = C.c_int
    lib.ero_mahalanobis.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.ero_mahalanobis.restype = C.c_double
    lib.ero_normalise.argtypes = [C.c_int, _dp, _dp]
    lib.ero_push.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _llp, _dp, _dp,
                             _dp, C.c_longlong, _dp, _dp, _dp, _dp, _ip, C.c_int]
    lib.ero_push.restype = C.c_longlong
    lib.ero_max_threads.restype = C.c_int
    if path == _LIB:
        _lib = lib
    return lib


def _p(a: Optional[np.ndarray], t=_dp):
    return None if a is None else a.ctypes.data_as(t)


def f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def max_threads(lib=None) -> int:
    return int((lib or load()).ero_max_threads())


class Stream:
    """One ERX stream in FP64: state (t, mu, K) plus the paper's per-line loop."""

    def __init__(self, bands: int, pixels: int, momentum: float, ridge: float = 1e-5,
                 lib=None, nthreads: int = 0):
        self.b, self.p = int(bands), int(pixels)
        self.alpha, self.eps = float(momentum), float(ridge)
        self.lib = lib or load()
        self.nthreads = int(nthreads)
        self.t = C.c_longlong(0)
        self.mu = np.zeros(self.b)
        self.K = np.zeros((self.b, self.b))

    def set_state(self, t: int, mu, K):
        self.t = C.c_longlong(int(t))
        self.mu = f64(mu).copy()
        self.K = f64(K).copy()

    def state(self):
        return int(self.t.value), self.mu.copy(), self.K.copy()

    def push(self, X, normalise: bool = False, history: bool = False):
        """Absorb and score lines X [n, p, b] (any real dtype; promoted to f64).

        Returns a dict with 'delta' [n, p], optionally 'delta_n', 'mu_hist',
        'K_hist', plus 'notpd' [n] flags.
        """
        X = f64(X)
        if X.ndim == 2:
            X = X[None]
        n = X.shape[0]
        if X.shape[1:] != (self.p, self.b):
            raise ValueError(f"lines must be [n, {self.p}, {self.b}], got {X.shape}")
        delta = np.empty((n, self.p))
        dn = np.empty((n, self.p)) if normalise else None
        mh = np.empty((n, self.b)) if history else None
        kh = np.empty((n, self.b, self.b)) if history else None
        notpd = np.zeros(n, np.int32)
        r = self.lib.ero_push(self.b, self.p, self.alpha, self.eps, C.byref(self.t),
                              _p(self.mu), _p(self.K), _p(X), n, _p(delta), _p(dn),
                              _p(mh), _p(kh), _p(notpd, _ip), self.nthreads)
        if r < 0:
            raise ValueError("invalid oracle arguments")
        out = dict(delta=delta, notpd=notpd)
        if normalise:
            out["delta_n"] = dn
        if history:
            out["mu_hist"], out["K_hist"] = mh, kh
        return out


def run(X, momentum: float, ridge: float = 1e-5, normalise: bool = False,
        history: bool = False, nthreads: int = 0, lib=None):
    """Score a whole stream from a fresh state."""
    X = f64(X)
    s = Stream(X.shape[2], X.shape[1], momentum, ridge, lib=lib, nthreads=nthreads)
    out = s.push(X, normalise=normalise, history=history)
    out["stream"] = s
    return out


def line_mean(X, lib=None):
    X = f64(X)
    p, b = X.shape
    mu = np.empty(b)
    (lib or load()).ero_line_mean(b, p, _p(X), _p(mu))
    return mu


def line_cov(X, mu=None, lib=None):
    X = f64(X)
    p, b = X.shape
    mu = line_mean(X, lib) if mu is None else f64(mu)
    K = np.empty((b, b))
    (lib or load()).ero_line_cov(b, p, _p(X), _p(mu), _p(K), 0)
    return K


def cholesky(A, lib=None):
    A = f64(A)
    b = A.shape[0]
    L = np.empty((b, b))
    info = (lib or load()).ero_cholesky(b, _p(A), _p(L))
    return L, int(info)


def mahalanobis(L, r, lib=None):
    L, r = f64(L), f64(r)
    m = np.empty(L.shape[0])
    d = (lib or load()).ero_mahalanobis(L.shape[0], _p(L), _p(r), _p(m))
    return float(d), m


def normalise(delta, lib=None):
    d = f64(delta)
    out = np.empty_like(d)
    (lib or load()).ero_normalise(d.shape[0], _p(d), _p(out))
    return out
