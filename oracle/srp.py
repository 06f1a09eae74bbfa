"""FP64 reference of the sparse random projection front end of ERX (Sec. III-B).

TEST INFRASTRUCTURE ONLY: imported by the tests.  The GPU library never imports or
calls anything here, and nothing here imports the GPU library.

Sec. III-B draws every weight of W in R^{b x d} independently:
    w_ij = sqrt(s / d) * (+1 with probability 1/(2s), 0 with 1 - 1/s, -1 with 1/(2s)),
with sparsity s = sqrt(b), so about d sqrt(b) weights are non-zero; each line X_t is
projected to Z_t = X_t W and ERX then runs on Z_t in d dimensions.

The random draws come from SplitMix64 used as a counter-based generator (its
published output function applied to seed + k * 0x9e3779b97f4a7c15): weight (i, j)
takes the k = i d + j + 1 -th output u, as the uniform number (u >> 11) 2^-53 in
[0, 1); it is +1 below 1/(2s), -1 below 1/s and 0 otherwise.  The GPU library
implements the same published generator on its own, so both sides draw the same W.
"""
from __future__ import annotations

import math

import numpy as np

import oracle

_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, k: int) -> int:
    """k-th output (k >= 1) of SplitMix64 started from state `seed`."""
    z = (seed + k * _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def srp_matrix(bands: int, dims: int, seed: int) -> np.ndarray:
    """W [bands][dims] of Sec. III-B (FP64)."""
    s = math.sqrt(bands)
    scale = math.sqrt(s / dims)
    p_half = 1.0 / (2.0 * s)
    W = np.zeros((bands, dims), np.float64)
    for i in range(bands):
        for j in range(dims):
            u = (splitmix64(seed, i * dims + j + 1) >> 11) * 2.0 ** -53
            if u < p_half:
                W[i, j] = scale
            elif u < 2.0 * p_half:
                W[i, j] = -scale
    return W


def project(X, W) -> np.ndarray:
    """Z_t = X_t W for every line of X [n][p][b] (FP64)."""
    return np.asarray(X, np.float64) @ W


def run(X, dims: int, seed: int, momentum: float, ridge: float = 1e-5, **kw) -> dict:
    """ERX (the FP64 oracle) on the projected lines Z = X W."""
    X = np.asarray(X, np.float64)
    W = srp_matrix(X.shape[2], dims, seed)
    return oracle.run(project(X, W), momentum, ridge, **kw)
