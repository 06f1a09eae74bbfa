"""FP64 reference of the learned band-projection surrogate of ERX (TEST
INFRASTRUCTURE ONLY: imported by tests/, the smoke check and bench.py's CPU
baseline, never by the product path).

The surrogate is a stated change to the method, the learned analogue of the
sparse random projection of Sec. III-B: instead of ERX on the b bands, ERX
(Sec. III-C/D, Eqs. (18)-(23)) runs on a learned 16-dimensional projection and a
small network corrects the score.

    z      = W x + c                       W: 16 x b, c: 16
    u      = L_z^{-1} (z - mu_z)           mu_z, K_z: ERX statistics of the z
                                           stream (same momentum, first-line
                                           initialisation and ridge), L_z L_z^T
                                           = K_z + eps I
    o      = w2 . relu(A1 u + a1) + c2     A1: 64 x 16, a1: 64, w2: 64, c2: 1
    score  = ||u|| exp(o)

Training loss over the pixels of a batch of lines:
    mean w (log score - log target)^2,   w = clip(target^2 / b, 1, 100)
with the targets the plain-ERX scores.  A background pixel's squared distance
averages b, so w is about 1 there; pixels that plain ERX scores far above the
background (the anomalies) weigh more, so that the 16 directions are not spent on
background alone.  The statistics mu_z and L_z are held
fixed (stop-gradient): gradients flow to W, c, A1, a1, w2 and c2 through u and
o only.  With W = I (b = 16), c = 0 and w2 = 0 the score is plain ERX.

The code below is the plain definition written out in FP64 with numpy: the
projection, a per-line ERX on z from the ERX oracle, the network, and the
hand-derived gradients of the loss.
"""
from __future__ import annotations

import numpy as np

K = 16        # projection width
HIDDEN = 64   # hidden units
LOSS_WCAP = 100.0  # largest loss weight of a pixel

PARAM_NAMES = ("W", "c", "A1", "a1", "w2", "c2")


def init_params(bands: int, seed: int = 0, scale: float = 1.0):
    """Deterministic initialisation (the GPU library uses its own; tests pass
    explicit parameters to both sides)."""
    rng = np.random.default_rng(seed)
    return {
        "W": rng.normal(0.0, scale / np.sqrt(bands), (K, bands)),
        "c": np.zeros(K),
        "A1": rng.normal(0.0, 1.0 / np.sqrt(K), (HIDDEN, K)),
        "a1": np.zeros(HIDDEN),
        "w2": rng.normal(0.0, 0.01, HIDDEN),
        "c2": np.zeros(1),
    }


def project(params, X):
    """z = W x + c for every pixel: X [n, p, b] -> Z [n, p, 16]."""
    X = np.asarray(X, np.float64)
    return X @ np.asarray(params["W"], np.float64).T + np.asarray(params["c"], np.float64)


def erx_stats(Z, momentum: float, ridge: float):
    """Per-line ERX statistics of the projected stream: mu [n, 16] and
    M = L^{-1} [n, 16, 16] with L L^T = K + ridge I."""
    from . import run
    out = run(Z, momentum, ridge, history=True)
    mu = out["mu_hist"]
    Ms = []
    for Kt in out["K_hist"]:
        L = np.linalg.cholesky(Kt + ridge * np.eye(Kt.shape[0]))
        Ms.append(np.linalg.inv(L))
    return mu, np.stack(Ms)


def forward(params, X, momentum: float, ridge: float = 1e-5, stats=None):
    """Scores of the surrogate for lines X [n, p, b].  Returns a dict with
    'score' [n, p] and the intermediate values the gradient needs."""
    Z = project(params, X)
    mu, M = erx_stats(Z, momentum, ridge) if stats is None else stats
    U = np.einsum("nij,npj->npi", M, Z - mu[:, None, :])          # u = M (z - mu)
    pre = U @ np.asarray(params["A1"], np.float64).T + params["a1"]  # [n, p, 64]
    H = np.maximum(pre, 0.0)
    o = H @ np.asarray(params["w2"], np.float64) + float(np.asarray(params["c2"]).reshape(-1)[0])
    nu2 = (U * U).sum(-1)
    score = np.sqrt(nu2) * np.exp(o)
    return {"score": score, "Z": Z, "mu": mu, "M": M, "U": U, "pre": pre, "H": H, "o": o, "nu2": nu2}


def loss_and_grads(params, X, target, momentum: float, ridge: float = 1e-5, stats=None):
    """Loss and its gradients with respect to every parameter, the line
    statistics held fixed."""
    X = np.asarray(X, np.float64)
    f = forward(params, X, momentum, ridge, stats)
    n, p = f["score"].shape
    N = n * p
    logs = 0.5 * np.log(f["nu2"]) + f["o"]
    e = logs - np.log(np.asarray(target, np.float64))
    b = X.shape[2]
    w = np.clip(np.asarray(target, np.float64) ** 2 / b, 1.0, LOSS_WCAP)
    loss = float((w * e * e).mean())
    G = 2.0 * w * e / N                               # d loss / d log score   [n, p]
    A1 = np.asarray(params["A1"], np.float64)
    w2 = np.asarray(params["w2"], np.float64)
    mask = (f["pre"] > 0.0).astype(np.float64)
    dPre = G[..., None] * w2[None, None, :] * mask     # [n, p, 64]
    g = {}
    g["c2"] = np.array([G.sum()])
    g["w2"] = np.einsum("np,npj->j", G, f["H"])
    g["A1"] = np.einsum("npj,npi->ji", dPre, f["U"])
    g["a1"] = dPre.sum((0, 1))
    # d log||u|| / du = u / ||u||^2
    dU = G[..., None] * f["U"] / f["nu2"][..., None] + dPre @ A1   # [n, p, 16]
    dZ = np.einsum("npi,nij->npj", dU, f["M"])        # dz = M^T du
    g["c"] = dZ.sum((0, 1))
    g["W"] = np.einsum("npi,npk->ik", dZ, X)
    return loss, g, f
