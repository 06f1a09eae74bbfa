"""Seeded synthetic scan-line generators.

This module produces INPUTS only: hyperspectral lines X_t in R^{p x b}
(pixels x bands, band index fastest) and their ground-truth anomaly masks.
It contains none of the detector's arithmetic, and both the FP64 oracle and
the GPU path consume exactly the arrays it returns.

The paper's datasets (Sec. IV-A) are not available, so seeded stand-ins with
the same structure are used: a mixture of smooth endmember spectra, a random
low-rank band covariance plus white noise, sparse anomalies with distinct
spectra, optionally a slow drift of the scene composition along the line
index (the "changing scenery" that motivates the exponential moving averages
in Sec. III-C) and 3x3 pixel-line anomaly patches.

Generation is chunkable: line t is produced from a generator keyed by
(config, stream, t // BLOCK), so any window of lines can be regenerated
without producing the lines before it, on the CPU or on a GPU.  The same seed
on two different devices gives different (but equally valid) random streams;
every consumer therefore receives the array actually generated, never a
regeneration.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import torch

BASE_SEED = 240814947
BLOCK = 64  # lines per generator key

__all__ = [
    "Scene", "smooth_curves", "make_scene", "lines", "config_scenes",
    "CONFIGS", "to_storage", "storage_to_float64",
]


def _seed(*keys: int) -> int:
    """63-bit integer seed derived from an integer key tuple."""
    ss = np.random.SeedSequence([BASE_SEED] + [int(k) for k in keys])
    a, b = ss.generate_state(2, dtype=np.uint32)
    return int((int(a) << 31) ^ int(b)) & ((1 << 63) - 1)


def smooth_curves(rng: np.random.Generator, n: int, b: int,
                  lo: float = 0.05, hi: float = 0.8, knots: int = 8) -> np.ndarray:
    """n smooth spectra over b bands with values in [lo, hi].

    Knot values are U[lo, hi] at `knots` equally spaced band positions; bands in
    between use cosine interpolation, so every value stays inside [lo, hi].
    """
    out = np.empty((n, b), np.float64)
    pos = np.linspace(0.0, max(b - 1, 1), knots)
    x = np.arange(b, dtype=np.float64)
    seg = np.clip(np.searchsorted(pos, x, side="right") - 1, 0, knots - 2)
    t = (x - pos[seg]) / (pos[seg + 1] - pos[seg])
    w = 0.5 * (1.0 - np.cos(math.pi * t))
    for k in range(n):
        v = rng.uniform(lo, hi, knots)
        out[k] = v[seg] * (1.0 - w) + v[seg + 1] * w
    return out


def _corr(a: np.ndarray, b: np.ndarray) -> float:
    a = a - a.mean()
    b = b - b.mean()
    d = math.sqrt(float(a @ a) * float(b @ b))
    return float(a @ b) / d if d > 0 else 1.0


@dataclasses.dataclass
class Scene:
    """Static description of one synthetic line stream."""
    cfg: int
    stream: int
    bands: int
    pixels: int
    lines: int
    kind: str                      # "mixture" (endmember mixture) or "gauss"
    storage: str                   # "f32", "f16" or "u16"
    momentum: float
    anomaly_rate: float            # fraction of pixels replaced by anomalies
    patches: bool                  # anomalies in 3x3 pixel-line patches
    drift: bool                    # endmember weights drift along the line index
    endmembers: np.ndarray         # [E, b] (mixture) or [1, b] mean (gauss)
    factor: np.ndarray             # [b, r] low-rank covariance factor
    noise: float                   # white-noise standard deviation
    anomalies: np.ndarray          # [3, b] anomaly spectra
    weights: np.ndarray            # [E] static mixture weights
    periods: np.ndarray            # [E] drift periods (lines)
    phases: np.ndarray             # [E] drift phases

    @property
    def seed(self) -> int:
        return _seed(self.cfg, self.stream)

    def mixture_weights(self, t: np.ndarray) -> np.ndarray:
        """Endmember probabilities for lines t (0-based), shape [len(t), E]."""
        if not self.drift:
            return np.broadcast_to(self.weights, (len(t), len(self.weights)))
        z = 2.0 * np.sin(2.0 * math.pi * t[:, None] / self.periods[None, :]
                         + self.phases[None, :])
        w = np.exp(z)
        return w / w.sum(1, keepdims=True)


def make_scene(cfg: int, stream: int, bands: int, pixels: int, lines: int,
               kind: str = "mixture", storage: str = "f32", momentum: float = 0.1,
               anomaly_rate: float = 0.005, patches: bool = False,
               drift: bool = False) -> Scene:
    """Draw the static parameters of one stream from its seed."""
    rng = np.random.default_rng(np.random.SeedSequence([BASE_SEED, cfg, stream, 7]))
    b = bands
    if kind == "mixture":
        E = smooth_curves(rng, 4, b)
        F = 0.01 * rng.standard_normal((b, 8))
        noise = 0.01
    elif kind == "gauss":
        E = smooth_curves(rng, 1, b)
        F = 0.05 * rng.standard_normal((b, (b + 1) // 2))
        noise = 0.01
    else:
        raise ValueError(kind)
    # anomaly spectra: distinct smooth curves, correlation <= 0.98 to every endmember
    A = []
    while len(A) < 3:
        c = smooth_curves(rng, 1, b)[0]
        if b < 3 or all(_corr(c, e) <= 0.98 for e in E):
            A.append(c)
    weights = rng.dirichlet(np.ones(E.shape[0]))
    periods = rng.uniform(5000.0, 20000.0, E.shape[0])
    phases = rng.uniform(0.0, 2.0 * math.pi, E.shape[0])
    return Scene(cfg, stream, b, pixels, lines, kind, storage, float(momentum),
                 float(anomaly_rate), bool(patches), bool(drift), E, F, float(noise),
                 np.stack(A), weights, periods, phases)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def _uniform_hash(seed: int, a: np.ndarray, c: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        key = (np.uint64(seed) ^ (a.astype(np.uint64) * np.uint64(0x100000001B3))
               ^ (c.astype(np.uint64) * np.uint64(0xC2B2AE3D27D4EB4F)))
    return (_splitmix64(key) >> np.uint64(11)).astype(np.float64) / float(1 << 53)


def _block(scene: Scene, blk: int, device: torch.device, span: int = BLOCK):
    """Lines [blk*span, (blk+1)*span) as float32 plus bool mask.  The default span is
    BLOCK; a longer span draws more lines per generator key (fewer, larger calls for
    whole streams), from a key space of its own."""
    n = min(span, scene.lines - blk * span) if scene.lines > 0 else span
    n = max(n, 0)
    p, b = scene.pixels, scene.bands
    g = torch.Generator(device=device)
    g.manual_seed(_seed(scene.cfg, scene.stream, 1000003 + blk) if span == BLOCK
                  else _seed(scene.cfg, scene.stream, 2000003, span, blk))
    f32 = dict(device=device, dtype=torch.float32)
    t = np.arange(blk * span, blk * span + n, dtype=np.float64)
    E = torch.as_tensor(scene.endmembers, **f32)
    F = torch.as_tensor(scene.factor, **f32)
    A = torch.as_tensor(scene.anomalies, **f32)
    if scene.kind == "mixture":
        cdf = torch.as_tensor(np.cumsum(scene.mixture_weights(t), 1), **f32)
        u = torch.rand((n, p), generator=g, **f32)
        k = torch.searchsorted(cdf.contiguous(), u.contiguous()).clamp_(max=E.shape[0] - 1)
        base = E[k]
    else:
        base = E[0].expand(n, p, b)
    lat = torch.randn((n, p, F.shape[1]), generator=g, **f32)
    noise = torch.randn((n, p, b), generator=g, **f32)
    common = torch.matmul(lat, F.t().contiguous()) + scene.noise * noise
    if scene.patches:
        # 3x3 pixel-line cells; a cell is a patch with probability anomaly_rate
        m = (t.astype(np.int64) // 3)[:, None].repeat(p, 1)
        q = np.broadcast_to(np.arange(p, dtype=np.int64) // 3, (n, p))
        full = np.broadcast_to(np.arange(p) < (p // 3) * 3, (n, p))
        h = _uniform_hash(scene.seed, m, q)
        mask_np = (h < scene.anomaly_rate) & full
        which_np = (_uniform_hash(scene.seed ^ 0x5DEECE66D, m, q) * 3).astype(np.int64)
        mask = torch.as_tensor(mask_np, device=device)
        which = torch.as_tensor(which_np, device=device).clamp_(max=2)
    else:
        mask = torch.rand((n, p), generator=g, **f32) < scene.anomaly_rate
        which = torch.randint(0, 3, (n, p), generator=g, device=device)
    x = torch.where(mask[..., None], A[which], base) + common
    return x, mask


def lines(scene: Scene, t0: int, n: int, device="cpu", storage: Optional[str] = None, span: int = BLOCK):
    """Lines [t0, t0+n) of a stream.

    Returns (X, mask): X has shape [n, p, b] in the stream's storage type
    (float32, float16, or uint16 raw counts whose value is u * 2**-16) and mask
    is a bool [n, p] tensor marking anomalous pixels.  span: lines per generator
    key (BLOCK by default; a different span gives a different, equally valid draw).
    """
    device = torch.device(device)
    storage = storage or scene.storage
    if n <= 0:
        X = torch.empty((0, scene.pixels, scene.bands), dtype=torch.float32, device=device)
        return to_storage(X, storage), torch.zeros((0, scene.pixels), dtype=torch.bool, device=device)
    xs, ms = [], []
    b0, b1 = t0 // span, (t0 + n - 1) // span
    for blk in range(b0, b1 + 1):
        x, m = _block(_unbounded(scene), blk, device, span)
        lo = max(t0 - blk * span, 0)
        hi = min(t0 + n - blk * span, span)
        xs.append(x[lo:hi])
        ms.append(m[lo:hi])
    X = torch.cat(xs) if len(xs) > 1 else xs[0]
    M = torch.cat(ms) if len(ms) > 1 else ms[0]
    return to_storage(X.contiguous(), storage), M.contiguous()


def _unbounded(scene: Scene) -> Scene:
    # block generation ignores the nominal length, so windows past it still work
    return dataclasses.replace(scene, lines=1 << 40)


def to_storage(x: torch.Tensor, storage: str) -> torch.Tensor:
    """float32 lines -> storage type.  u16 holds round(clip(x,0,1)*65535)."""
    if storage == "f32":
        return x
    if storage == "f16":
        return x.to(torch.float16)
    if storage == "u16":
        u = torch.round(torch.clamp(x, 0.0, 1.0) * 65535.0).to(torch.int32)
        return u.to(torch.uint16) if hasattr(torch, "uint16") else u.to(torch.int16)
    raise ValueError(storage)


def storage_to_float64(x: torch.Tensor | np.ndarray, storage: str) -> np.ndarray:
    """Exact promotion of stored lines to float64 (u16 values are u * 2**-16)."""
    if isinstance(x, torch.Tensor):
        x = x.detach().cpu()
        if storage == "u16":
            x = x.view(torch.int16).numpy().view(np.uint16)
        else:
            x = x.numpy()
    if storage == "u16":
        return np.ldexp(x.astype(np.float64), -16)
    return x.astype(np.float64)


# ---------------------------------------------------------------------------
# Workload configurations (shapes, storage types and scene recipes)
# ---------------------------------------------------------------------------
CONFIGS = {
    1: dict(name="plain-108", bands=108, pixels=640, lines=500, storage="f32",
            momentum=0.1, anomaly_rate=0.005),
    2: dict(name="long-scan-224", bands=224, pixels=1024, lines=20000, storage="f32",
            momentum=0.1, anomaly_rate=0.002, patches=True, drift=True),
    3: dict(name="batched-u16", streams=64, storage="u16", momentum=0.1,
            anomaly_rate=0.005),
    4: dict(name="batched-multispectral-f16", streams=1024, pixels=1280, lines=5000,
            storage="f16", kind="gauss", anomaly_rate=0.005),
    5: dict(name="surrogate", bands=(108, 224), pixels=640, storage="f32",
            momentum=0.1, anomaly_rate=0.005),
}


def config_scenes(cfg: int, scale_lines: Optional[int] = None,
                  streams: Optional[int] = None) -> Sequence[Scene]:
    """Scenes of a workload configuration.

    scale_lines caps each stream's length (for reduced-size test variants);
    streams caps the number of streams of a batched configuration.
    """
    c = CONFIGS[cfg]
    out = []
    if cfg in (1, 2):
        T = c["lines"] if scale_lines is None else min(scale_lines, c["lines"])
        out.append(make_scene(cfg, 0, c["bands"], c["pixels"], T, storage=c["storage"],
                              momentum=c["momentum"], anomaly_rate=c["anomaly_rate"],
                              patches=c.get("patches", False), drift=c.get("drift", False)))
    elif cfg == 3:
        rng = np.random.default_rng(np.random.SeedSequence([BASE_SEED, 3, 99]))
        ns = c["streams"] if streams is None else min(streams, c["streams"])
        P = rng.integers(256, 2049, c["streams"])
        B = rng.integers(32, 301, c["streams"])
        L = rng.integers(2000, 10001, c["streams"])
        for s in range(ns):
            T = int(L[s]) if scale_lines is None else min(scale_lines, int(L[s]))
            out.append(make_scene(3, s, int(B[s]), int(P[s]), T, storage="u16",
                                  momentum=c["momentum"], anomaly_rate=c["anomaly_rate"]))
    elif cfg == 4:
        rng = np.random.default_rng(np.random.SeedSequence([BASE_SEED, 4, 99]))
        ns = c["streams"] if streams is None else min(streams, c["streams"])
        B = rng.integers(4, 17, c["streams"])
        A = rng.uniform(0.01, 0.3, c["streams"])
        for s in range(ns):
            T = c["lines"] if scale_lines is None else min(scale_lines, c["lines"])
            out.append(make_scene(4, s, int(B[s]), c["pixels"], T, kind="gauss",
                                  storage="f16", momentum=float(A[s]),
                                  anomaly_rate=c["anomaly_rate"]))
    elif cfg == 5:
        ns = 1 if streams is None else streams
        for s in range(ns):
            for b in c["bands"]:
                T = 5000 if scale_lines is None else scale_lines
                out.append(make_scene(5, s * 1000 + b, b, c["pixels"], T,
                                      momentum=c["momentum"], anomaly_rate=c["anomaly_rate"]))
    else:
        raise ValueError(cfg)
    return out
