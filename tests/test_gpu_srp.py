"""The sparse random projection front end (Sec. III-B) through the C ABI: a detector
with srp_dims = d projects each line with the weights of erx_srp_matrix and runs ERX
on the projection.  Checked against the FP64 oracle run on Z = X W with the same
weights (the reference generator draws them), per pixel within 1e-4."""
import sys

import numpy as np
import pytest
import torch

import datagen
from oracle import srp as oracle_srp

pytestmark = pytest.mark.gpu
TOL = 1e-4


def log(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def erx():
    import paper_2408_14947_amd as m
    m.load()
    return m


def rel_err(got, want):
    return np.abs(np.asarray(got, np.float64) - want) / np.maximum(np.abs(want), 1.0)


@pytest.mark.parametrize("b,p,T,d,storage", [(108, 640, 120, 5, "f32"), (224, 300, 70, 5, "f32"),
                                             (90, 600, 80, 1, "f32"), (40, 200, 60, 16, "f16"),
                                             (13, 1116, 50, 3, "u16"), (300, 256, 30, 32, "f32")])
def test_srp_detector_matches_oracle(erx, b, p, T, d, storage):
    log(f"SRP detector b={b} p={p} T={T} d={d} {storage}")
    scene = datagen.make_scene(41, b * 7 + d, b, p, T)
    X, _ = datagen.lines(scene, 0, T)
    Xs = datagen.to_storage(X, storage)
    seed = 1000 + d
    det = erx.Detector(b, p, 0.1, dtype=storage, srp_dims=d, srp_seed=seed, block_lines=48, scan_lines=16)
    det.push(Xs.cuda())
    got = det.scores().cpu().numpy()
    torch.cuda.synchronize()
    Xf = datagen.storage_to_float64(Xs, storage)
    want = oracle_srp.run(Xf, d, seed, 0.1)["delta"]
    err = rel_err(got, want)
    t, mu, K = det.state()
    log(f"  max err {err.max():.3e}  state dims {mu.shape[0]}")
    assert mu.shape == (d,) and K.shape == (d, d) and t == T
    assert err.max() <= TOL
