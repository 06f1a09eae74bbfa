"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that the pins catch each one.

Every mutant is compiled from a textual edit of a temporary copy of the
oracle's C source; the committed oracle is never modified.
"""
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import frac_erx, numpy_erx

SRC = os.path.join(os.path.dirname(oracle.__file__), "erx_oracle.c")

MUTANTS = {
    # covariance normalised by p instead of p-1 (Sec. III-C, Eq. (19))
    "cov_over_p": ("s /= (double)(p - 1);", "s /= (double)p;"),
    # momentum applied to the wrong term (Sec. III-C, Eqs. (20)-(21))
    "ema_swapped": ("mu[j] = (1.0 - alpha) * mu[j] + alpha * mu_hat[j];",
                    "mu[j] = alpha * mu[j] + (1.0 - alpha) * mu_hat[j];"),
    "ema_swapped_K": ("K[e] = (1.0 - alpha) * K[e] + alpha * K_hat[e];",
                      "K[e] = alpha * K[e] + (1.0 - alpha) * K_hat[e];"),
    # ridge dropped (Sec. III-D)
    "no_ridge": ("A[(size_t)j * b + j] += eps;", "A[(size_t)j * b + j] += 0.0;"),
    # ridge added twice
    "double_ridge": ("A[(size_t)j * b + j] += eps;", "A[(size_t)j * b + j] += 2.0 * eps;"),
    # transposed factor in the forward substitution (Sec. III-D, Eq. (23))
    "transposed_L": ("s -= L[(size_t)i * b + k] * m[k];", "s -= L[(size_t)k * b + i] * m[k];"),
    # covariance not centred
    "uncentred": ("Ct[(size_t)j * p + i] = X[(size_t)i * b + j] - mu_hat[j];",
                  "Ct[(size_t)j * p + i] = X[(size_t)i * b + j];"),
    # first line not used as the initial background (Sec. III-C)
    "no_first_line_init": ("if (*t == 0) {", "if (0) {"),
    # squared distance returned instead of the distance
    "no_sqrt": ("return sqrt(ss);", "return ss;"),
    # wrong sign in the residual
    "residual_sign": ("r[j] = xi[j] - mu[j];", "r[j] = xi[j] + mu[j];"),
    # score with the line's own mean instead of the background mean
    "score_line_mean": ("r[j] = xi[j] - mu[j];", "r[j] = xi[j] - mu_hat[j];"),
    # sample instead of population deviation in the normalisation (Sec. III-E)
    "norm_sample_std": ("var /= (double)p;", "var /= (double)(p - 1);"),
    # off-by-one in the Cholesky inner loop
    "chol_off_by_one": ("for (int k = 0; k < j; ++k) s -= L[(size_t)i * b + k] * L[(size_t)j * b + k];",
                        "for (int k = 0; k + 1 < j; ++k) s -= L[(size_t)i * b + k] * L[(size_t)j * b + k];"),
}


def _pins_pass(lib) -> bool:
    """A compact run of the pins against a given oracle build."""
    rng = np.random.default_rng(4242)
    # exact brute force
    Xi = rng.integers(-6, 7, size=(5, 5, 3))
    for a, e in [(Fraction(1, 2), Fraction(1, 100000)), (Fraction(1, 10), Fraction(0))]:
        ex = np.array(frac_erx(Xi.tolist(), a, e), dtype=float)
        got = oracle.run(Xi.astype(float), float(a), float(e), lib=lib)["delta"] ** 2
        if not np.allclose(got, ex, rtol=1e-12, atol=1e-12):
            return False
    # numpy brute force
    X = rng.standard_normal((20, 16, 5)) @ rng.standard_normal((5, 5)) + 1.0
    if not np.allclose(oracle.run(X, 0.1, 1e-5, lib=lib)["delta"], numpy_erx(X, 0.1, 1e-5),
                       rtol=1e-10):
        return False
    # normalisation: population deviation
    r = oracle.run(X, 0.1, 1e-5, normalise=True, lib=lib)
    if not np.allclose(r["delta_n"].std(1), 1.0, rtol=1e-10):
        return False
    return True


def _build_mutant(tmp, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    path = os.path.join(tmp, f"{name}.c")
    open(path, "w").write(src.replace(old, new, 1))
    out = os.path.join(tmp, f"lib{name}.so")
    oracle.build(src=path, out=out)
    return oracle.load(out)


@pytest.fixture(scope="module")
def tmpdir_mod():
    d = tempfile.mkdtemp(prefix="ero_mut_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def test_unmutated_oracle_passes(tmpdir_mod):
    assert _pins_pass(oracle.load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmpdir_mod):
    old, new = MUTANTS[name]
    lib = _build_mutant(tmpdir_mod, name, old, new)
    assert not _pins_pass(lib), f"mutant {name} survived the pins"
