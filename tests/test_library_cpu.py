"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/erx.h declares, and rejects invalid arguments
before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "erx.h")


def _lib():
    import paper_2408_14947_amd as erx
    if not os.path.exists(erx.LIB_PATH):
        pytest.skip("liberx.so not built (run __graft_entry__.build())")
    return erx, erx.load()


def declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"ERX_API[^;(]*?\b(erx_\w+)\s*\(", txt)))


def test_header_lists_the_binding_exports():
    import paper_2408_14947_amd as erx
    assert declared_functions() == sorted(erx.EXPORTS)


def test_library_exports_every_declared_symbol():
    erx, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # nothing but the C ABI is exported
    out = os.popen(f"nm -D --defined-only {erx.LIB_PATH}").read().split("\n")
    text = [l.split()[-1] for l in out if " T " in l]
    assert sorted(text) == declared_functions()


@pytest.mark.parametrize("field,value", [("bands", 0), ("bands", 305), ("pixels", 1),
                                         ("momentum", 0.0), ("momentum", 1.5),
                                         ("momentum", float("nan")), ("ridge", -1e-3),
                                         ("dtype", 7), ("precision", 4), ("block_lines", 0), ("scan_lines", 0),
                                         ("warmup", -1), ("fp64_cond_threshold", -1.0),
                                         ("cond_estimate", 2), ("state_fp32", 2), ("score_tiles", 3),
                                         ("gram_macro", 96)])
def test_create_rejects_invalid_config(field, value):
    erx, lib = _lib()
    cfg = erx.Config()
    lib.erx_config_default(C.byref(cfg), 8, 16, 0.1)
    setattr(cfg, field, value)
    assert not lib.erx_create_ex(C.byref(cfg))
    assert field.split("_")[0] in erx.last_error() or "unknown" in erx.last_error() \
        or "must" in erx.last_error()


def test_null_handle_is_rejected():
    erx, lib = _lib()
    assert lib.erx_push_lines_ex(None, None, 1) == erx.ERX_EINVAL
    assert lib.erx_scores(None, None) == erx.ERX_EINVAL
    assert lib.erx_set_state(None, 0, None, None) == erx.ERX_EINVAL
    lib.erx_destroy(None)


def test_defaults():
    erx, lib = _lib()
    cfg = erx.Config()
    lib.erx_config_default(C.byref(cfg), 108, 640, 0.1)
    assert (cfg.bands, cfg.pixels, cfg.dtype, cfg.precision) == (108, 640, 0, 3)
    assert abs(cfg.ridge - 1e-5) < 1e-12 and cfg.fp64_cond_threshold == 0.0
    assert cfg.block_lines == 2048 and cfg.scan_lines == 64
    assert (cfg.srp_dims, cfg.background, cfg.state_fp32) == (0, 0, 0)


def test_config_layout_matches_the_header():
    """erx_config_default clears the whole C struct: every byte of the binding's Config
    (its last field included) is written and nothing after it."""
    erx, lib = _lib()
    n = C.sizeof(erx.Config)
    buf = (C.c_ubyte * (n + 64))(*([0xAB] * (n + 64)))
    lib.erx_config_default(C.cast(buf, C.POINTER(erx.Config)), 8, 16, 0.1)
    assert all(v == 0xAB for v in buf[n:])
    cfg = erx.Config.from_buffer_copy(bytes(buf[:n]))
    assert cfg.state_fp32 == 0 and cfg.gram_macro == 0 and cfg.bands == 8


def test_state_fp32_combinations_rejected():
    """FP32 storage is for the moving averages: the IMC moments and the RX Baseline's
    running sums stay FP64, and the allocation-free entry point takes an FP64 state."""
    erx, lib = _lib()
    cfg = erx.Config()
    lib.erx_config_default(C.byref(cfg), 8, 16, 0.1)
    cfg.state_fp32 = 1
    cfg.background = 1
    assert not lib.erx_create_ex(C.byref(cfg)) and "state_fp32" in erx.last_error()
    cfg.background = 0
    assert not lib.erx_rxb_create(C.byref(cfg), 5)
    dummy = C.c_void_p(16)
    assert lib.erx_push_lines_noalloc(C.byref(cfg), dummy, 0, dummy, 4, dummy, None) == erx.ERX_EINVAL
    assert "state_fp32" in erx.last_error()


def test_tune_cache_lookup(tmp_path):
    """The autotuner's JSON cache is read without any device work: an entry for the
    same shape is returned, another shape gives None, a file of another form is an
    error (and a missing file an empty cache)."""
    erx, _ = _lib()
    path = str(tmp_path / "tune.json")
    assert erx.tune_lookup(224, 1024, path) is None  # no file yet
    with open(path, "w") as f:
        f.write('{"erx_tune": 1, "entries": [\n'
                '  {"bands": 224, "pixels": 1024, "dtype": 0, "precision": 3, "normalise": 0, "nstreams": 1, '
                '"fp64_cond_threshold": 0, "block_lines": 4096, "scan_lines": 32, "small_path": -1, '
                '"us_per_line": 11.5},\n'
                '  {"bands": 8, "pixels": 1280, "dtype": 1, "precision": 3, "normalise": 0, "nstreams": 1024, '
                '"fp64_cond_threshold": 0, "block_lines": 1024, "scan_lines": 64, "small_path": 1, '
                '"us_per_line": 0.04}\n]}\n')
    r = erx.tune_lookup(224, 1024, path)
    assert r == {"block_lines": 4096, "scan_lines": 32, "small_path": -1, "score_tiles": 0, "gram_macro": 0,
                 "candidates": 0, "us_per_line": 11.5}
    # the arithmetic is part of the key (entries without it were written for the defaults)
    assert erx.tune_lookup(224, 1024, path, score_arith="fp32") is None
    assert erx.tune_lookup(224, 1024, path, state_fp32=True) is None
    r = erx.tune_lookup(8, 1280, path, dtype="f16", nstreams=1024)
    assert r["small_path"] == 1 and r["block_lines"] == 1024
    assert erx.tune_lookup(8, 1280, path, dtype="f16", nstreams=1) is None        # other stream count
    assert erx.tune_lookup(224, 1024, path, precision="bf16") is None             # other precision
    assert erx.tune_lookup(224, 1024, path, precision="fp32") is None
    assert erx.tune_lookup(224, 1024, path, fp64_cond_threshold=1e6) is None      # other threshold
    with open(path, "w") as f:
        f.write('{"something": "else"}\n')
    with pytest.raises(erx.ErxError) as e:
        erx.tune_lookup(224, 1024, path)
    assert e.value.code == erx.ERX_EINVAL
    with pytest.raises(erx.ErxError):
        erx.autotune(224, 1024, nstreams=0)  # rejected before any device work


def test_noalloc_rejects_invalid_arguments_before_device_work():
    """erx_push_lines_noalloc checks its arguments on the host before any HIP call,
    so these return ERX_EINVAL on a machine without a GPU."""
    erx, lib = _lib()
    dummy = C.c_void_p(16)  # never dereferenced: every case fails before device work
    cases = [dict(bands=305), dict(bands=0), dict(pixels=1), dict(momentum=0.0), dict(normalise=1),
             dict(dtype=5), dict(precision=9), dict(block_lines=0), dict(scan_lines=0)]
    for case in cases:
        cfg = erx.Config()
        lib.erx_config_default(C.byref(cfg), 16, 32, 0.1)
        for k, v in case.items():
            setattr(cfg, k, v)
        assert lib.erx_push_lines_noalloc(C.byref(cfg), dummy, 0, dummy, 4, dummy, None) == erx.ERX_EINVAL, case
    cfg = erx.Config()
    lib.erx_config_default(C.byref(cfg), 16, 32, 0.1)
    assert lib.erx_push_lines_noalloc(C.byref(cfg), dummy, 0, dummy, 0, dummy, None) == erx.ERX_EINVAL
    assert "n must be" in erx.last_error()
    assert lib.erx_push_lines_noalloc(C.byref(cfg), dummy, -1, dummy, 4, dummy, None) == erx.ERX_EINVAL
    assert lib.erx_push_lines_noalloc(None, dummy, 0, dummy, 4, dummy, None) == erx.ERX_EINVAL
    assert erx.noalloc_state_entries(224) == 256 * 105 + 224


def test_srp_matrix_matches_reference_generator():
    """erx_srp_matrix (host code of the library) draws exactly the weights of the FP64
    reference (both implement the published SplitMix64 generator): same zero pattern
    and signs, values equal after rounding the reference's to FP32."""
    erx, _ = _lib()
    from oracle import srp
    for b, d, seed in [(108, 5, 0), (224, 5, 12345), (13, 3, 7), (300, 32, 2 ** 63 + 5)]:
        W = erx.srp_matrix(b, d, seed)
        ref = srp.srp_matrix(b, d, seed)
        assert W.shape == (b, d)
        assert np.array_equal(W, ref.astype(np.float32)), (b, d, seed)
    with pytest.raises(erx.ErxError):
        erx.srp_matrix(100, 33, 0)
    with pytest.raises(erx.ErxError):
        erx.srp_matrix(0, 5, 0)
