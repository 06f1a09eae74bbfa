"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/erx.h declares, and rejects invalid arguments
before touching the device."""
import ctypes as C
import os
import re

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
                                         ("dtype", 7), ("precision", 3), ("block_lines", 0), ("scan_lines", 0),
                                         ("warmup", -1), ("fp64_cond_threshold", -1.0),
                                         ("cond_estimate", 2)])
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
    assert (cfg.bands, cfg.pixels, cfg.dtype, cfg.precision) == (108, 640, 0, 0)
    assert abs(cfg.ridge - 1e-5) < 1e-12 and cfg.fp64_cond_threshold == 0.0
    assert cfg.block_lines == 2048 and cfg.scan_lines == 64
