"""CPU checks of the C-ABI library: it loads without a GPU and exports every
entry point that include/sketch.h declares (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sketch.h")
LIB = os.path.join(ROOT, "paper_2601_02019_amd", "libsketch.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:SK_EXPORT\s+)?(?:sk_status|const char\*|int64_t)\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["sketch_create", "sketch_update", "sketch_query", "window_advance", "sketch_merge",
              "sketch_destroy", "sketch_sync", "sketch_last_error", "sketch_update_csr",
              "sketch_update_batch", "sketch_merge_tree"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsketch.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsketch.so not built")
def test_library_loads_and_rejects_bad_config_without_gpu():
    from paper_2601_02019_amd import _lib
    lib = _lib.load()
    cfg = _lib.sketch_config()
    assert lib.sketch_config_init(ctypes.byref(cfg)) == 0
    assert cfg.q == 1 and cfg.state_dtype == _lib.SK_F64
    h = ctypes.c_void_p()
    # d = 0 is rejected before any device call
    assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
    assert b"d >= 1" in lib.sketch_last_error()
    assert lib.sketch_update(None, None, 1, 1, 0, 1) == _lib.SK_EINVAL
    assert lib.sketch_destroy(None) == _lib.SK_OK


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsketch.so not built")
def test_amplification_parameters_are_validated_without_gpu():
    from paper_2601_02019_amd import _lib
    lib = _lib.load()
    cfg = _lib.sketch_config()
    assert lib.sketch_config_init(ctypes.byref(cfg)) == 0
    assert (cfg.amplify_r, cfg.amplify_s) == (1, 0)
    cfg.d, cfg.ell, cfg.kind, cfg.window_N, cfg.R = 8, 4, _lib.SK_WINDOW, 10, 2.0
    h = ctypes.c_void_p()
    for r, s in [(0, 1), (17, 0), (2, -1), (2, 17)]:
        cfg.amplify_r, cfg.amplify_s = r, s
        assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
        assert b"amplify_r" in lib.sketch_last_error()
    cfg.kind, cfg.amplify_r, cfg.amplify_s = _lib.SK_PERSISTENT, 2, 1
    assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
    assert b"amplification" in lib.sketch_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsketch.so not built")
def test_p5_configuration_is_validated_without_gpu():
    from paper_2601_02019_amd import _lib
    lib = _lib.load()
    cfg = _lib.sketch_config()
    assert lib.sketch_config_init(ctypes.byref(cfg)) == 0
    assert cfg.sites == 0
    cfg.d, cfg.ell, cfg.kind = 8, 4, _lib.SK_P5
    h = ctypes.c_void_p()
    for m in (0, 4097):
        cfg.sites = m
        assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
        assert b"sites" in lib.sketch_last_error()
    st = (ctypes.c_int64 * 8)()
    assert lib.p5_stats(None, st) == _lib.SK_EINVAL
    assert lib.p5_update(None, None, None, 1, 8, 0, 1) == _lib.SK_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libsketch.so not built")
def test_cod_configuration_is_validated_without_gpu():
    from paper_2601_02019_amd import _lib
    lib = _lib.load()
    cfg = _lib.sketch_config()
    assert lib.sketch_config_init(ctypes.byref(cfg)) == 0
    cfg.d, cfg.ell, cfg.kind, cfg.window_N, cfg.theta = 8, 4, _lib.SK_COD, 10, 1.0
    h = ctypes.c_void_p()
    cfg.d_y = 0
    assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
    assert b"d_y" in lib.sketch_last_error()
    cfg.d_y, cfg.theta = 6, 0.0
    assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
    assert b"theta" in lib.sketch_last_error()
    cfg.theta, cfg.d, cfg.d_y = 1.0, 600, 700
    assert lib.sketch_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.SK_EINVAL
    assert lib.cod_update(None, None, 1, None, 1, 1, 0, 1) == _lib.SK_EINVAL
