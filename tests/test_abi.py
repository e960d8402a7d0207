"""The C ABI without a GPU: the library loads, exports every symbol that
include/gm.h declares, and rejects bad arguments on the host before touching
a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2302_05176_amd import _native, build
    if not build.up_to_date():
        build.build(force=True)
    return _native.load()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gm_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for s in ("gm_sketch", "gm_sketch_plain", "gm_sketch_batched", "gm_sketch_update",
              "gm_jaccard_est",
              "gm_jaccard_est_pairs", "gm_wcard_est", "gm_merge", "gm_setops", "gm_get_data_errors",
              "gm_lsh_build", "gm_lsh_query", "gm_lsh_free", "gm_release"):
        assert s in syms


def test_library_exports_every_declared_symbol(lib):
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_host_side_argument_validation(lib):
    from paper_2302_05176_amd import _native as N
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x1000)
    u = ctypes.c_uint64(1)
    # nvec < 0, k out of range, null pointers: rejected before any device call
    assert lib.gm_sketch(fake, fake, fake, -1, 8, u, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch(fake, fake, fake, 1, 0, u, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch(fake, fake, fake, 1, 4097, u, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch(nul, fake, fake, 1, 8, u, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch_plain(fake, fake, fake, 1, 8, u, nul, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch_update(fake, fake, fake, 1, 0, u, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch_update(fake, fake, fake, 1, 8, u, fake, nul, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch_update(nul, nul, nul, 0, 8, u, nul, nul, nul) == N.GM_OK
    assert lib.gm_sketch_batched(fake, fake, fake, 1, nul, fake, 8, u, 0, fake, fake,
                                 nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_sketch_batched(fake, fake, fake, 1, fake, fake, 8, u, 7, fake, fake,
                                 nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_wcard_est(fake, 1, 1, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_setops(fake, fake, fake, fake, 1, 1, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_setops(fake, fake, fake, fake, -1, 8, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_setops(fake, nul, fake, fake, 1, 8, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_setops(nul, nul, nul, nul, 0, 8, nul, nul) == N.GM_OK
    assert lib.gm_jaccard_est(fake, fake, -1, 8, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_jaccard_est_pairs(fake, 1, 8, nul, fake, 1, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_merge(fake, fake, 0, 8, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_get_data_errors(None, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_rate_probe(2, 64, 8, u, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_rate_probe(0, 64, 0, u, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_rate_probe(0, 64, 8, u, nul, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_rate_probe(1, 0, 8, u, nul, nul) == N.GM_OK
    h = ctypes.c_void_p()
    assert lib.gm_lsh_build(nul, 10, 16, 4, 4, ctypes.byref(h), nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_lsh_build(fake, 10, 16, 0, 4, ctypes.byref(h), nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_lsh_build(fake, 10, 16, 65, 1, ctypes.byref(h), nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_lsh_build(fake, 10, 16, 5, 4, ctypes.byref(h), nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_lsh_build(fake, 10, 16, 4, 4, None, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_lsh_build(fake, 1 << 30, 64, 16, 4, ctypes.byref(h), nul) == N.GM_ERR_UNSUPPORTED
    assert not h.value
    assert lib.gm_lsh_query(nul, fake, 1, 4, fake, fake, nul) == N.GM_ERR_INVALID_ARG
    assert lib.gm_lsh_info(nul, None, None, None, None) == N.GM_ERR_INVALID_ARG
    lib.gm_lsh_free(nul)
    # empty work is a no-op
    assert lib.gm_sketch(nul, nul, nul, 0, 8, u, nul, nul, nul) == N.GM_OK
    assert lib.gm_jaccard_est(nul, nul, 0, 8, nul, nul) == N.GM_OK


def test_options_validation(lib):
    from paper_2302_05176_amd import _native as N
    assert lib.gm_set_option(0, 7) == N.GM_ERR_INVALID_ARG
    assert lib.gm_set_option(0, 30) == N.GM_ERR_INVALID_ARG
    assert lib.gm_set_option(2, 17) == N.GM_ERR_INVALID_ARG
    assert lib.gm_set_option(3, 3) == N.GM_ERR_INVALID_ARG
    assert lib.gm_set_option(99, 1) == N.GM_ERR_INVALID_ARG
    assert lib.gm_set_option(0, 31) == N.GM_OK
    assert lib.gm_set_option(3, 4) == N.GM_OK
    # timing: 0 off, 1 every launch, 2 the sketch kernels only
    assert lib.gm_set_option(7, 3) == N.GM_ERR_INVALID_ARG
    assert lib.gm_set_option(7, -1) == N.GM_ERR_INVALID_ARG
    for level in (2, 1, 0):
        assert lib.gm_set_option(7, level) == N.GM_OK
    # registers-per-block tiling: 0 or 2^m - 1, m = 4..15
    for bad in (7, 100, 2048, 65535, -1):
        assert lib.gm_set_option(8, bad) == N.GM_ERR_INVALID_ARG
    for good in (0, 15, 511, 8191, 32767, 2047):
        assert lib.gm_set_option(8, good) == N.GM_OK
    assert lib.gm_status_string(1) == b"invalid argument"


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2302_05176_amd import _native, build
    monkeypatch.setattr(build, "LIB", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(ImportError):
        _native.load()
