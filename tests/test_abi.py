"""The C-ABI library loads and exports every entry point include/gfors.h declares
(no device work: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfors.h")
LIB = os.path.join(ROOT, "paper_2510_27117_amd", "libgfors.so")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gfors_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2510_27117_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_names_cover_header():
    from paper_2510_27117_amd import gfors
    assert sorted(gfors.EXPORTS) == declared_symbols()


def test_default_params_and_workspace_size(lib):
    from paper_2510_27117_amd import gfors
    p = gfors.default_params()
    assert p.sigma == 0.99 and p.K_max == 1024 and p.k_int == 100 and p.power_iters == 200
    L = gfors.load_library()
    nb = ctypes.c_size_t(0)
    assert L.gfors_workspace_bytes(2_000_000, 200_000, 0, 10_000_000, 0, 0, 1,
                                   ctypes.byref(p), ctypes.byref(nb)) == 0
    # candidates alone take n * K/64 * 8 bytes
    assert nb.value > 2_000_000 * 16 * 8
    # bad K_max is rejected with a message
    p.K_max = 100
    assert L.gfors_workspace_bytes(10, 1, 0, 1, 0, 0, 1, ctypes.byref(p), ctypes.byref(nb)) == -1
    assert b"K_max" in L.gfors_last_error()
    p.K_max = 1024
    assert L.gfors_workspace_bytes(0, 1, 0, 1, 0, 0, 1, ctypes.byref(p), ctypes.byref(nb)) == -1


def test_missing_library_fails_loudly(tmp_path):
    from paper_2510_27117_amd import gfors
    saved = gfors._lib
    gfors._lib = None
    try:
        with pytest.raises(RuntimeError):
            gfors.load_library(str(tmp_path / "nope.so"))
    finally:
        gfors._lib = saved
