"""The C-ABI library loads and exports every entry point include/glmb.h declares (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glmb.h")
LIB = os.path.join(ROOT, "paper_2512_06230_amd", "libglmb.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(glmb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("glmb_predict", "glmb_update", "glmb_truncate", "glmb_estimate", "glmb_create", "glmb_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libglmb.so is not built (run python paper_2512_06230_amd/build.py)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_same_symbols():
    from paper_2512_06230_amd import glmb
    assert sorted(glmb.EXPORTS) == declared()


def test_status_strings_without_gpu():
    from paper_2512_06230_amd import glmb
    L = glmb.load_library()
    assert L.glmb_status_string(0) == b"ok"
    assert L.glmb_status_string(-2) == b"capacity exceeded"
    # argument errors are reported before any device work
    assert L.glmb_create(None, 0, None, None) == glmb.GLMB_E_ARG
    assert L.glmb_destroy(None) == glmb.GLMB_E_ARG
    assert L.glmb_update(None, 0, None, 0) == glmb.GLMB_E_ARG
