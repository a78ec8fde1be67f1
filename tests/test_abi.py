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


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and field offsets of the ABI structs, from a C program built against the header."""
    import subprocess
    from paper_2512_06230_amd import glmb
    src = tmp_path / "sz.c"
    fields = {"glmb_params": glmb.Params, "glmb_state_host": glmb.StateHost, "glmb_step_stats": glmb.StepStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "glmb.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in py._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines.append("return 0; }")
    src.write_text("\n".join(lines))
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, py in fields.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out["%s.%s" % (cname, f)]) == getattr(py, f).offset, (cname, f)


def test_new_entry_points_reject_null_context():
    from paper_2512_06230_amd import glmb
    L = glmb.load_library()
    assert L.glmb_set_proposal(None, None, None, 0.5, 0) == glmb.GLMB_E_ARG
    assert L.glmb_pair_features(None, 0, None, 0, 0, None, None, None, None, None) == glmb.GLMB_E_ARG
    assert L.glmb_proposal_lost(None, 0, None, 0, 1, None, None) == glmb.GLMB_E_ARG
    assert L.glmb_mlp_forward(None, None, None, None, 0, None) == glmb.GLMB_E_ARG
    assert L.glmb_mlp_grad(None, None, None, None, None, None, 1, None, None) == glmb.GLMB_E_ARG
    assert L.glmb_mlp_adam(None, None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8) == glmb.GLMB_E_ARG
