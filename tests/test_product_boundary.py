"""Host-side rules of the product path, checked without a GPU: one GPU only in the benchmark,
no route from the package to the oracle, and a loud failure when the HIP library is absent."""
import ast
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2512_06230_amd")


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no JSON line


def _imports(path):
    tree = ast.parse(open(path).read(), filename=path)
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                yield a.name
        elif isinstance(node, ast.ImportFrom):
            yield ("." * node.level) + (node.module or "")


@pytest.mark.parametrize("name", sorted(f for f in os.listdir(PKG) if f.endswith(".py")))
def test_package_never_imports_the_oracle(name):
    for mod in _imports(os.path.join(PKG, name)):
        assert "oracle" not in mod.split("."), (name, mod)


def test_missing_library_fails_loudly(tmp_path):
    # a fresh interpreter, so that no library is cached in the binding
    code = ("import paper_2512_06230_amd.glmb as G\n"
            "try:\n"
            "    G.load_library(%r)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    print('loaded')\n") % str(tmp_path / "libglmb.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("raised:") and "not built" in r.stdout
