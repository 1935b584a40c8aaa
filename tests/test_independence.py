"""Structural checks on the CPU: the oracle and the GPU path share no code, the
product path never reaches the oracle, and the shared input generator holds
none of the method's arithmetic."""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2501_02747_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _files(top, exts):
    for d, _, names in os.walk(top):
        if "__pycache__" in d:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def _imports(path):
    tree = ast.parse(open(path).read())
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out |= {a.name.split(".")[0] for a in node.names}
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.add(node.module.split(".")[0])
    return out


def test_package_never_imports_the_oracle():
    for f in _files(PKG, (".py",)):
        assert "oracle" not in _imports(f), f


def test_oracle_never_imports_the_package():
    for f in _files(ORACLE, (".py",)):
        assert "paper_2501_02747_amd" not in _imports(f), f


def test_native_sources_share_no_file():
    """The C oracle and the HIP library include nothing from each other's folder."""
    inc = re.compile(r'#\s*include\s*[<"]([^>"]+)[>"]')
    hip = list(_files(os.path.join(PKG, "csrc"), (".hip", ".h", ".cpp")))
    ora = list(_files(ORACLE, (".c", ".h")))
    hip_names = {os.path.basename(f) for f in hip}
    ora_names = {os.path.basename(f) for f in ora}
    for f in ora:
        for m in inc.findall(open(f).read()):
            assert os.path.basename(m) not in hip_names and "ivm.h" not in m, (f, m)
    for f in hip:
        for m in inc.findall(open(f).read()):
            assert os.path.basename(m) not in ora_names, (f, m)


def test_generator_holds_no_method_arithmetic():
    """scenegen imports neither side, and names none of the visibility steps."""
    src = os.path.join(ROOT, "scenegen", "__init__.py")
    assert not ({"oracle", "paper_2501_02747_amd"} & _imports(src))
    text = open(src).read()
    for word in ("segment_clear", "segtri", "any_hit", "orient(", "visible_pairs"):
        assert word not in text, word


def test_product_path_fails_loudly_without_library_or_gpu():
    """No fallback: a missing library raises on load, and a scene cannot be built
    without a visible GPU (this container has none)."""
    import subprocess
    import sys
    code = ("import paper_2501_02747_amd as p\n"
            "try:\n    p.load_library('/nonexistent/libivm.so')\nexcept ImportError:\n    print('raised')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.stdout.strip() == "raised", r.stderr
    import torch
    if not torch.cuda.is_available():
        import pytest
        import paper_2501_02747_amd as ivm
        import scenegen as sg
        s = sg.gen_c1(1, n_snap=1)
        with pytest.raises(RuntimeError):
            ivm.GpuScene.from_scene(s)
