"""The product path and the oracle share no code: no module of the package
imports the oracle, no HIP/C source includes anything from it, and no oracle
module imports the package (the seeded input generators, which hold none of
the method's arithmetic, are handed to both sides by the tests)."""
import ast
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1708_07853_amd")


def _imports(path):
    tree = ast.parse(open(path).read(), path)
    out = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out.update(a.name.split(".")[0] for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module and node.level == 0:
            out.add(node.module.split(".")[0])
    return out


def _files(top, exts):
    for d, _, names in os.walk(top):
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def test_package_never_imports_the_oracle():
    files = list(_files(PKG, (".py",)))
    assert files
    for f in files:
        assert "oracle" not in _imports(f), f


def test_native_sources_reference_no_oracle_file():
    files = list(_files(PKG, (".hip", ".cpp", ".h"))) + list(_files(os.path.join(ROOT, "include"), (".h",)))
    assert len(files) >= 6
    for f in files:
        for line in open(f):
            if line.lstrip().startswith("#include"):
                assert "oracle" not in line, (f, line)


def test_oracle_never_imports_the_package():
    files = list(_files(os.path.join(ROOT, "oracle"), (".py",)))
    assert files
    for f in files:
        assert "paper_1708_07853_amd" not in _imports(f), f
        assert "torch" not in _imports(f), f
