"""The oracle and the GPU path share no code: no Python module of one imports
the other, the seeded input generators import neither, the C and HIP sources
include nothing across the boundary, and outside tests/ the oracle is reached
only from the CPU-baseline leg of bench.py, from smoke(), and from build(),
which compiles the oracle's C library without running it."""
import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = "paper_2005_09870_amd"


def _imports(path):
    """(top-level module name, enclosing function name or None) of every import."""
    tree = ast.parse(open(path).read(), filename=path)
    out = []

    def visit(node, fn):
        for ch in ast.iter_child_nodes(node):
            name = ch.name if isinstance(ch, (ast.FunctionDef, ast.AsyncFunctionDef)) else fn
            if isinstance(ch, ast.Import):
                out.extend((a.name.split(".")[0], fn) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom) and ch.module and ch.level == 0:
                out.append((ch.module.split(".")[0], fn))
            visit(ch, name)

    visit(tree, None)
    return out


def _py(folder):
    d = os.path.join(ROOT, folder)
    return [os.path.join(d, f) for f in sorted(os.listdir(d)) if f.endswith(".py")]


def test_oracle_does_not_import_the_gpu_package():
    for f in _py("oracle"):
        assert all(m != PKG for m, _ in _imports(f)), f


def test_gpu_package_does_not_import_the_oracle():
    for f in _py(PKG):
        assert all(m != "oracle" for m, _ in _imports(f)), f


def test_input_generators_import_neither():
    for f in _py("syninputs"):
        assert all(m not in ("oracle", PKG) for m, _ in _imports(f)), f


def test_oracle_reached_only_from_cpu_baseline_and_smoke():
    for f, allowed in ((os.path.join(ROOT, "bench.py"), {"cpu_baseline"}),
                       (os.path.join(ROOT, "__graft_entry__.py"), {"smoke", "build"})):
        for m, fn in _imports(f):
            if m == "oracle":
                assert fn in allowed, (f, fn)


def test_native_sources_do_not_cross_the_boundary():
    csrc = os.path.join(ROOT, PKG, "csrc")
    inc = re.compile(r'#include\s+"([^"]+)"')
    for f in os.listdir(csrc):
        for h in inc.findall(open(os.path.join(csrc, f)).read()):
            assert "oracle" not in h, (f, h)
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h")):
            for h in inc.findall(open(os.path.join(ROOT, "oracle", f)).read()):
                assert "pd" not in h and PKG not in h, (f, h)
