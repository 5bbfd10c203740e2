"""The oracle and the GPU path share no code: the package never names the oracle, the oracle
never imports the package, and the benchmark reaches the oracle only from its CPU-baseline
functions (CPU only)."""

import ast
import glob
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_0802_0748_amd")


def _imports(path):
    tree = ast.parse(open(path).read())
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            out += [a.name for a in node.names]
        elif isinstance(node, ast.ImportFrom) and node.module:
            out.append(node.module)
    return tree, out


def test_package_never_reaches_the_oracle():
    files = glob.glob(os.path.join(PKG, "*.py")) + glob.glob(os.path.join(PKG, "csrc", "*"))
    assert any(f.endswith("kernels.hip") for f in files)
    for f in files:
        if f.endswith((".o", ".so")):
            continue
        assert "oracle" not in open(f, errors="replace").read(), f


def test_oracle_never_imports_the_package():
    for f in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        _, mods = _imports(f)
        assert not any(m.startswith("paper_0802_0748_amd") for m in mods), f
    src = open(os.path.join(ROOT, "oracle", "scocg_oracle.c")).read()
    assert "#include \"" not in src  # system headers only


def test_benchmark_uses_the_oracle_only_for_its_cpu_baseline():
    tree, _ = _imports(os.path.join(ROOT, "bench.py"))
    users = set()
    for fn in ast.walk(tree):
        if isinstance(fn, (ast.FunctionDef, ast.AsyncFunctionDef)):
            for node in ast.walk(fn):
                if isinstance(node, ast.ImportFrom) and node.module and node.module.startswith("oracle"):
                    users.add(fn.name)
                if isinstance(node, ast.Import) and any(a.name.startswith("oracle") for a in node.names):
                    users.add(fn.name)
    assert users and all("cpu_baseline" in u for u in users), users
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    for n in top:
        names = [a.name for a in n.names] if isinstance(n, ast.Import) else [n.module or ""]
        assert not any(x.startswith("oracle") for x in names)
