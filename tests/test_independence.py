"""The oracle and the HIP path share no code (CPU only, static checks).

* Nothing in the package (Python binding, HIP sources, headers) imports or
  includes the oracle or the test helpers; the seeded input module imports
  neither side.
* The oracle imports nothing from the package but the seeded inputs.
* bench.py reaches the oracle only inside its cpu_baseline leg, and
  __graft_entry__.py only inside smoke(); bench.py may use the closed-form
  solutions, which reach no oracle code."""

import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2305_04711_amd")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def _imports(tree):
    """(module name, enclosing function name or None) for every import."""
    out = []

    def visit(node, fn):
        for ch in ast.iter_child_nodes(node):
            name = ch.name if isinstance(ch, (ast.FunctionDef, ast.AsyncFunctionDef)) else fn
            if isinstance(ch, ast.Import):
                out.extend((a.name, fn) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom):
                mod = ("." * ch.level) + (ch.module or "")
                out.append((mod, fn))
                out.extend(("%s.%s" % (mod, a.name), fn) for a in ch.names)
            visit(ch, name)

    visit(tree, None)
    return out


def test_package_does_not_reach_the_oracle():
    for path in _sources(PKG, (".py",)):
        tree = ast.parse(open(path).read())
        for mod, _ in _imports(tree):
            assert not re.match(r"(\.*)oracle\b", mod), (path, mod)
            assert "parity_helpers" not in mod and "closed_forms" not in mod, (path, mod)
    for path in _sources(PKG, (".hip", ".hpp", ".h", ".cpp")):
        text = open(path).read()
        for inc in re.findall(r'#include\s*[<"]([^>"]+)[>"]', text):
            assert "oracle" not in inc, (path, inc)


def test_inputs_module_imports_neither_side():
    tree = ast.parse(open(os.path.join(PKG, "inputs.py")).read())
    for mod, _ in _imports(tree):
        # torch only to evaluate the same fields on device tensors
        assert mod.split(".")[0] in ("numpy", "math", "torch", "__future__"), mod


def test_oracle_uses_only_the_seeded_inputs_from_the_package():
    for path in _sources(os.path.join(ROOT, "oracle"), (".py",)):
        tree = ast.parse(open(path).read())
        for mod, _ in _imports(tree):
            if mod.startswith("paper_2305_04711_amd"):
                assert mod in ("paper_2305_04711_amd", "paper_2305_04711_amd.inputs"), (path, mod)
            assert "torch" not in mod and "capi" not in mod and mod != "paper_2305_04711_amd.cpm", (path, mod)


def test_closed_forms_import_no_oracle():
    # tests/closed_forms.py holds analytic solutions written from the
    # mathematics; bench.py may use them to state errors against the closed
    # form, because they reach neither the oracle nor the parity helpers
    tree = ast.parse(open(os.path.join(ROOT, "tests", "closed_forms.py")).read())
    for mod, _ in _imports(tree):
        assert not mod.startswith("oracle") and "parity_helpers" not in mod, mod
        if mod.startswith("paper_2305_04711_amd"):
            assert mod in ("paper_2305_04711_amd", "paper_2305_04711_amd.inputs"), mod


def test_bench_and_entry_reach_the_oracle_only_where_allowed():
    for name, allowed in (("bench.py", {"cpu_baseline"}), ("__graft_entry__.py", {"smoke"})):
        tree = ast.parse(open(os.path.join(ROOT, name)).read())
        for mod, fn in _imports(tree):
            if mod.startswith("oracle") or "parity_helpers" in mod:
                assert fn in allowed, (name, mod, fn)
            if "closed_forms" in mod and name == "__graft_entry__.py":
                assert fn in allowed, (name, mod, fn)
