"""The oracle and the HIP path share nothing: the package never imports,
links or runs the oracle, the oracle never uses the package, and the only
module both sides use is the seeded input generator (which holds none of the
sort's arithmetic)."""
import ast
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1305_1157_amd")


def imported_modules(path):
    tree = ast.parse(open(path).read(), path)
    mods = set()
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            mods.update(a.name for a in node.names)
        elif isinstance(node, ast.ImportFrom) and node.module:
            mods.add(node.module)
            mods.update(f"{node.module}.{a.name}" for a in node.names)
    return mods


def test_package_never_uses_the_oracle():
    for path in glob.glob(os.path.join(PKG, "**", "*.py"), recursive=True):
        assert not any(m == "oracle" or m.startswith("oracle.") for m in imported_modules(path)), path
    for path in glob.glob(os.path.join(PKG, "csrc", "*")):
        text = open(path).read()
        assert not re.search(r'#include\s+[<"][^>"]*oracle', text), path
        assert "s5_oracle" not in text, path
    build = open(os.path.join(PKG, "build.py")).read()
    assert "oracle" not in build


def test_oracle_never_uses_the_package():
    for path in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        mods = imported_modules(path)
        assert not any(m.startswith("paper_1305_1157_amd") for m in mods), path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*.c")):
        text = open(path).read()
        assert "s5_internal" not in text and "s5_word" not in text and "csrc" not in text, path


def test_oracle_callers():
    """Only the tests, the smoke check and the benchmark's CPU baseline use the oracle."""
    allowed = {os.path.join(ROOT, "__graft_entry__.py"), os.path.join(ROOT, "bench.py")}
    for path in glob.glob(os.path.join(ROOT, "*.py")):
        mods = imported_modules(path)
        if any(m == "oracle" or m.startswith("oracle.") for m in mods):
            assert path in allowed, path
    bench = open(os.path.join(ROOT, "bench.py")).read()
    # calls into the oracle and its imports
    uses = [m.start() for m in re.finditer(r"\boracle\.|import oracle\b", bench)]
    spans = []  # the CPU-baseline functions: cpu_baseline and cpu_baseline_sets
    for m in re.finditer(r"\ndef cpu_baseline\w*\(", bench):
        end = bench.index("\ndef ", m.start() + 1)
        spans.append((m.start(), end))
    assert len(spans) == 2 and uses
    assert all(any(a < u < b for a, b in spans) for u in uses), \
        "bench.py uses the oracle outside its CPU baselines"
