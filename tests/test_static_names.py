"""Every name a function of the Python sources reads resolves: a local, an enclosing
scope's, a module-level definition or import, or a builtin (catches a mistyped name in
a code path that only the GPU runs)."""
import builtins
import glob
import os
import symtable

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = sorted([os.path.join(ROOT, "bench.py"), os.path.join(ROOT, "__graft_entry__.py")] +
               glob.glob(os.path.join(ROOT, "paper_1410_1921_amd", "*.py")) +
               glob.glob(os.path.join(ROOT, "oracle", "*.py")))


def unresolved(path):
    src = open(path).read()
    top = symtable.symtable(src, path, "exec")
    defined = {s.get_name() for s in top.get_symbols()
               if s.is_assigned() or s.is_imported() or s.is_namespace()}
    defined |= {"__file__", "__name__", "__doc__", "__spec__", "__package__"}
    star = "import *" in src
    bad = []

    def walk(t):
        for s in t.get_symbols():
            if t.get_type() == "module":
                continue
            if s.is_referenced() and s.is_global() and not s.is_declared_global():
                n = s.get_name()
                if n not in defined and not hasattr(builtins, n) and not star:
                    bad.append(f"{t.get_name()}: {n}")
        for c in t.get_children():
            walk(c)

    walk(top)
    return bad


@pytest.mark.parametrize("path", FILES, ids=[os.path.relpath(f, ROOT) for f in FILES])
def test_names_resolve(path):
    assert unresolved(path) == []
