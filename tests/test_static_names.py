"""Every name a function of the committed Python sources reads either is bound
in that function (or an enclosing one), at module level, or is a builtin: a
name left over from an edit (a NameError that only a rarely run mode of the
benchmark would reach) fails here, without running anything."""
import builtins
import os
import symtable

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ["bench.py", "__graft_entry__.py", "oracle/__init__.py"] + [
    os.path.join("paper_2605_25282_amd", f) for f in sorted(os.listdir(os.path.join(ROOT, "paper_2605_25282_amd")))
    if f.endswith(".py")]


def _unbound(path):
    with open(os.path.join(ROOT, path)) as f:
        top = symtable.symtable(f.read(), path, "exec")
    module = set(top.get_identifiers())
    bad = []

    def walk(t):
        for ch in t.get_children():
            if ch.get_type() == "function":
                for sym in ch.get_symbols():
                    n = sym.get_name()
                    if (sym.is_referenced() and sym.is_global() and not sym.is_declared_global()
                            and n not in module and not hasattr(builtins, n)):
                        bad.append(f"{ch.get_name()}:{n}")
            walk(ch)

    walk(top)
    return bad


@pytest.mark.parametrize("path", SOURCES)
def test_no_unbound_names(path):
    assert _unbound(path) == []


def test_the_check_sees_an_unbound_name():
    src = "def f():\n    return undefined_name + 1\n"
    t = symtable.symtable(src, "x.py", "exec")
    f = t.get_children()[0]
    sym = f.lookup("undefined_name")
    assert sym.is_global() and sym.is_referenced() and "undefined_name" not in t.get_identifiers()
