"""The ctypes structures of the binding have the C layout of include/dg.h:
a small C program built with the host compiler against the header prints
sizeof and offsetof of every field, and the binding's structures must
match them exactly (same field names, same offsets, same sizes).  CPU only.
"""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dg():
    from paper_2110_01409_amd import dg as _dg
    return _dg


def _structs(dg):
    out = {}
    for name in dir(dg):
        obj = getattr(dg, name)
        if isinstance(obj, type) and issubclass(obj, C.Structure) and name.startswith("dg_") and obj._fields_:
            out[name] = obj
    return out


def test_binding_structs_match_header(dg, tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = _structs(dg)
    assert {"dg_stats", "dg_graph_info", "dg_plan_info", "dg_graph_opts", "dg_set_opts"} <= set(structs)
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "dg.h"', "int main(void) {"]
    for name, st in sorted(structs.items()):
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for fname, _ in st._fields_:
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr  # a field the header lacks fails here
    got = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout.split("\n")
    c_layout = {}
    for line in filter(None, got):
        name, field, value = line.split()
        c_layout[(name, field)] = int(value)
    for name, st in structs.items():
        assert C.sizeof(st) == c_layout[(name, "sizeof")], name
        for fname, _ in st._fields_:
            assert getattr(st, fname).offset == c_layout[(name, fname)], (name, fname)
