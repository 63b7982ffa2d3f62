"""The ctypes mirrors of the structures in include/bc.h have the C layout.

A small C program built with the host compiler against the header prints the
size of every structure and the offset of every field; the binding's
``ctypes.Structure`` classes must agree field by field (a field added to the
header but not to the binding, or in another order, fails here).  No GPU.
"""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import paper_1710_07769_amd as bc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["bc_opts", "bc_stats", "rip_graph_t", "rip_opts"]


def c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "bc.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(bc, name)
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));'
                         % (name, field, name, field))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return dict((k, int(v)) for k, v in (ln.rsplit(" ", 1) for ln in out.splitlines()))


def test_struct_layouts_match_header(tmp_path):
    got = c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(bc, name)
        assert got[name + " size"] == C.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got["%s.%s" % (name, field)] == getattr(cls, field).offset, (name, field)
