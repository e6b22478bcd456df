"""The binding's ctypes structures lay out their fields as include/mitopk.h
does: a C program built against the header prints each struct's size and the
offset of every field the binding names, and both must agree (a field added on
one side only, or reordered, fails here rather than corrupting a call)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2601_19911_amd as tk
from paper_2601_19911_amd import batched, join, serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = [tk.tk_info, tk.tk_tuning, batched.tk_plan_params, join.tk_join_table,
           serve.tk_cost_model, serve.tk_server_cfg, serve.tk_req_info, serve.tk_server_counters]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "mitopk.h"', "int main(void) {"]
    for s in STRUCTS:
        n = s.__name__
        lines.append(f'  printf("{n} size %zu\\n", sizeof({n}));')
        for f in s._fields_:
            lines.append(f'  printf("{n} {f[0]} %zu\\n", offsetof({n}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        name, field, value = line.split()
        table[(name, field)] = int(value)
    return table


@pytest.mark.parametrize("struct", STRUCTS, ids=lambda s: s.__name__)
def test_struct_matches_header(struct, c_layout):
    n = struct.__name__
    assert ctypes.sizeof(struct) == c_layout[(n, "size")], f"{n}: size differs from the header"
    for f in struct._fields_:
        assert getattr(struct, f[0]).offset == c_layout[(n, f[0])], f"{n}.{f[0]}: offset differs"
