"""The ctypes structures of the binding against the C header: every field's
offset and every structure's size, as a C compiler lays them out (gcc on the
header alone; no library call, no GPU).  A field appended to the header but not
to the binding, or the other way round, fails here."""
import ctypes
import os
import shutil
import subprocess

import pytest

zolo = pytest.importorskip("paper_1701_08935_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["zolo_filter_coeffs", "zolo_opts", "zolo_stats", "zolo_kernel_profile", "zolo_query_info",
           "zolo_server_info", "zolo_filter_stats"]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "zolo.h"', "int main(void) {"]
    for s in STRUCTS:
        cls = getattr(zolo, s)
        lines.append(f'  printf("{s} sizeof %zu\\n", sizeof({s}));')
        for name, _ in cls._fields_:
            lines.append(f'  printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return table


@pytest.mark.parametrize("name", STRUCTS)
def test_struct_layout_matches_header(c_layout, name):
    cls = getattr(zolo, name)
    assert ctypes.sizeof(cls) == c_layout[(name, "sizeof")], name
    for field, _ in cls._fields_:
        assert getattr(cls, field).offset == c_layout[(name, field)], f"{name}.{field}"
