"""The ctypes structures of the Python binding have the layout that
include/tbh.h gives them: gcc compiles a probe that prints sizeof of every
option/report struct and offsetof of each field the binding declares, and
the binding's offsets and sizes must be the same (a field added, dropped or
reordered on one side only fails here).  CPU only: gcc, no GPU."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_1003_4570_amd as tbh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = sorted(n for n in dir(tbh) if n.startswith("tbh_") and isinstance(getattr(tbh, n), type)
                 and issubclass(getattr(tbh, n), ctypes.Structure))


def test_binding_declares_the_option_and_report_structs():
    for name in ("tbh_scf_opts", "tbh_scf_report", "tbh_build_opts", "tbh_lanczos_opts", "tbh_filter_opts"):
        assert name in STRUCTS


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match_the_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "tbh.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'    printf("{s} . %zu\\n", sizeof({s}));')
        for field, _ in getattr(tbh, s)._fields_:
            lines.append(f'    printf("{s} {field} %zu\\n", offsetof({s}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    c = {}
    for line in out.splitlines():
        s, field, v = line.split()
        c[(s, field)] = int(v)
    for s in STRUCTS:
        cls = getattr(tbh, s)
        assert ctypes.sizeof(cls) == c[(s, ".")], (s, ctypes.sizeof(cls), c[(s, ".")])
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c[(s, field)], (s, field, getattr(cls, field).offset, c[(s, field)])
