"""Every entry point the binding declares has, in include/tbh.h, a prototype
with the same number of parameters, each of the same kind (pointer, 32-bit
integer, 64-bit integer, double): a parameter added or retyped on one side
only fails here.  CPU only (reads the header; loads nothing)."""
import ctypes as C
import os
import re

import paper_1003_4570_amd as tbh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_prototypes():
    text = open(os.path.join(ROOT, "include", "tbh.h")).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    protos = {}
    for m in re.finditer(r"(?:^|\n)\s*(?:const\s+)?(?:int|char\s*\*|const\s+char\s*\*)\s*\**\s*(tbh_\w+)\s*\(([^;{]*?)\)\s*;",
                         text):
        protos[m.group(1)] = [p.strip() for p in m.group(2).replace("\n", " ").split(",")
                              if p.strip() and p.strip() != "void"]
    return protos


def _c_kind(param):
    if "*" in param or "[" in param:
        return "ptr"
    if re.search(r"\bint64_t\b", param):
        return "i64"
    if re.search(r"\b(int32_t|int)\b", param):
        return "i32"
    if re.search(r"\bdouble\b", param):
        return "f64"
    raise AssertionError(f"unclassified parameter {param!r}")


def _py_kind(t):
    if t in (C.c_void_p, C.c_char_p) or (isinstance(t, type) and issubclass(t, C._Pointer)):
        return "ptr"
    if t in (C.c_int32, C.c_int) and C.sizeof(t) == 4:
        return "i32"
    if t is C.c_int64:
        return "i64"
    if t is C.c_double:
        return "f64"
    raise AssertionError(f"unclassified ctypes type {t!r}")


def test_every_bound_entry_point_matches_its_prototype():
    protos = _header_prototypes()
    assert len(protos) >= 40
    for name, _, args in tbh._SIGS:
        assert name in protos, f"{name} has no prototype in tbh.h"
        want = [_c_kind(p) for p in protos[name]]
        got = [_py_kind(a) for a in args]
        assert got == want, (name, got, want)


def test_every_prototype_is_bound():
    bound = {s[0] for s in tbh._SIGS}
    missing = sorted(set(_header_prototypes()) - bound)
    assert not missing, missing
