"""The C structs of include/kmvwave.h and their ctypes mirrors in the Python binding
agree field by field: same names in the same order, same offsets, same total size.
Offsets are taken from the header itself, compiled by the host C compiler
(offsetof), so a field appended to one side only, or a type changed on one side,
fails here on the CPU."""
import os
import re
import shutil
import subprocess
import tempfile

import ctypes as C
import pytest

from paper_2108_10946_amd import kmvwave as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kmvwave.h")
STRUCTS = {"kmv_options": K.kmv_options, "kmv_request": K.kmv_request, "kmv_result": K.kmv_result}


def header_fields():
    """{struct name: [field names in order]} from the header's typedef struct blocks."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", txt, flags=re.S):
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            # "type a, b, c" or "const double* x": names are the trailing identifiers
            head, *rest = [s.strip() for s in decl.split(",")]
            names.append(re.findall(r"(\w+)\s*$", head)[0])
            names += [re.findall(r"(\w+)\s*$", r)[0] for r in rest]
        out[name] = names
    return out


def test_header_and_binding_list_the_same_fields():
    hf = header_fields()
    for name, cls in STRUCTS.items():
        assert name in hf, name
        assert [f[0] for f in cls._fields_] == hf[name], name


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_offsets_and_sizes_match_the_compiled_header():
    hf = header_fields()
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in hf[name]:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "abi.c"), os.path.join(d, "abi")
        open(src, "w").write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c99", "-o", exe, src], check=True)
        res = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in res:
        if ln:
            s, f, v = ln.split()
            got[(s, f)] = int(v)
    for name, cls in STRUCTS.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f in hf[name]:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
