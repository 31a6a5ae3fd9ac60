"""The ctypes structures of the binding match the C header byte for byte.

Every `typedef struct { ... } name;` of include/lhf.h is compiled with gcc in a
small program that prints sizeof(name) and offsetof(name, field) for each
field; the ctypes class of the same name in paper_1702_00339_amd/lhf.py must
list the same fields in the same order at the same offsets, with the same
total size.  Runs on the CPU (gcc only; the library is not loaded)."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lhf.h")


def header_structs():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct \{(.*?)\}\s*(\w+);", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            # "type a", or "type a, b[3], c": every comma part ends with a name
            for part in decl.split(","):
                m = re.match(r".*?(\w+)\s*(\[\s*\w+\s*\])?$", part.strip())
                assert m, decl
                fields.append(m.group(1))
        out[name] = fields
    return out


def binding_classes():
    import importlib.util
    spec = importlib.util.spec_from_file_location("lhf_binding", os.path.join(ROOT, "paper_1702_00339_amd", "lhf.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return {k: v for k, v in vars(mod).items() if isinstance(v, type) and issubclass(v, C.Structure)}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_binding_structs_match_header_layout(tmp_path):
    structs = header_structs()
    assert {"lhf_cell", "lhf_lattice", "lhf_sizes", "lhf_step_args", "lhf_tuning", "lhf_box",
            "lhf_toeplitz_info"} <= set(structs)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lhf.h"', "int main(void) {"]
    for name, fields in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    classes = binding_classes()
    for name, fields in structs.items():
        assert name in classes, f"no ctypes class for {name}"
        cls = classes[name]
        assert [f for f, _ in cls._fields_] == fields, name
        assert C.sizeof(cls) == got[(name, "size")], name
        for f in fields:
            assert getattr(cls, f).offset == got[(name, f)], f"{name}.{f}"
