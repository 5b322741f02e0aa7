"""The ctypes structures of the binding have the layout of the C header:
a small C program built from include/pf.h prints every field's offset and
every structure's size, and they must equal the ctypes ones (no GPU)."""

import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2011_11880_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "pf_network": capi.pf_network,
    "pf_schedule": capi.pf_schedule,
    "pf_setup_opts": capi.pf_setup_opts,
    "pf_batch_spec": capi.pf_batch_spec,
    "pf_info_t": capi.pf_info_t,
    "pf_newton_opts": capi.pf_newton_opts,
    "pf_newton_report": capi.pf_newton_report,
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structures_match_header(tmp_path):
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pf.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = str(tmp_path / "layout")
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Werror", "-I",
                           os.path.join(ROOT, "include"), str(src), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        name, what, val = line.split()
        got[(name, what)] = int(val)
    for name, cls in STRUCTS.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
