"""The Python binding's ctypes structures against the C header's structs:
every field's offset and every struct's size, as the C compiler lays them
out (host only: compiles a tiny C program against include/stokes_ifmm.h)."""
import os
import shutil
import subprocess

import pytest

from paper_1609_04484_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = {
    "sbie_geom": L.SbieGeom,
    "ifmm_params": L.IfmmParams,
    "ifmm_stats": L.IfmmStats,
    "gmres_params": L.GmresParams,
    "gmres_result": L.GmresResult,
    "gmres_member": L.GmresMember,
    "fmm_params": L.FmmParams,
    "fmm_stats": L.FmmStats,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "stokes_ifmm.h"', "int main(void) {"]
    for cname, cls in PAIRS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        cname, field, value = line.split()
        table[(cname, field)] = int(value)
    return table


@pytest.mark.parametrize("cname", sorted(PAIRS))
def test_struct_matches_header(c_layout, cname):
    cls = PAIRS[cname]
    assert ctypes_size(cls) == c_layout[(cname, "size")]
    for fname, _ in cls._fields_:
        assert getattr(cls, fname).offset == c_layout[(cname, fname)], fname


def ctypes_size(cls):
    import ctypes
    return ctypes.sizeof(cls)
