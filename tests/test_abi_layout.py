"""The ctypes structures of the Python binding against the C declarations of
include/rts.h: a small C program built with the host compiler prints every
structure's size and every field's offset, which must equal the binding's.
(Host compiler only; no GPU.)"""
import os
import shutil
import subprocess

import pytest

from paper_2107_08145_amd import rts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("rts_grid", rts.Grid), ("rts_desc", rts.Desc), ("rts_inputs", rts.Inputs),
         ("rts_outputs", rts.Outputs), ("rts_seeds", rts.Seeds), ("rts_grads", rts.Grads),
         ("rts_schedule", rts.Schedule)]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "rts.h"', "int main(void) {"]
    for cname, py in PAIRS:
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    src, exe = d / "layout.c", d / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {k: int(v) for k, v in (l.split() for l in out.splitlines())}


@pytest.mark.parametrize("cname,py", PAIRS, ids=[c for c, _ in PAIRS])
def test_struct_layout_matches_header(c_layout, cname, py):
    import ctypes
    assert ctypes.sizeof(py) == c_layout[cname], cname
    for f, _ in py._fields_:
        assert getattr(py, f).offset == c_layout[f"{cname}.{f}"], (cname, f)
