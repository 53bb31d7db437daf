"""The ctypes mirrors of the C ABI's structs have the C layout: a small C
program compiled against include/se.h with the host compiler prints every
field's offset and each struct's size, and the ctypes classes must agree
(a mismatch would let the library write past a Python-owned buffer)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1712_04732_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"se_params": L.se_params, "se_plan_info": L.se_plan_info, "se_stage_record": L.se_stage_record,
           "se_tune_report": L.se_tune_report}


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "se.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{name} {fname} %zu\\n", offsetof({name}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for ln in out.splitlines():
        name, field, val = ln.split()
        table[(name, field)] = int(val)
    return table


def test_ctypes_structs_match_the_c_layout(tmp_path):
    c = _c_layout(tmp_path)
    for name, cls in STRUCTS.items():
        assert ctypes.sizeof(cls) == c[(name, "sizeof")], name
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == c[(name, fname)], (name, fname)
