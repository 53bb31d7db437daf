"""Properties of the gfx950 device code, checked on its assembly (CPU only).

A register array indexed with a run-time value is lowered to indexed VGPR
moves; when such an access is guarded by a range test, the compiler may
if-convert it into an unconditional indexed read whose index is out of range
(outside the wave's registers), which faults the GPU.  The kernels keep every
register array index a compile-time constant; this test holds them to it.
"""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_1712_04732_amd"))


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    import build_lib as b
    text = []
    for src in (f for f in b.SOURCES if f.endswith(".hip")):
        out = tmp_path_factory.mktemp("asm") / (src + ".s")
        cmd = [b.HIPCC, *[f for f in b.FLAGS if f != "-fPIC"], "--cuda-device-only", "-S", "-x", "hip",
               os.path.join(b.CSRC, src), "-o", str(out)]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("hipcc unavailable: " + r.stderr[-300:])
        text.append(out.read_text())
    return "\n".join(text)


def test_no_indexed_register_access(device_asm):
    hits = re.findall(r"^\s+(s_set_gpr_idx_on|v_movrel\w*|s_movrel\w*)\b", device_asm, re.M)
    assert not hits, f"{len(hits)} indexed register accesses"


def test_no_scratch_memory(device_asm):
    assert not re.search(r"^\s+scratch_(load|store)", device_asm, re.M)

