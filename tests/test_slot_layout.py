"""Host check of the per-side output slots that the CG applies store into
(every element row has its own in-range slot; each node's slot sum reads
exactly its rows), compiled from the library's layout header."""

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_slot_layout(tmp_path):
    exe = str(tmp_path / "slot_layout_check")
    subprocess.run([HIPCC, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
                    "-I" + os.path.join(ROOT, "paper_1601_08179_amd", "csrc"),
                    os.path.join(HERE, "slot_layout_check.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
