"""CPU checks of the library's word-level helpers (``csrc/s5_word.h``).

The helpers that the kernels use to build keys, compare them and descend the
splitter tree are compiled for the host and compared with byte-level
definitions: key extraction (also next to an inaccessible page, so a read past
a string's last aligned word would fault), lcp of keys, the level-order /
in-order index map, recursive splitter selection and classification versus
``2 * lower_bound + [equal]``, the workgroup renumbering over the XCDs (a
bijection), and the worked tree of Figure 1
(``tests/golden/fig1_ternary_v3.txt``).
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_word_helpers(tmp_path):
    exe = tmp_path / "word_helpers_test"
    subprocess.check_call([HIPCC, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                           "-I", os.path.join(ROOT, "paper_1305_1157_amd", "csrc"),
                           os.path.join(ROOT, "tests", "cpu", "word_helpers_test.cpp"),
                           "-o", str(exe)], stderr=subprocess.DEVNULL)
    r = subprocess.run([str(exe), os.path.join(ROOT, "tests", "golden", "fig1_ternary_v3.txt")],
                       stdout=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout
