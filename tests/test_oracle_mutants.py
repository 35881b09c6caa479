"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle's C source, plants one plausible mistake, builds
the copy with gcc (CPU only) and runs the same pins as ``test_oracle.py``
against it; at least one pin must fail.
"""
import ctypes
import os
import random
import subprocess

import numpy as np
import pytest

from paper_1305_1157_amd import gen
from test_oracle import (TINY_ALPHABET, brute_D, lib_lcp, lib_sorted_perm,
                         rand_strings)

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "s5_oracle.c")

MUTANTS = {
    "ties_reversed": [("if (*s == 0) return a < b;", "if (*s == 0) return a > b;"),
                      ("return (x > y) - (x < y);", "return (x < y) - (x > y);")],
    "signed_bytes": [("if (*s != *t) return *s < *t;",
                      "if (*s != *t) return (int8_t)*s < (int8_t)*t;"),
                     ("return chars[offsets[i] + depth];",
                      "return (uint8_t)(chars[offsets[i] + depth] ^ 0x80);")],
    "lcp_counts_terminator": [("while (s[k] == t[k] && s[k] != 0) ++k;",
                               "while (s[k] == t[k] && s[k] != 0) ++k;\n    if (s[k] == t[k]) ++k;")],
    "D_no_plus_one": [("uint64_t m = (l > r ? l : r) + 1;", "uint64_t m = (l > r ? l : r);")],
    "D_left_neighbour_only": [("uint64_t m = (l > r ? l : r) + 1;", "uint64_t m = l + 1;")],
    "equal_part_not_refined": [("st[top++] = (task_t){lt, gt, t.depth + 1};", "")],
    "pivot_partition_sign": [("if (x < c)", "if (x > c)"), ("else if (x > c)", "else if (x < c)")],
}


def build_mutant(tmp_path, name):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert old in src, (name, old)
        src = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.oracle_sort.argtypes = [P, P, ctypes.c_uint32, P, P]
    lib.oracle_dist_prefix.argtypes = [P, P, P, P, ctypes.c_uint64]
    lib.oracle_dist_prefix.restype = ctypes.c_uint64
    return lib


def pins_fail(lib):
    """Run the pins against ``lib``; return True if any of them fails."""
    def srt(strings):
        chars, offs = gen.from_strings(strings)
        n = len(strings)
        perm = np.empty(n, np.uint32)
        lcp = np.empty(n, np.uint32)
        if n:
            lib.oracle_sort(chars.ctypes.data, offs.ctypes.data, n, perm.ctypes.data,
                            lcp.ctypes.data)
            d = lib.oracle_dist_prefix(chars.ctypes.data, offs.ctypes.data, perm.ctypes.data,
                                       lcp.ctypes.data, n)
        else:
            d = 0
        return perm.tolist(), lcp.tolist(), d

    cases = []
    for seed in range(30):
        rng = random.Random(seed)
        cases.append(rand_strings(rng, rng.randint(2, 6), TINY_ALPHABET, 4))
    rng = random.Random(5)
    cases.append(rand_strings(rng, 2000, [0x01, 0x7F, 0x80, 0xFF], 10))
    cases.append(rand_strings(rng, 2000, [ord("a"), ord("b")], 30))
    for seed in range(5):
        r2 = random.Random(1000 + seed)
        cases.append(rand_strings(r2, r2.randint(1, 60), [ord("a"), ord("b"), ord("c")], 8))
    cases.append([b"hello"] * 5 + [b"hell", b"help"])
    for strings in cases:
        perm, lcp, d = srt(strings)
        ref = lib_sorted_perm(strings)
        if perm != ref or lcp != lib_lcp(strings, ref) or d != brute_D(strings):
            return True
    return False


def test_unmutated_passes(tmp_path):
    src = open(SRC).read()
    c = tmp_path / "orig.c"
    so = tmp_path / "orig.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", str(c), "-o", str(so)])
    lib = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    lib.oracle_sort.argtypes = [P, P, ctypes.c_uint32, P, P]
    lib.oracle_dist_prefix.argtypes = [P, P, P, P, ctypes.c_uint64]
    lib.oracle_dist_prefix.restype = ctypes.c_uint64
    assert not pins_fail(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_caught(tmp_path, name):
    assert pins_fail(build_mutant(tmp_path, name)), f"mutant {name} survived the pins"
