"""Seeded synthetic string sets (inputs only; none of the sort's arithmetic).

The five workloads follow the shapes of the paper's dataset classes (Section 4:
random strings, URLs, DNA reads, word lists) without reproducing any real
dataset.  Every workload is a host arena of null-terminated strings plus uint64
offsets; see ``gen.c`` for the exact recipes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "_s5gen.so")
_lib = None

KIND = {"random": 1, "url": 2, "dna": 3, "words": 4}

# name -> (kind, n, seed); the batched workload is listed separately
WORKLOADS = {
    "random_1M": ("random", 1_000_000, 0x5EED0001),
    "url_10M": ("url", 10_000_000, 0x5EED0002),
    "dna_16M": ("dna", 16_000_000, 0x5EED0003),
    "words_50M": ("words", 50_000_000, 0x5EED0004),
}
BATCHED = {"sets_4096": dict(num_sets=4096, min_size=100, max_size=1_000_000,
                             kinds=("random", "url", "dna"), seed=0x5EED0005)}


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.s5gen_max_len.argtypes = [ctypes.c_int]
        lib.s5gen_max_len.restype = ctypes.c_uint64
        lib.s5gen_generate.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, P,
                                       ctypes.c_uint64, P]
        lib.s5gen_generate.restype = ctypes.c_int64
        lib.s5gen_batched_plan.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                           ctypes.c_uint64, P, ctypes.c_int, P, P]
        lib.s5gen_batched_plan.restype = None
        lib.s5gen_batched.argtypes = [ctypes.c_uint32, ctypes.c_uint64, P, P, P,
                                      ctypes.c_uint64, P]
        lib.s5gen_batched.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def generate(kind: str, n: int, seed: int):
    """Return ``(chars uint8, offsets uint64)`` for ``n`` strings of ``kind``."""
    lib = _load()
    k = KIND[kind]
    cap = max(1, n * int(lib.s5gen_max_len(k)))
    chars = np.empty(cap, dtype=np.uint8)
    offsets = np.empty(n, dtype=np.uint64)
    used = lib.s5gen_generate(k, n, seed & (2**64 - 1), _p(chars), cap, _p(offsets))
    if used < 0:
        raise RuntimeError(f"generator {kind} failed ({used})")
    return chars[:used].copy() if used < cap // 2 else chars[:used], offsets


def workload(name: str, n: int | None = None):
    """A named workload, optionally cut to its first ``n`` strings' recipe
    (a smaller ``n`` regenerates with the same seed and recipe)."""
    kind, n0, seed = WORKLOADS[name]
    return generate(kind, n0 if n is None else n, seed)


def batched(num_sets: int, min_size: int, max_size: int, kinds=("random", "url", "dna"),
            seed: int = 0x5EED0005):
    """Return ``(chars, offsets, set_begin)``: ``num_sets`` independent sets of
    log-uniform size, each from one generator chosen uniformly from ``kinds``."""
    lib = _load()
    ks = np.array([KIND[k] for k in kinds], dtype=np.int32)
    sizes = np.empty(num_sets, dtype=np.uint64)
    skind = np.empty(num_sets, dtype=np.int32)
    lib.s5gen_batched_plan(num_sets, seed, min_size, max_size, _p(ks), len(ks), _p(sizes),
                           _p(skind))
    set_begin = np.zeros(num_sets + 1, dtype=np.uint64)
    np.cumsum(sizes, out=set_begin[1:])
    n = int(set_begin[-1])
    maxlen = np.array([lib.s5gen_max_len(int(k)) for k in skind], dtype=np.uint64)
    cap = max(1, int((sizes * maxlen).sum()))
    chars = np.empty(cap, dtype=np.uint8)
    offsets = np.empty(n, dtype=np.uint64)
    used = lib.s5gen_batched(num_sets, seed, _p(sizes), _p(skind), _p(chars), cap,
                             _p(offsets))
    if used < 0:
        raise RuntimeError(f"batched generator failed ({used})")
    return chars[:used], offsets, set_begin


def from_strings(strings):
    """Arena + offsets for a list of ``bytes`` (each must contain no zero byte)."""
    offs = np.empty(len(strings), dtype=np.uint64)
    parts = []
    p = 0
    for i, s in enumerate(strings):
        if b"\x00" in s:
            raise ValueError("strings may not contain the terminator byte")
        offs[i] = p
        parts.append(s + b"\x00")
        p += len(s) + 1
    chars = np.frombuffer(b"".join(parts), dtype=np.uint8).copy() if parts else \
        np.zeros(0, dtype=np.uint8)
    return chars, offs


def to_strings(chars: np.ndarray, offsets: np.ndarray):
    """List of ``bytes`` (without terminator) for the strings at ``offsets``."""
    raw = chars.tobytes()
    out = []
    for o in offsets.tolist():
        e = raw.index(b"\x00", o)
        out.append(raw[o:e])
    return out
