"""CPU oracle for string sorting (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never calls it, links
it or loads it, and the two share no code.

``sort`` returns the unique permutation that orders the strings by unsigned
lexicographic byte order up to their terminator, equal strings by ascending
input index, plus the LCP array of that order (Bingmann & Sanders, Section 2,
definitions of the input, of lcp and of D).  The C source implements multikey
quicksort (Section 2.1) and an explicit LCP pass; see ``s5_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "s5_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_s5_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/_s5_oracle.so``."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_sort.argtypes = [P, P, ctypes.c_uint32, P, P]
        lib.oracle_sort.restype = ctypes.c_int
        lib.oracle_sort_batched.argtypes = [P, P, P, ctypes.c_uint32, P, P]
        lib.oracle_sort_batched.restype = ctypes.c_int
        lib.oracle_dist_prefix.argtypes = [P, P, P, P, ctypes.c_uint64]
        lib.oracle_dist_prefix.restype = ctypes.c_uint64
        lib.oracle_lcp.argtypes = [P, P, P, ctypes.c_uint64, P]
        lib.oracle_lcp.restype = None
        lib.oracle_check_perm.argtypes = [P, P, ctypes.c_uint32, ctypes.c_uint64]
        lib.oracle_check_perm.restype = ctypes.c_int
        lib.oracle_check_pairs.argtypes = [P, P, P, ctypes.c_uint32, ctypes.c_uint64, P, P, P,
                                           ctypes.c_uint64]
        lib.oracle_check_pairs.restype = ctypes.c_uint64
        lib.oracle_check_all_pairs.argtypes = [P, P, P, ctypes.c_uint32, ctypes.c_uint64, P, P,
                                               ctypes.c_int]
        lib.oracle_check_all_pairs.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check(chars, offsets):
    chars = np.ascontiguousarray(chars, dtype=np.uint8)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    if offsets.size >= 2**32:
        raise ValueError("at most 2^32 - 1 strings")
    return chars, offsets


def sort(chars: np.ndarray, offsets: np.ndarray):
    """Return ``(perm, lcp)`` as uint32 arrays for the strings at ``offsets``."""
    chars, offsets = _check(chars, offsets)
    n = offsets.size
    perm = np.empty(n, dtype=np.uint32)
    lcp = np.empty(n, dtype=np.uint32)
    if n and _load().oracle_sort(_ptr(chars), _ptr(offsets), n, _ptr(perm), _ptr(lcp)):
        raise MemoryError("oracle_sort ran out of memory")
    return perm, lcp


def sort_batched(chars: np.ndarray, offsets: np.ndarray, set_begin: np.ndarray):
    """Sort every set ``[set_begin[s], set_begin[s+1])`` on its own.

    ``perm`` holds set-local indices and ``lcp`` is 0 at every set's first slot.
    """
    chars, offsets = _check(chars, offsets)
    set_begin = np.ascontiguousarray(set_begin, dtype=np.uint64)
    n = offsets.size
    perm = np.empty(n, dtype=np.uint32)
    lcp = np.empty(n, dtype=np.uint32)
    ns = set_begin.size - 1
    if ns > 0 and _load().oracle_sort_batched(
            _ptr(chars), _ptr(offsets), _ptr(set_begin), ns, _ptr(perm), _ptr(lcp)):
        raise ValueError("oracle_sort_batched failed (bad set_begin or no memory)")
    return perm, lcp


def lcp_of(chars: np.ndarray, offsets: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Explicit LCP pass over any given order ``perm``."""
    chars, offsets = _check(chars, offsets)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.empty(perm.size, dtype=np.uint32)
    if perm.size:
        _load().oracle_lcp(_ptr(chars), _ptr(offsets), _ptr(perm), perm.size, _ptr(lcp))
    return lcp


def dist_prefix(chars: np.ndarray, offsets: np.ndarray, perm: np.ndarray,
                lcp: np.ndarray) -> int:
    """Distinguishing prefix size D of the set, terminators counted."""
    chars, offsets = _check(chars, offsets)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.ascontiguousarray(lcp, dtype=np.uint32)
    if perm.size == 0:
        return 0
    return int(_load().oracle_dist_prefix(_ptr(chars), _ptr(offsets), _ptr(perm),
                                          _ptr(lcp), perm.size))


def keys_at(chars: np.ndarray, offsets: np.ndarray, depth: int = 0) -> np.ndarray:
    """The 8 bytes of every string from byte ``depth`` on, packed big-endian
    (first byte most significant) and zero from the terminator on, so that
    unsigned key order is the lexicographic order of those bytes (Section 3.1:
    a machine word of characters).  Requires depth <= every string's length."""
    chars, offsets = _check(chars, offsets)
    padded = np.concatenate([chars, np.zeros(8, dtype=np.uint8)])
    idx = offsets.astype(np.int64)[:, None] + depth + np.arange(8)[None, :]
    b = padded[idx].astype(np.uint64)
    ended = np.maximum.accumulate(b == 0, axis=1)
    b[ended] = 0
    shifts = np.arange(56, -8, -8, dtype=np.uint64)
    return np.bitwise_or.reduce(b << shifts[None, :], axis=1).astype(np.uint64)


def check_perm(perm: np.ndarray, set_begin: np.ndarray | None = None) -> bool:
    """True if ``perm`` restricted to every set is a permutation of the set's
    local indices (whole-array check, any size)."""
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    sb = None if set_begin is None else np.ascontiguousarray(set_begin, dtype=np.uint64)
    ns = 1 if sb is None else sb.size - 1
    r = _load().oracle_check_perm(_ptr(perm), None if sb is None else _ptr(sb), ns, perm.size)
    if r < 0:
        raise MemoryError("oracle_check_perm ran out of memory")
    return bool(r)


def check_pairs(chars: np.ndarray, offsets: np.ndarray, perm: np.ndarray, lcp: np.ndarray,
                positions: np.ndarray, set_begin: np.ndarray | None = None) -> int:
    """Number of the given positions p whose neighbours (perm[p-1], perm[p]) are
    out of order (bytes, then index) or whose lcp[p] is wrong; lcp must be 0 at
    a set's first slot.  Checks a result one pair at a time, at any size."""
    chars, offsets = _check(chars, offsets)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.ascontiguousarray(lcp, dtype=np.uint32)
    pos = np.ascontiguousarray(positions, dtype=np.uint64)
    sb = None if set_begin is None else np.ascontiguousarray(set_begin, dtype=np.uint64)
    ns = 1 if sb is None else sb.size - 1
    return int(_load().oracle_check_pairs(_ptr(chars), _ptr(offsets),
                                          None if sb is None else _ptr(sb), ns, perm.size,
                                          _ptr(perm), _ptr(lcp), _ptr(pos), pos.size))


def check_all_pairs(chars: np.ndarray, offsets: np.ndarray, perm: np.ndarray, lcp: np.ndarray,
                    set_begin: np.ndarray | None = None, threads: int | None = None) -> int:
    """``check_pairs`` at every position: the number of positions whose pair is out
    of order or whose lcp is wrong.  Together with ``check_perm`` this checks a
    result completely (the order with ties by index is unique).  Disjoint ranges
    of positions are checked on ``threads`` host threads (default: all cores,
    at most 16)."""
    chars, offsets = _check(chars, offsets)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    lcp = np.ascontiguousarray(lcp, dtype=np.uint32)
    sb = None if set_begin is None else np.ascontiguousarray(set_begin, dtype=np.uint64)
    ns = 1 if sb is None else sb.size - 1
    if threads is None:
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
    return int(_load().oracle_check_all_pairs(_ptr(chars), _ptr(offsets),
                                              None if sb is None else _ptr(sb), ns, perm.size,
                                              _ptr(perm), _ptr(lcp), threads))
