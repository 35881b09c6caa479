"""Pins of the CPU oracle against things other than itself.

* exhaustive brute force over all permutations of tiny inputs (exactly one
  order satisfies "non-descending, equal strings by ascending index");
* Python's ``sorted`` on ``(bytes, index)`` (a library routine), on fixed
  alphabets and on property-based random inputs;
* ``os.path.commonprefix`` for every LCP entry (a library routine);
* pairwise brute force for D (a string's distinguishing prefix is one more
  than its longest common prefix with any other string, capped at |s|);
* conventions printed in Table 1 (``tests/golden/table1_conventions.txt``).
"""
import itertools
import os
import random

import numpy as np
import pytest

import oracle
from paper_1305_1157_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lib_sorted_perm(strings):
    return sorted(range(len(strings)), key=lambda i: (strings[i], i))


def lib_lcp(strings, perm):
    out = [0] * len(perm)
    for i in range(1, len(perm)):
        out[i] = len(os.path.commonprefix([strings[perm[i - 1]], strings[perm[i]]]))
    return out


def rand_strings(rng, n, alphabet, maxlen, minlen=0):
    return [bytes(rng.choice(alphabet) for _ in range(rng.randint(minlen, maxlen)))
            for _ in range(n)]


def run_oracle(strings):
    chars, offs = gen.from_strings(strings)
    perm, lcp = oracle.sort(chars, offs)
    return perm.tolist(), lcp.tolist()


TINY_ALPHABET = [0x01, ord("a"), ord("b"), 0xFF]


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_tiny(seed):
    rng = random.Random(seed)
    n = rng.randint(0, 6)
    strings = rand_strings(rng, n, TINY_ALPHABET, 4)
    valid = []
    for p in itertools.permutations(range(n)):
        ok = all(strings[p[i - 1]] < strings[p[i]] or
                 (strings[p[i - 1]] == strings[p[i]] and p[i - 1] < p[i])
                 for i in range(1, n))
        if ok:
            valid.append(list(p))
    assert len(valid) == 1
    perm, lcp = run_oracle(strings)
    assert perm == valid[0]
    assert lcp == lib_lcp(strings, perm)


@pytest.mark.parametrize("alphabet,maxlen,n", [
    (list(range(1, 256)), 12, 3000),          # full byte range, high bytes sort high
    ([0x01, 0x7F, 0x80, 0xFF], 10, 3000),     # signed/unsigned boundary
    ([ord("a"), ord("b")], 30, 3000),         # long shared prefixes, many duplicates
    ([ord("x")], 40, 500),                    # prefixes of one another
])
def test_vs_library_sort(alphabet, maxlen, n):
    rng = random.Random(n + maxlen)
    strings = rand_strings(rng, n, alphabet, maxlen)
    perm, lcp = run_oracle(strings)
    assert perm == lib_sorted_perm(strings)
    assert lcp == lib_lcp(strings, perm)


@pytest.mark.parametrize("name", ["random_1M", "url_10M", "dna_16M", "words_50M"])
def test_workloads_vs_library_sort(name):
    chars, offs = gen.workload(name, 20000)
    strings = gen.to_strings(chars, offs)
    perm, lcp = oracle.sort(chars, offs)
    ref = lib_sorted_perm(strings)
    assert perm.tolist() == ref
    assert lcp.tolist() == lib_lcp(strings, ref)


def test_edge_cases():
    assert run_oracle([]) == ([], [])
    assert run_oracle([b"abc"]) == ([0], [0])
    assert run_oracle([b"", b"", b""]) == ([0, 1, 2], [0, 0, 0])
    s = [b"ab", b"ab", b"a", b"", b"abc", b"ab"]
    perm, lcp = run_oracle(s)
    assert perm == [3, 2, 0, 1, 5, 4]
    assert lcp == [0, 0, 1, 2, 2, 2]
    # equal strings: lcp(s, s) = |s| without the terminator
    perm, lcp = run_oracle([b"hello"] * 5)
    assert perm == list(range(5)) and lcp == [0, 5, 5, 5, 5]
    # a 1,000-byte shared prefix
    base = b"q" * 1000
    strings = [base + bytes([c]) for c in (5, 3, 9, 3)] + [base]
    perm, lcp = run_oracle(strings)
    assert perm == [4, 1, 3, 0, 2]
    assert lcp == [0, 1000, 1001, 1000, 1000]


def test_overlapping_offsets_suffixes():
    text = b"mississippi_banana_mississippi"
    chars = np.frombuffer(text + b"\x00", dtype=np.uint8).copy()
    offs = np.arange(len(text), dtype=np.uint64)
    perm, lcp = oracle.sort(chars, offs)
    sufs = [text[i:] for i in range(len(text))]
    assert perm.tolist() == lib_sorted_perm(sufs)
    assert lcp.tolist() == lib_lcp(sufs, perm.tolist())


def brute_D(strings):
    d = 0
    for i, s in enumerate(strings):
        m = 0
        for j, t in enumerate(strings):
            if i != j:
                m = max(m, len(os.path.commonprefix([s, t])))
        d += min(len(s) + 1, m + 1)
    return d


@pytest.mark.parametrize("seed", range(10))
def test_dist_prefix_bruteforce(seed):
    rng = random.Random(1000 + seed)
    strings = rand_strings(rng, rng.randint(1, 60), [ord("a"), ord("b"), ord("c")], 8)
    chars, offs = gen.from_strings(strings)
    perm, lcp = oracle.sort(chars, offs)
    assert oracle.dist_prefix(chars, offs, perm, lcp) == brute_D(strings)


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_table1_conventions():
    g = read_golden("table1_conventions.txt")
    # Random: one string of every length in [0,20): N/n equals the printed avg |s|
    lo, hi = int(g["random_len_lo"]), int(g["random_len_hi_excl"])
    strings = [b"r" * L for L in range(lo, hi)]
    chars, offs = gen.from_strings(strings)
    assert chars.size / len(strings) == g["random_avg_s"]
    # Sinha DNA: 9-mers that all occur at least twice -> D/N = 100 %, avg |s| = 10
    rng = random.Random(7)
    L = int(g["dna_len"])
    kmers = [bytes(rng.choice(b"ACGT") for _ in range(L)) for _ in range(300)]
    strings = kmers + kmers[::-1] + kmers[:50]
    rng.shuffle(strings)
    chars, offs = gen.from_strings(strings)
    perm, lcp = oracle.sort(chars, offs)
    D = oracle.dist_prefix(chars, offs, perm, lcp)
    assert chars.size / len(strings) == g["dna_avg_s"]
    assert D / chars.size == g["dna_D_over_N"]
    assert D == brute_D(strings)


def test_batched_equals_per_set():
    chars, offs, sb = gen.batched(12, 1, 300, kinds=("random", "url", "dna", "words"),
                                  seed=99)
    perm, lcp = oracle.sort_batched(chars, offs, sb)
    for s in range(12):
        b, e = int(sb[s]), int(sb[s + 1])
        strings = gen.to_strings(chars, offs[b:e])
        ref = lib_sorted_perm(strings)
        assert perm[b:e].tolist() == ref
        assert lcp[b:e].tolist() == lib_lcp(strings, ref)


# ---- checkers for results too large to recompute --------------------------

def _batched_case():
    from paper_1305_1157_amd import gen
    chars, offs, sb = gen.batched(12, 1, 3000, kinds=("random", "url", "dna", "words"), seed=77)
    perm, lcp = oracle.sort_batched(chars, offs, sb)
    return chars, offs, sb, perm, lcp


def test_checkers_accept_correct_results():
    chars, offs, sb, perm, lcp = _batched_case()
    assert oracle.check_perm(perm, sb)
    allpos = np.arange(perm.size, dtype=np.uint64)
    assert oracle.check_pairs(chars, offs, perm, lcp, allpos, sb) == 0
    # single set
    p1, l1 = oracle.sort(chars, offs)
    assert oracle.check_perm(p1)
    assert oracle.check_pairs(chars, offs, p1, l1, np.arange(p1.size, dtype=np.uint64)) == 0


def test_checkers_catch_planted_mistakes():
    chars, offs, sb, perm, lcp = _batched_case()
    allpos = np.arange(perm.size, dtype=np.uint64)
    s0 = int(sb[2])  # a position inside a set with >= 3 strings
    while int(sb[np.searchsorted(sb, s0, side="right")]) - s0 < 3:
        s0 += 1
    # a duplicated index is no permutation
    bad = perm.copy()
    bad[s0 + 1] = bad[s0]
    assert not oracle.check_perm(bad, sb)
    # an index beyond its set
    bad = perm.copy()
    bad[s0] = 10**6
    assert not oracle.check_perm(bad, sb)
    # two distinct neighbours swapped: order broken at p or p+1
    bad = perm.copy()
    for p in range(s0 + 1, perm.size):
        a, b = int(offs[s0 + perm[p - 1]]), int(offs[s0 + perm[p]])
        if lcp[p] < 1000 and chars[a + lcp[p]] != chars[b + lcp[p]]:
            break
    bad[p - 1], bad[p] = bad[p], bad[p - 1]
    assert oracle.check_pairs(chars, offs, bad, lcp, allpos, sb) > 0
    # one wrong LCP value
    badl = lcp.copy()
    badl[s0 + 1] += 1
    assert oracle.check_pairs(chars, offs, perm, badl, allpos, sb) == 1
    # non-zero LCP at a set's first slot
    badl = lcp.copy()
    badl[int(sb[3])] = 1
    assert oracle.check_pairs(chars, offs, perm, badl, allpos, sb) >= 1


def test_check_all_pairs_equals_every_position():
    """The threaded whole-array check counts exactly what the per-position check
    counts over every position, on correct and on planted-bad results."""
    chars, offs, sb, perm, lcp = _batched_case()
    allpos = np.arange(perm.size, dtype=np.uint64)
    for threads in (1, 3, 8):
        assert oracle.check_all_pairs(chars, offs, perm, lcp, sb, threads=threads) == 0
    rng = np.random.default_rng(2)
    badl = lcp.copy()
    hits = rng.choice(perm.size, size=17, replace=False)
    badl[hits] += 1
    want = oracle.check_pairs(chars, offs, perm, badl, allpos, sb)
    assert want == 17
    for threads in (1, 4):
        assert oracle.check_all_pairs(chars, offs, perm, badl, sb, threads=threads) == want
    p1, l1 = oracle.sort(chars, offs)
    assert oracle.check_all_pairs(chars, offs, p1, l1) == 0
    bad = p1.copy()
    bad[[5, 6]] = bad[[6, 5]]
    assert oracle.check_all_pairs(chars, offs, bad, l1) == \
        oracle.check_pairs(chars, offs, bad, l1, np.arange(p1.size, dtype=np.uint64)) > 0


def test_keys_at_by_bytes():
    """8-byte big-endian keys written out byte by byte from the definition."""
    rng = random.Random(4)
    strings = [bytes(rng.choice([1, 0x41, 0x7F, 0x80, 0xFE, 0xFF]) for _ in range(rng.randint(0, 20)))
               for _ in range(500)]
    chars, offs = gen.from_strings(strings)
    for depth in (0, 3):
        sel = [i for i, x in enumerate(strings) if len(x) >= depth]
        keys = oracle.keys_at(chars, offs[sel], depth)
        for j, i in enumerate(sel):
            b = strings[i][depth:depth + 8]
            assert int(keys[j]) == int.from_bytes(b.ljust(8, b"\x00"), "big")


def test_check_pairs_tie_break_by_index():
    # equal strings must appear in ascending input order
    chars, offs = gen.from_strings([b"same", b"same", b"other", b"same"])
    perm, lcp = oracle.sort(chars, offs)
    assert list(perm) == [2, 0, 1, 3]
    bad = perm.copy()
    bad[1], bad[2] = bad[2], bad[1]  # same strings, indices descending
    assert oracle.check_pairs(chars, offs, bad, lcp, np.arange(4, dtype=np.uint64)) == 1


# property-based: arbitrary byte strings (no zero byte), including empty
# strings, duplicates and strings that are prefixes of others
try:
    from hypothesis import given, settings, strategies as st
except ImportError:  # pragma: no cover
    given = None

if given is not None:
    _strings = st.lists(
        st.one_of(st.binary(max_size=24), st.sampled_from([b"", b"a", b"ab", b"abc", b"\xff"]))
        .map(lambda b: b.replace(b"\x00", b"\x01")),
        max_size=60)

    @settings(max_examples=300, deadline=None)
    @given(_strings)
    def test_property_vs_library_sort(strings):
        perm, lcp = run_oracle(strings)
        assert perm == lib_sorted_perm(strings)
        assert lcp == lib_lcp(strings, perm)
