"""Parity of the HIP S^5 path with the CPU oracle (bit-exact perm and LCP)."""
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import assert_parity, gpu_sort, strings_parity, to_dev  # noqa: E402
from paper_1305_1157_amd import gen, s5  # noqa: E402

# configurations that force many passes, tiny trees and every unroll variant
CFGS = {
    "default": None,
    "tiny_T_v7": s5.make_config(splitters=7, base_threshold=64, tile=64),
    "v255_tile2048": s5.make_config(tile=2048),
    "v511_tile_big": s5.make_config(splitters=511, tile=65536),
    "v1023_u8": s5.make_config(splitters=1023, unroll=8, base_threshold=2048),
    "v31_u1_T128": s5.make_config(splitters=31, unroll=1, base_threshold=128, tile=128),
    "v63_u2_a4": s5.make_config(splitters=63, unroll=2, oversample=4, base_threshold=256),
    "equal": s5.make_config(classifier=s5.CLASSIFY_EQUAL),
    "equal_v7_u1_T64": s5.make_config(classifier=s5.CLASSIFY_EQUAL, splitters=7, unroll=1,
                                      base_threshold=64, tile=64),
    "equal_v1023_u8": s5.make_config(classifier=s5.CLASSIFY_EQUAL, splitters=1023, unroll=8),
    "jump": s5.make_config(classifier=s5.CLASSIFY_JUMP),
    "jump_v7_u2_T64": s5.make_config(classifier=s5.CLASSIFY_JUMP, splitters=7, unroll=2,
                                     base_threshold=64, tile=64),
    "jump_v1023_u8": s5.make_config(classifier=s5.CLASSIFY_JUMP, splitters=1023, unroll=8),
    # two moves per level by the digits of the bucket ids (appendix A, multipass)
    "two_pass": s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS),
    "two_pass_v7_T64": s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS, splitters=7,
                                      base_threshold=64, tile=64),
    "two_pass_v1023_u8": s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS, splitters=1023,
                                        unroll=8, base_threshold=2048),
    "two_pass_v31_T128_jump": s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS, splitters=31,
                                             base_threshold=128, tile=128,
                                             classifier=s5.CLASSIFY_JUMP),
}


def test_prefix_keys_vs_bytes():
    rng = random.Random(3)
    strings = [bytes(rng.choice([1, 0x41, 0x7F, 0x80, 0xFE, 0xFF]) for _ in range(rng.randint(0, 30)))
               for _ in range(3000)]
    chars, offs = gen.from_strings(strings)
    raw = chars.tobytes()
    for depth in (0, 1, 5):
        sel = [i for i, s in enumerate(strings) if len(s) >= depth]
        o = offs[sel] + depth
        keys = s5.prefix_keys(to_dev(chars), to_dev(o), 0).cpu().numpy()
        for j, i in enumerate(sel):
            b = raw[o[j]:o[j] + 8].split(b"\x00")[0][:8]
            want = int.from_bytes(b.ljust(8, b"\x00"), "big")
            assert int(keys[j]) == want, (depth, i)


@pytest.mark.parametrize("variant", ["unroll", "jump"])
def test_classify_vs_searchsorted(variant):
    """2 lower_bound + [equal]: the Unroll descent, and the same descent
    started from the jump table (splitters spread over 64 bits, and packed
    close together so that they share a long common prefix)."""
    rng = np.random.default_rng(5)
    var = {"unroll": s5.CLASSIFY_UNROLL, "jump": s5.CLASSIFY_JUMP}[variant]
    for v in (1, 3, 7, 255, 1023):
        for spread in (2**63, 2**20):
            base = np.uint64(0x6162636465000000)
            spl = np.sort(base + rng.integers(0, spread, size=v, dtype=np.uint64))
            if v > 3:
                spl[v // 2] = spl[v // 2 - 1]  # a duplicate splitter
            keys = np.concatenate([base + rng.integers(0, spread, size=5000, dtype=np.uint64),
                                   rng.integers(0, 2**64 - 1, size=500, dtype=np.uint64), spl,
                                   spl - np.uint64(1), np.array([0, 2**64 - 1], dtype=np.uint64)])
            got = s5.classify(to_dev(keys), to_dev(spl), var).cpu().numpy().astype(np.int64)
            j = np.searchsorted(spl, keys, side="left")
            eq = (j < v) & (spl[np.minimum(j, v - 1)] == keys)
            want = 2 * j + eq
            assert np.array_equal(got, want), (v, spread)


def test_classify_equal_variant():
    """The Equal descent: with distinct splitters exactly 2 lower_bound + [equal];
    with repeated splitters every key equal to a splitter lands in an equality
    bucket of a splitter equal to it and every other key in the range bucket
    between its neighbours."""
    rng = np.random.default_rng(6)
    for v in (1, 3, 7, 255, 1023):
        for dup in (False, True):
            spl = np.sort(rng.integers(0, 2**63, size=v, dtype=np.uint64))
            if dup and v > 3:
                spl[v // 3: v // 3 + 5] = spl[v // 3]  # a run of repeated splitters
                spl = np.sort(spl)
            keys = np.concatenate([rng.integers(0, 2**63, size=5000, dtype=np.uint64), spl,
                                   spl + np.uint64(1), np.array([0, 2**64 - 1], dtype=np.uint64)])
            got = s5.classify(to_dev(keys), to_dev(spl), s5.CLASSIFY_EQUAL).cpu().numpy()
            got = got.astype(np.int64)
            j = np.searchsorted(spl, keys, side="left")
            eq = (j < v) & (spl[np.minimum(j, v - 1)] == keys)
            if not dup or v <= 3:
                assert np.array_equal(got, 2 * j + eq), v
            else:
                odd = (got & 1) == 1
                assert np.array_equal(odd, eq), v
                assert np.all(spl[np.minimum(got[odd] // 2, v - 1)] == keys[odd])
                assert np.array_equal(got[~eq], 2 * j[~eq])


def test_fig1_tree():
    spl = np.array([0x6161610000000000, 0x6D6D6D0000000000, 0x7878780000000000], dtype=np.uint64)
    keys = np.array([0, 0x6161600000000000, 0x6161610000000000, 0x6161610000000001,
                     0x6A00000000000000, 0x6D6D6D0000000000, 0x6D6D6D6100000000,
                     0x7878780000000000, 0x7878780100000000, 2**64 - 1], dtype=np.uint64)
    for variant in (s5.CLASSIFY_UNROLL, s5.CLASSIFY_EQUAL, s5.CLASSIFY_JUMP):
        got = s5.classify(to_dev(keys), to_dev(spl), variant).cpu().numpy().tolist()
        assert got == [0, 0, 1, 2, 2, 3, 4, 5, 6, 6]


EDGE = {
    "one": [b"abc"],
    "two_equal": [b"x", b"x"],
    "two": [b"b", b"a"],
    "all_empty": [b""] * 5000,
    "all_equal": [b"same string here"] * 7000,
    "key_boundary": [b"k" * L for L in (7, 8, 9, 15, 16, 17, 0, 1)] * 700,
    "prefixes_of_each_other": [b"q" * (i % 97) for i in range(9000)],
    "high_bytes": [bytes([0x80 + (i * 7) % 128, 0xFF, 0x01 + i % 3]) for i in range(6000)],
    "long_shared_prefix": [b"p" * 1000 + bytes([65 + (i * 31) % 26, 65 + i % 26]) for i in range(5000)],
    "giant_eq_bucket_plus_tiny": [b"giant" if i % 4 else bytes([97 + i % 26]) * (1 + i % 13)
                                  for i in range(40000)],
}


def _dup_groups(seed, n_distinct, max_rep, length):
    """Long strings over a 2-letter alphabet, each repeated 1..max_rep times, shuffled:
    groups that stay undecided for many 8-byte rounds."""
    rng = random.Random(seed)
    base = [bytes(rng.choice(b"AC") for _ in range(length)) for _ in range(n_distinct)]
    out = [s for s in base for _ in range(rng.randint(1, max_rep))]
    rng.shuffle(out)
    return out


def _near_duplicates(seed, n_groups, length):
    """Runs of equal strings next to strings that differ from them only at
    the end (last character changed, one character more or less, the byte
    after a shared 8-byte key), so that a run of equal keys holds equal and
    unequal pairs: the whole run must be refined, not finished as duplicates."""
    rng = random.Random(seed)
    out = []
    for _ in range(n_groups):
        x = bytes(rng.choice(b"ACGT") for _ in range(length))
        kind = rng.randrange(4)
        out += [x] * rng.randint(2, 5)
        if kind == 0:
            out.append(x[:-1] + (b"A" if x[-1:] != b"A" else b"C"))
        elif kind == 1:
            out.append(x + b"T")
        elif kind == 2:
            out.append(x[:-1])
        else:
            out.append(x[:8] + bytes([x[8] ^ 1]) + x[9:])
    rng.shuffle(out)
    return out


EDGE.update({
    "near_duplicates": _near_duplicates(5, 1500, 90),
    "dup_groups_long": _dup_groups(1, 400, 20, 120),
    "dup_pairs_dna_like": _dup_groups(2, 3000, 2, 100),
    "bucket_sizes_64_65_512_513": [bytes([65 + g]) + bytes([97 + (i * 7919) % 26]) * 12
                                   for g, size in enumerate((64, 65, 512, 513, 2, 3, 4096))
                                   for i in range(size)],
})


@pytest.mark.parametrize("name", sorted(EDGE))
@pytest.mark.parametrize("cfg", ["default", "tiny_T_v7", "v1023_u8", "equal_v7_u1_T64",
                                 "jump_v7_u2_T64", "two_pass_v7_T64", "two_pass_v1023_u8"])
def test_edge_cases(name, cfg):
    strings_parity(EDGE[name], CFGS[cfg], label=f"{name}/{cfg}")


def test_empty_input():
    perm, lcp = gpu_sort(np.zeros(8, np.uint8), np.zeros(0, np.uint64))
    assert perm.size == 0 and lcp.size == 0


def test_suffixes_overlapping_offsets():
    rng = random.Random(11)
    text = bytes(rng.choice(b"abab" b"c") for _ in range(30000))
    chars = np.frombuffer(text + b"\x00", dtype=np.uint8).copy()
    offs = np.arange(len(text), dtype=np.uint64)
    for cfg in ("default", "tiny_T_v7"):
        assert_parity(chars, offs, CFGS[cfg], label=f"suffixes/{cfg}")


def test_many_copies_of_one_string():
    chars, offs = gen.from_strings([b"copy-me"])
    offs = np.zeros(1 << 20, dtype=np.uint64)
    st = assert_parity(chars, offs, None, label="2^20 copies")
    assert st["passes"] >= 1


@pytest.mark.parametrize("name,n", [("random_1M", 200_000), ("url_10M", 200_000),
                                    ("dna_16M", 100_000), ("words_50M", 300_000)])
@pytest.mark.parametrize("cfg", sorted(CFGS))
def test_workloads(name, n, cfg):
    chars, offs = gen.workload(name, n)
    assert_parity(chars, offs, CFGS[cfg], label=f"{name}[{n}]/{cfg}")


def test_random_1M_full():
    chars, offs = gen.workload("random_1M")
    st = assert_parity(chars, offs, None, label="random_1M full")
    assert st["passes"] >= 1 and st["moved_M"] >= 1_000_000


def test_one_bucket_statistic():
    """Strings that share their first 16 bytes fall into one bucket in the first
    pass (moved only to advance the depth); random strings never do."""
    rng = random.Random(12)
    shared = [b"prefix-common-16" + bytes(rng.choice(b"abcdefgh") for _ in range(12))
              for _ in range(20000)]
    st = strings_parity(shared, None, label="shared 16-byte prefix")
    assert st["moved_one_bucket"] >= len(shared)
    chars, offs = gen.workload("random_1M", 100_000)
    st = assert_parity(chars, offs, None, label="random")
    assert st["moved_one_bucket"] == 0


def test_two_pass_same_passes_and_moves():
    """The two-pass distribution moves each level twice but splits the same way:
    the level count and the strings distributed per level are those of one move."""
    chars, offs = gen.workload("words_50M", 400_000)
    one = assert_parity(chars, offs, None, label="one move")
    two = assert_parity(chars, offs, CFGS["two_pass"], label="two moves")
    assert one["passes"] == two["passes"] and one["moved_M"] == two["moved_M"]


def test_output_independent_of_seed():
    chars, offs = gen.workload("words_50M", 100_000)
    a = gpu_sort(chars, offs, s5.make_config(seed=1, base_threshold=128))
    b = gpu_sort(chars, offs, s5.make_config(seed=99, base_threshold=128))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_six_argument_entry_point():
    chars, offs = gen.workload("random_1M", 50_000)
    dc, do = to_dev(chars), to_dev(offs)
    perm = torch.empty(offs.size, dtype=torch.uint32, device=dc.device)
    lcp = torch.empty(offs.size, dtype=torch.uint32, device=dc.device)
    s5.sort_plain(dc, do, perm, lcp)
    torch.cuda.synchronize()
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(perm.cpu().numpy(), rp) and np.array_equal(lcp.cpu().numpy(), rl)


def test_user_workspace():
    chars, offs = gen.workload("url_10M", 30_000)
    cfg = s5.make_config(base_threshold=256)
    ws = torch.empty(s5.workspace_bytes(offs.size, cfg), dtype=torch.uint8, device="cuda")
    perm, lcp = s5.sort(to_dev(chars), to_dev(offs), cfg=cfg, workspace=ws)
    torch.cuda.synchronize()
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(perm.cpu().numpy(), rp) and np.array_equal(lcp.cpu().numpy(), rl)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(s5.S5Error):
        s5.sort(to_dev(chars), to_dev(offs), cfg=cfg, workspace=small)


@pytest.mark.parametrize("name,n,cfg", [("url_10M", 70_001, "default"),
                                        ("dna_16M", 50_003, "tiny_T_v7"),
                                        ("words_50M", 40_009, "v1023_u8")])
def test_no_writes_outside_outputs_and_workspace(name, n, cfg):
    """Guard bytes around the outputs and after a caller workspace stay as
    they were (ragged sizes: the last sub-tile of a tile is partly empty)."""
    chars, offs = gen.workload(name, n)
    c = CFGS[cfg]
    pad, fill = 1 << 16, 0x5A5A5A5A
    wsb = s5.workspace_bytes(n, c)
    ws = torch.full((wsb + 4 * pad,), 0xA5, dtype=torch.uint8, device="cuda")
    big_p = torch.full((n + 2 * pad,), fill, dtype=torch.int64, device="cuda").to(torch.uint32)
    big_l = big_p.clone()
    perm, lcp = big_p[pad:pad + n], big_l[pad:pad + n]
    s5.sort(to_dev(chars), to_dev(offs), cfg=c, out_perm=perm, out_lcp=lcp, workspace=ws[:wsb])
    torch.cuda.synchronize()
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(perm.cpu().numpy(), rp) and np.array_equal(lcp.cpu().numpy(), rl)
    assert bool((ws[wsb:] == 0xA5).all())
    for big in (big_p, big_l):
        h = big.cpu().numpy()
        assert (h[:pad] == fill).all() and (h[pad + n:] == fill).all()


@pytest.mark.parametrize("cfg", ["default", "tiny_T_v7", "equal", "jump"])
def test_batched_small(cfg):
    chars, offs, sb = gen.batched(60, 1, 5000, kinds=("random", "url", "dna", "words"), seed=7)
    # include empty sets and single-string sets
    sizes = np.diff(sb).astype(np.int64)
    sizes[3] = 0
    sizes[5] = 1
    sb2 = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=sb2[1:])
    offs2 = np.concatenate([offs[int(sb[s]):int(sb[s]) + int(sizes[s])] for s in range(sizes.size)])
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs2), to_dev(sb2), cfg=CFGS[cfg])
    torch.cuda.synchronize()
    rp, rl = oracle.sort_batched(chars, offs2, sb2)
    assert np.array_equal(perm.cpu().numpy(), rp)
    assert np.array_equal(lcp.cpu().numpy(), rl)


# Common start of all strings: the key cache starts at the prefix of the
# smallest and largest sampled first key (at most 8 bytes), after checking
# every string; one string without it (placed where the sample does not look)
# sends the key cache back to depth 0.
def _prefixed(prefix, n, seed, odd=None):
    rng = random.Random(seed)
    strings = [prefix + bytes(rng.choice(b"abcxyz") for _ in range(rng.randint(0, 12)))
               for _ in range(n)]
    strings[n // 2] = prefix  # a string that is the prefix itself
    if odd is not None:
        strings[1] = odd  # index 1 is not among the sampled strings at this n
    return strings


@pytest.mark.parametrize("plen", [3, 7, 8, 11])
def test_common_prefix_skipped(plen):
    prefix = b"http://www.example"[:plen]
    st = strings_parity(_prefixed(prefix, 40_000, plen), label=f"prefix {plen}")
    assert st["root_depth"] == min(plen, 8)


@pytest.mark.parametrize("odd", [b"zz", b"htt", b""], ids=["other", "shorter", "empty"])
def test_common_prefix_missed_by_the_sample(odd):
    st = strings_parity(_prefixed(b"http://w", 40_000, 5, odd), label=f"odd {odd!r}")
    assert st["root_depth"] == 0


@pytest.mark.parametrize("odd", [None, b"ab"], ids=["shared", "missed"])
def test_common_prefix_batched(odd):
    chars, offs = gen.from_strings(_prefixed(b"abcdef", 40_000, 9, odd))
    sb = np.array([0, 15_000, 15_001, 40_000], dtype=np.uint64)
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb))
    torch.cuda.synchronize()
    rp, rl = oracle.sort_batched(chars, offs, sb)
    assert np.array_equal(perm.cpu().numpy(), rp)
    assert np.array_equal(lcp.cpu().numpy(), rl)
    assert s5.stats()["root_depth"] == (6 if odd is None else 0)
