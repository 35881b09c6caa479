"""Alphabet compression (appendix A, "Alphabet compression") on the GPU: with
S5_ALPHABET_AUTO and at most 7 byte values the sort runs on 3-bit codes, 21
characters per key, and the output stays bit-exact against the oracle; a byte
outside the sampled alphabet makes the call sort again with byte keys."""
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import assert_parity, strings_parity, to_dev  # noqa: E402
from paper_1305_1157_amd import gen, s5  # noqa: E402

AUTO = s5.make_config(alphabet=s5.ALPHABET_AUTO)
CFGS = {
    "auto": AUTO,
    "auto_tiny": s5.make_config(alphabet=s5.ALPHABET_AUTO, splitters=7, base_threshold=64, tile=64),
    "auto_v1023_u8": s5.make_config(alphabet=s5.ALPHABET_AUTO, splitters=1023, unroll=8,
                                    base_threshold=2048),
    "auto_jump_learned": s5.make_config(alphabet=s5.ALPHABET_AUTO, classifier=s5.CLASSIFY_JUMP,
                                        splitter_mode=s5.SPLIT_LEARNED, imbalance_bound=1e9),
    "auto_two_pass": s5.make_config(alphabet=s5.ALPHABET_AUTO,
                                    distribution=s5.DISTRIBUTE_TWO_PASS),
}


@pytest.mark.parametrize("cfg", sorted(CFGS))
@pytest.mark.parametrize("n", [3_000, 120_000])
def test_dna_packed(cfg, n):
    chars, offs = gen.workload("dna_16M", n)
    st = assert_parity(chars, offs, CFGS[cfg], label=f"dna[{n}]/{cfg}")
    assert st["char_bits"] == 3 and st["alphabet_retries"] == 0


def _strings(seed, alphabet, n, maxlen, dup=0.2):
    rng = random.Random(seed)
    out = [bytes(rng.choice(alphabet) for _ in range(rng.randint(0, maxlen))) for _ in range(n)]
    out += [rng.choice(out) for _ in range(int(dup * n))]
    # prefixes of one another around the key boundaries (21, 42, 63 characters)
    base = bytes(rng.choice(alphabet) for _ in range(130))
    out += [base[:L] for L in (0, 1, 20, 21, 22, 41, 42, 43, 62, 63, 64, 84, 126, 130)] * 30
    rng.shuffle(out)
    return out


@pytest.mark.parametrize("alphabet", [b"ACGT", b"AC", b"A", b"ACGTNRY", b"\x01\x7f\x80\xfe\xff",
                                      b"ab"])
@pytest.mark.parametrize("cfg", ["auto", "auto_tiny"])
def test_small_alphabets(alphabet, cfg):
    st = strings_parity(_strings(len(alphabet), alphabet, 20_000, 100), CFGS[cfg],
                        label=f"{alphabet!r}/{cfg}")
    assert st["char_bits"] == 3


@pytest.mark.parametrize("cfg", ["auto", "auto_tiny"])
def test_duplicate_runs_packed(cfg):
    """Runs of equal DNA strings beside strings that differ from them only at
    the end (the base case finishes a run at once only if all its strings are
    equal)."""
    rng = random.Random(8)
    strs = []
    for _ in range(1200):
        x = bytes(rng.choice(b"ACGT") for _ in range(rng.randint(30, 110)))
        strs += [x] * rng.randint(2, 4)
        strs.append([x[:-1] + b"G", x + b"A", x[:-2]][rng.randrange(3)])
    rng.shuffle(strs)
    st = strings_parity(strs, CFGS[cfg], label=f"duplicate runs/{cfg}")
    assert st["char_bits"] == 3


def test_eight_values_use_bytes():
    st = strings_parity(_strings(9, b"ACGTNRYK", 20_000, 60), AUTO, label="8 values")
    assert st["char_bits"] == 8


def test_byte_outside_sample_falls_back():
    """A string outside the sampled strings holds a byte the sample never saw:
    the packed sort reports it and the call sorts again with byte keys."""
    n = 100_000
    chars, offs = gen.workload("dna_16M", n)
    sampled = {(j * n) // 65536 for j in range(65536)}
    victim = next(i for i in range(n // 2, n) if i not in sampled)
    chars = chars.copy()
    chars[int(offs[victim]) + 3] = ord("N")
    st = assert_parity(chars, offs, AUTO, label="fallback")
    assert st["alphabet_retries"] == 1 and st["char_bits"] == 8


def test_byte_beyond_sampled_length():
    """Bytes past the first 256 of a string are not sampled: a string that is
    decided before them never loads them (packed sort, exact output); one whose
    twin shares them is loaded and makes the sort fall back."""
    rng = random.Random(4)
    strs = [bytes(rng.choice(b"ACGT") for _ in range(300)) for _ in range(2000)]
    late = bytes(rng.choice(b"ACGT") for _ in range(280)) + b"Z" + b"ACGT" * 4  # unique early
    st = strings_parity(strs + [late], AUTO, label="late byte, decided early")
    assert st["char_bits"] == 3
    twin = strs[5][:280] + b"Z" + strs[5][281:]
    st = strings_parity(strs + [twin, twin[:290] + b"Q"], AUTO, label="late byte, compared")
    assert st["char_bits"] == 8 and st["alphabet_retries"] == 1


def test_batched_packed():
    chars, offs, sb = gen.batched(8, 1, 80_000, kinds=("dna",), seed=23)
    cfg = s5.make_config(alphabet=s5.ALPHABET_AUTO)
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), cfg=cfg)
    torch.cuda.synchronize()
    import oracle
    rp, rl = oracle.sort_batched(chars, offs, sb)
    assert np.array_equal(perm.cpu().numpy(), rp) and np.array_equal(lcp.cpu().numpy(), rl)
    assert s5.stats()["char_bits"] == 3
