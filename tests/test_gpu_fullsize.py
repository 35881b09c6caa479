"""The workloads at their full sizes, in the configurations the benchmark times,
checked through the oracle's checkers: the permutation of every set, and the
order and LCP of sampled neighbour pairs (too large for the oracle to re-sort).
Smaller cases of the same recipes are checked element by element elsewhere."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from paper_1305_1157_amd import autotune, gen, s5  # noqa: E402

PAIRS = 2_000_000


def _check(chars, offs, perm, lcp, sb=None, label=""):
    hp, hl = perm.cpu().numpy(), lcp.cpu().numpy()
    print(f"{label}: checking {hp.size:,} strings", flush=True)
    assert oracle.check_perm(hp, sb), f"{label}: not a permutation"
    rng = np.random.default_rng(hash(label) & 0xFFFF)
    pos = rng.integers(0, hp.size, size=min(PAIRS, hp.size)).astype(np.uint64)
    bad = oracle.check_pairs(chars, offs, hp, hl, pos, sb)
    assert bad == 0, f"{label}: {bad} of {pos.size} sampled neighbour pairs wrong"
    # the first and last positions of the output too
    ends = np.concatenate([np.arange(min(1000, hp.size)), np.arange(max(0, hp.size - 1000), hp.size)])
    assert oracle.check_pairs(chars, offs, hp, hl, ends.astype(np.uint64), sb) == 0


@pytest.mark.parametrize("name", ["url_10M", "words_50M"])
def test_full_plain(name):
    chars, offs = gen.workload(name)
    perm, lcp = s5.sort(to_dev(chars), to_dev(offs))
    torch.cuda.synchronize()
    _check(chars, offs, perm, lcp, label=name)


def test_full_dna_learned_equals_sampled():
    chars, offs = gen.workload("dna_16M")
    dc, do = to_dev(chars), to_dev(offs)
    p1, l1 = s5.sort(dc, do)
    p2, l2 = s5.sort(dc, do, cfg=s5.make_config(splitter_mode=s5.SPLIT_LEARNED))
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(l1, l2)
    _check(chars, offs, p1, l1, label="dna_16M")


def test_full_batched_graph():
    spec = gen.BATCHED["sets_4096"]
    chars, offs, sb = gen.batched(**spec)
    sizes = np.diff(sb).astype(np.int64)
    table = autotune.load_table()
    cfg = s5.make_config(unroll=table["unroll"])
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), cfg=cfg,
                                tuning=s5.make_tuning(autotune.tuning_for(sizes, table)))
    torch.cuda.synchronize()
    _check(chars, offs, perm, lcp, sb=sb, label="sets_4096")
    # whole small sets against the oracle, element by element
    hp, hl = perm.cpu().numpy(), lcp.cpu().numpy()
    rng = np.random.default_rng(7)
    for s_ in rng.choice(np.flatnonzero((sizes > 1) & (sizes <= 100_000)), size=6, replace=False):
        b, e = int(sb[s_]), int(sb[s_ + 1])
        rp, rl = oracle.sort(chars, offs[b:e])
        assert np.array_equal(hp[b:e], rp) and np.array_equal(hl[b:e], rl), f"set {s_}"
