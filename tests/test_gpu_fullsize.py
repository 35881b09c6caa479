"""The workloads at their full sizes, in the configurations the benchmark times,
checked completely through the oracle's checkers: the permutation of every set
(check_perm) and, at EVERY position, the order of the neighbour pair (bytes,
then input index) and its LCP recomputed from the bytes (check_all_pairs).
The order with ties by index is unique, so the two checks together pin the
whole result.  Smaller cases of the same recipes are compared element by
element with the oracle's own sort elsewhere."""
import time

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from paper_1305_1157_amd import autotune, gen, s5  # noqa: E402

LEARNED = s5.make_config(splitter_mode=s5.SPLIT_LEARNED)


def _check(chars, offs, perm, lcp, sb=None, label=""):
    hp, hl = perm.cpu().numpy(), lcp.cpu().numpy()
    t0 = time.time()
    print(f"{label}: checking all {hp.size:,} positions", flush=True)
    assert oracle.check_perm(hp, sb), f"{label}: not a permutation"
    bad = oracle.check_all_pairs(chars, offs, hp, hl, sb)
    assert bad == 0, f"{label}: {bad} of {hp.size} neighbour pairs wrong"
    print(f"{label}: complete check {time.time() - t0:.1f} s", flush=True)


@pytest.mark.parametrize("name", ["random_1M", "url_10M", "words_50M", "dna_16M"])
def test_full_plain(name):
    chars, offs = gen.workload(name)
    perm, lcp = s5.sort(to_dev(chars), to_dev(offs))
    torch.cuda.synchronize()
    _check(chars, offs, perm, lcp, label=name)


@pytest.mark.parametrize("name", ["dna_16M", "words_50M"])
def test_full_learned(name):
    """Learned splitters at full size (the benchmark's learned lines): checked
    completely, and equal to the sampled-splitter result."""
    chars, offs = gen.workload(name)
    dc, do = to_dev(chars), to_dev(offs)
    p2, l2 = s5.sort(dc, do, cfg=LEARNED)
    torch.cuda.synchronize()
    _check(chars, offs, p2, l2, label=f"{name} learned")
    p1, l1 = s5.sort(dc, do)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(l1, l2)


@pytest.mark.parametrize("learned", [False, True], ids=["sampled", "learned"])
def test_full_batched_graph(learned):
    spec = gen.BATCHED["sets_4096"]
    chars, offs, sb = gen.batched(**spec)
    sizes = np.diff(sb).astype(np.int64)
    table = autotune.load_table()
    cfg = autotune.launch_config(
        table, splitter_mode=s5.SPLIT_LEARNED if learned else s5.SPLIT_SAMPLED)
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), cfg=cfg,
                                tuning=s5.make_tuning(autotune.tuning_for(sizes, table)))
    torch.cuda.synchronize()
    _check(chars, offs, perm, lcp, sb=sb, label=f"sets_4096 {'learned' if learned else ''}")
    # whole small sets against the oracle's own sort, element by element
    hp, hl = perm.cpu().numpy(), lcp.cpu().numpy()
    rng = np.random.default_rng(7)
    for s_ in rng.choice(np.flatnonzero((sizes > 1) & (sizes <= 100_000)), size=6, replace=False):
        b, e = int(sb[s_]), int(sb[s_ + 1])
        rp, rl = oracle.sort(chars, offs[b:e])
        assert np.array_equal(hp[b:e], rp) and np.array_equal(hl[b:e], rl), f"set {s_}"
