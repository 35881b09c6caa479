"""Batched sorting in one hipGraph: parity with the oracle set by set, the
host continuation past the captured levels, graph replays, learned splitters
inside the graph, per-set tuning, and agreement with the single-set path."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from paper_1305_1157_amd import gen, s5  # noqa: E402


def check(chars, offs, sb, perm, lcp, label):
    torch.cuda.synchronize()
    rp, rl = oracle.sort_batched(chars, offs, sb)
    gp, gl = perm.cpu().numpy(), lcp.cpu().numpy()
    if not np.array_equal(gp, rp):
        bad = np.nonzero(gp != rp)[0]
        raise AssertionError(f"{label}: perm differs at {bad.size} positions, first {bad[:8]}")
    if not np.array_equal(gl, rl):
        bad = np.nonzero(gl != rl)[0]
        raise AssertionError(f"{label}: lcp differs at {bad.size} positions, first {bad[:8]}")


def with_edges(chars, offs, sb):
    """Make sets 0 and 3 empty and set 5 a single string."""
    sizes = np.diff(sb).astype(np.int64)
    sizes[0] = 0
    sizes[3] = 0
    sizes[5] = 1
    sb2 = np.zeros(sizes.size + 1, dtype=np.uint64)
    np.cumsum(sizes, out=sb2[1:])
    offs2 = np.concatenate([offs[int(sb[s]):int(sb[s]) + int(sizes[s])] for s in range(sizes.size)])
    return chars, offs2, sb2


@pytest.mark.parametrize("kinds,nsets,lo,hi", [
    (("random", "url", "dna", "words"), 200, 1, 20_000),
    (("url",), 40, 2_000, 60_000),
    (("dna",), 24, 10_000, 100_000),
])
def test_graph_parity(kinds, nsets, lo, hi):
    chars, offs, sb = with_edges(*gen.batched(nsets, lo, hi, kinds=kinds, seed=31))
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb))
    check(chars, offs, sb, perm, lcp, f"graph {kinds}")
    st = s5.stats()
    assert st["passes"] >= 1 and st["moved_M"] > 0


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_host_continues_past_captured_levels(levels):
    # URL-like sets need several passes: the graph holds only `levels` of them
    chars, offs, sb = gen.batched(30, 5_000, 80_000, kinds=("url",), seed=32)
    cfg = s5.make_config(graph_levels=levels, base_threshold=256)
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), cfg=cfg)
    check(chars, offs, sb, perm, lcp, f"levels={levels}")
    assert s5.stats()["passes"] > levels


def test_graph_replays():
    chars, offs, sb = gen.batched(50, 10, 30_000, kinds=("random", "url", "words"), seed=33)
    dc, do, ds = to_dev(chars), to_dev(offs), to_dev(sb)
    n = offs.size
    perm = torch.empty(n, dtype=torch.uint32, device="cuda")
    lcp = torch.empty(n, dtype=torch.uint32, device="cuda")
    rp, rl = oracle.sort_batched(chars, offs, sb)
    for rep in range(4):
        perm.fill_(0xFFFF)
        lcp.fill_(0xFFFF)
        torch.cuda.synchronize()
        s5.sort_batched(dc, do, ds, out_perm=perm, out_lcp=lcp)  # same key: replay
        torch.cuda.synchronize()
        assert np.array_equal(perm.cpu().numpy(), rp), f"replay {rep}"
        assert np.array_equal(lcp.cpu().numpy(), rl), f"replay {rep}"
        _ = (torch.arange(1000, device="cuda") * 3).sum().item()  # eager work in between


def test_graph_matches_single_set_path():
    chars, offs = gen.workload("words_50M", 300_000)
    sb = np.array([0, offs.size], dtype=np.uint64)
    dc, do = to_dev(chars), to_dev(offs)
    p1, l1 = s5.sort(dc, do)
    st1 = s5.stats()
    p2, l2 = s5.sort_batched(dc, do, to_dev(sb))
    st2 = s5.stats()
    torch.cuda.synchronize()
    assert torch.equal(p1, p2) and torch.equal(l1, l2)
    for k in ("passes", "moved_M", "segments", "max_bucket", "base_items"):
        assert st1[k] == st2[k], k
    assert abs(st1["entropy_bits"] - st2["entropy_bits"]) < 1e-9


@pytest.mark.parametrize("beta", [0.0, 1e-6, 1e9])
def test_graph_learned(beta):
    chars, offs, sb = gen.batched(6, 70_000, 160_000, kinds=("random", "dna", "url"), seed=34)
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED, imbalance_bound=beta)
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), cfg=cfg)
    check(chars, offs, sb, perm, lcp, f"learned beta={beta}")
    st = s5.stats()
    if beta == 1e-6:
        assert st["fallbacks"] >= 1
    if beta == 1e9:
        assert st["fallbacks"] == 0


def test_tuned_sets():
    chars, offs, sb = with_edges(*gen.batched(40, 1, 50_000, kinds=("random", "url", "dna"),
                                              seed=35))
    rng = np.random.default_rng(5)
    rows = [(int(rng.choice([7, 63, 255, 1023])), int(rng.choice([64, 256, 1024, 2048])),
             int(rng.choice([64, 1024, 4096]))) for _ in range(sb.size - 1)]
    rows[1] = (0, 0, 0)  # defaults from the config
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb),
                                tuning=s5.make_tuning(rows))
    check(chars, offs, sb, perm, lcp, "tuned")


def test_tuned_rejects_bad_entries():
    chars, offs, sb = gen.batched(4, 10, 100, seed=36)
    for bad in [(100, 0, 0), (0, 32, 0), (0, 4096, 0), (0, 0, 100)]:
        rows = [(0, 0, 0)] * 4
        rows[2] = bad
        with pytest.raises(s5.S5Error):
            s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), tuning=s5.make_tuning(rows))
