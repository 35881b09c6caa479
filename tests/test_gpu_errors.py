"""Error paths and output writes, through the C-ABI on the GPU.

* Device-side argument checks: an offset at or past chars_len, an arena whose
  last byte is not a terminator, and a set table that is not non-decreasing
  within n each end in S5_ERR_INVALID with nothing written past the outputs.
* A planner capacity check that fails (a capacity shrunk by the test hook
  s5_debug_limit_capacity) ends in S5_ERR_DEVICE, in the host-driven sort and
  in the graph-captured batched sort, with every kernel exiting normally: the
  same process then sorts correctly again.  The planner writes nothing for a
  workgroup whose allocation failed (it returns before emitting any record),
  and every later kernel exits once the status word is set.
* Read-back fallback: with the per-level counter publications made to miss the
  flag the host polls (test hook s5_debug_miss_publish), every read-back waits,
  finds the stream drained and copies the counters instead; host-driven and
  batched sorts stay exact.
* Write counts (the write-check build): every out_perm slot is written exactly
  once, every out_lcp slot once or twice (a bucket boundary is flagged by the
  redistribution, then completed), and no output write lands outside the two
  arrays.
"""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from paper_1305_1157_amd import gen, s5  # noqa: E402

GUARD = 4096
PATTERN = 0xA5A5A5A5
CAP_LARGE, CAP_BASE0 = 0, 1


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _guarded(n, dev):
    """Output tensors of n + GUARD entries filled with PATTERN."""
    return (torch.full((n + GUARD,), PATTERN, dtype=torch.uint32, device=dev),
            torch.full((n + GUARD,), PATTERN, dtype=torch.uint32, device=dev))


def _guard_intact(*ts):
    n = ts[0].numel() - GUARD
    return all(bool((t[n:] == PATTERN).all()) for t in ts)


def _sort_ex(lib, dc, chars_len, do, n, perm, lcp, cfg=None):
    return lib.s5_sort_ex(_p(dc), chars_len, _p(do), n, _p(perm), _p(lcp),
                          ctypes.byref(cfg) if cfg is not None else None, None, 0,
                          s5._stream())


def _sort_batched(lib, dc, chars_len, do, sb, perm, lcp, cfg=None):
    return lib.s5_sort_batched(_p(dc), chars_len, _p(do), _p(sb), sb.numel() - 1, _p(perm),
                               _p(lcp), ctypes.byref(cfg) if cfg is not None else None,
                               s5._stream())


# byte keys; DNA with the alphabet sampled first (its sample reads no byte at
# or past chars_len) and packed codes
@pytest.mark.parametrize("name,cfg", [
    ("url_10M", None), ("dna_16M", s5.make_config(alphabet=s5.ALPHABET_AUTO))],
    ids=["bytes", "alphabet_auto"])
def test_offset_past_arena_is_invalid(name, cfg):
    lib = s5.load()
    chars, offs = gen.workload(name, 30_000)
    n = offs.size
    dc = to_dev(chars)
    perm, lcp = _guarded(n, dc.device)
    bad = offs.copy()
    bad[n // 2] = chars.size  # one past the end
    rc = _sort_ex(lib, dc, chars.size, to_dev(bad), n, perm, lcp, cfg)
    torch.cuda.synchronize()
    assert rc == s5.S5_ERR_INVALID
    assert _guard_intact(perm, lcp)
    # the same offsets with the arena length unknown are the caller's
    # responsibility; the valid table sorts
    rc = _sort_ex(lib, dc, chars.size, to_dev(offs), n, perm, lcp, cfg)
    torch.cuda.synchronize()
    assert rc == s5.S5_OK
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(perm[:n].cpu().numpy(), rp) and np.array_equal(lcp[:n].cpu().numpy(), rl)


def test_unterminated_arena_is_invalid():
    lib = s5.load()
    chars, offs = gen.from_strings([b"abc", b"abd", b"x" * 40])
    chars = chars[:-1].copy()  # drop the last terminator
    dc = to_dev(np.concatenate([chars, np.zeros(8, np.uint8)]))
    perm, lcp = _guarded(3, dc.device)
    assert _sort_ex(lib, dc, chars.size, to_dev(offs), 3, perm, lcp) == s5.S5_ERR_INVALID
    torch.cuda.synchronize()
    assert _guard_intact(perm, lcp)
    # with the terminator inside the stated length it sorts
    assert _sort_ex(lib, dc, chars.size + 1, to_dev(offs), 3, perm, lcp) == s5.S5_OK
    torch.cuda.synchronize()
    assert perm[:3].cpu().tolist() == [0, 1, 2]


@pytest.mark.parametrize("table", [[0, 1000, 20], [0, 15, 10, 20], [0, 5, 3, 3, 20]])
def test_bad_set_table_is_invalid(table):
    lib = s5.load()
    chars, offs = gen.workload("random_1M", 20)
    dc = to_dev(chars)
    perm, lcp = _guarded(20, dc.device)
    sb = to_dev(np.array(table, dtype=np.uint64))
    rc = _sort_batched(lib, dc, chars.size, to_dev(offs), sb, perm, lcp)
    torch.cuda.synchronize()
    assert rc == s5.S5_ERR_INVALID
    assert _guard_intact(perm, lcp)


def test_set_table_past_offsets_rejected_by_binding():
    # n = set_begin[num_sets] larger than the offsets given: no offsets length
    # crosses the ABI, so the binding checks it before the call
    chars, offs = gen.workload("random_1M", 20)
    with pytest.raises(ValueError):
        s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(np.array([0, 20, 25], np.uint64)))
    with pytest.raises(ValueError):
        s5.sort(to_dev(chars), to_dev(offs), out_perm=torch.empty(19, dtype=torch.uint32,
                                                                   device="cuda"))


def _device_failure(which, limit, name, n, batched):
    lib = s5.load()
    chars, offs = gen.workload(name, n)
    dc, do = to_dev(chars), to_dev(offs)
    perm, lcp = _guarded(n, dc.device)
    assert lib.s5_debug_limit_capacity(which, limit) == s5.S5_OK
    try:
        print(f"capacity {which} <= {limit}: {name} n={n} batched={batched}", flush=True)
        if batched:
            sb = to_dev(np.array([0, n // 3, n], dtype=np.uint64))
            rc = _sort_batched(lib, dc, chars.size, do, sb, perm, lcp)
        else:
            rc = _sort_ex(lib, dc, chars.size, do, n, perm, lcp)
        torch.cuda.synchronize()
        assert rc == s5.S5_ERR_DEVICE, s5.load().s5_strerror(rc)
        st = s5.Stats()
        assert lib.s5_stats_get(s5._stream(), ctypes.byref(st)) == s5.S5_ERR_DEVICE
        assert _guard_intact(perm, lcp)
    finally:
        assert lib.s5_debug_limit_capacity(which, 0) == s5.S5_OK
    # every kernel exited normally: the next sort in this process is exact
    p2, l2 = s5.sort(dc, do)
    torch.cuda.synchronize()
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(p2.cpu().numpy(), rp) and np.array_equal(l2.cpu().numpy(), rl)


@pytest.mark.parametrize("batched", [False, True])
def test_large_segment_capacity_failure(batched):
    _device_failure(CAP_LARGE, 1, "url_10M", 200_000, batched)


@pytest.mark.parametrize("batched", [False, True])
def test_base_item_capacity_failure(batched):
    _device_failure(CAP_BASE0, 1, "words_50M", 100_000, batched)


def test_read_back_fallback():
    lib = s5.load()
    chars, offs = gen.workload("url_10M", 40_000)
    dc, do = to_dev(chars), to_dev(offs)
    # tiny trees and base cases: several levels, each read back
    cfg = s5.make_config(splitters=31, base_threshold=64, tile=64)
    sb_host = np.array([0, 15_000, 40_000], dtype=np.uint64)
    bcfg = s5.make_config(splitters=31, base_threshold=64, tile=64, graph_levels=1)
    assert lib.s5_debug_miss_publish(1) == s5.S5_OK
    try:
        print("read-back fallback: url n=40000, host-driven and batched", flush=True)
        p1, l1 = s5.sort(dc, do, cfg=cfg)
        torch.cuda.synchronize()
        passes = s5.stats()["passes"]
        p2, l2 = s5.sort_batched(dc, do, to_dev(sb_host), cfg=bcfg)
        torch.cuda.synchronize()
    finally:
        assert lib.s5_debug_miss_publish(0) == s5.S5_OK
    assert passes >= 3
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(p1.cpu().numpy(), rp) and np.array_equal(l1.cpu().numpy(), rl)
    bp, bl = oracle.sort_batched(chars, offs, sb_host)
    assert np.array_equal(p2.cpu().numpy(), bp) and np.array_equal(l2.cpu().numpy(), bl)


def _counted(run, n, dev):
    """Run `run(lib, perm, lcp)` on the write-check build with counting on."""
    lib = s5.load_wcheck()
    perm = torch.empty(n, dtype=torch.uint32, device=dev)
    lcp = torch.empty(n, dtype=torch.uint32, device=dev)
    pc = torch.zeros(n, dtype=torch.uint32, device=dev)
    lc = torch.zeros(n, dtype=torch.uint32, device=dev)
    stray = torch.zeros(1, dtype=torch.uint32, device=dev)
    assert lib.s5_debug_count_writes(_p(perm), _p(lcp), n, _p(pc), _p(lc), _p(stray)) == s5.S5_OK
    try:
        assert run(lib, perm, lcp) == s5.S5_OK
        torch.cuda.synchronize()
    finally:
        lib.s5_debug_count_writes(None, None, 0, None, None, None)
    return perm.cpu().numpy(), lcp.cpu().numpy(), pc.cpu().numpy(), lc.cpu().numpy(), \
        int(stray.item())


CASES = [("url_10M", 200_000, None), ("dna_16M", 100_000, None),
         ("words_50M", 300_000, s5.make_config(base_threshold=128, splitters=31)),
         ("random_1M", 100_000, s5.make_config(splitter_mode=s5.SPLIT_LEARNED)),
         ("url_10M", 150_001, s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS, splitters=63,
                                             base_threshold=128))]


@pytest.mark.parametrize("name,n,cfg", CASES,
                         ids=[c[0] + ("_two_pass" if c[2] is not None and c[2].distribution else "")
                              for c in CASES])
def test_every_output_slot_written_once(name, n, cfg):
    chars, offs = gen.workload(name, n)
    dc, do = to_dev(chars), to_dev(offs)
    perm, lcp, pc, lc, stray = _counted(
        lambda lib, p, l: _sort_ex(lib, dc, chars.size, do, n, p, l, cfg), n, dc.device)
    rp, rl = oracle.sort(chars, offs)
    assert np.array_equal(perm, rp) and np.array_equal(lcp, rl)
    assert stray == 0
    assert np.all(pc == 1), f"perm slots written {np.bincount(pc)} times"
    assert np.all((lc == 1) | (lc == 2)), f"lcp slots written {np.bincount(lc)} times"


def test_every_output_slot_written_once_batched():
    chars, offs, sb = gen.batched(40, 1, 60_000, kinds=("random", "url", "dna"), seed=31)
    n = offs.size
    dc, do, dsb = to_dev(chars), to_dev(offs), to_dev(sb)
    perm, lcp, pc, lc, stray = _counted(
        lambda lib, p, l: _sort_batched(lib, dc, chars.size, do, dsb, p, l), n, dc.device)
    rp, rl = oracle.sort_batched(chars, offs, sb)
    assert np.array_equal(perm, rp) and np.array_equal(lcp, rl)
    assert stray == 0 and np.all(pc == 1) and np.all((lc == 1) | (lc == 2))


def test_product_build_does_not_count():
    assert s5.load().s5_debug_count_writes(None, None, 0, None, None, None) == s5.S5_ERR_INVALID
