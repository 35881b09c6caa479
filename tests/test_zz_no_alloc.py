"""The sort without allocations (``s5_sort_static``) against ``s5_sort_ex`` with a
caller workspace: identical permutation and LCP array on two calls in a row (the
second smaller, so it runs on the first call's leftover scratch contents), and
a clean error for a sort larger than the static array."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
from gpu_util import to_dev  # noqa: E402
from paper_1305_1157_amd import gen, s5  # noqa: E402


def _both(chars, offs, cfg=None):
    """(static perm, static lcp, ex perm, ex lcp) as host arrays."""
    dc, do = to_dev(chars), to_dev(offs)
    n = offs.size
    ws = torch.empty(s5.workspace_bytes(n, cfg), dtype=torch.uint8, device=dc.device)
    ep, el = s5.sort(dc, do, cfg=cfg, workspace=ws)
    sp = torch.full((n,), 0xFFFFFFFF, dtype=torch.uint32, device=dc.device)
    sl = torch.full((n,), 0xFFFFFFFF, dtype=torch.uint32, device=dc.device)
    rc = s5.sort_static(dc, do, sp, sl, cfg=cfg)
    assert rc == s5.S5_OK, s5.load().s5_strerror(rc)
    torch.cuda.synchronize()
    return sp.cpu().numpy(), sl.cpu().numpy(), ep.cpu().numpy(), el.cpu().numpy()


def test_static_equals_ex_twice_second_smaller():
    cases = [("url_10M", 400_000, None), ("dna_16M", 60_000, s5.make_config(base_threshold=256))]
    for name, n, cfg in cases:
        chars, offs = gen.workload(name, n)
        print(f"static sort: {name} n={n}", flush=True)
        sp, sl, ep, el = _both(chars, offs, cfg)
        assert np.array_equal(sp, ep), f"{name}: perm differs from s5_sort_ex"
        assert np.array_equal(sl, el), f"{name}: lcp differs from s5_sort_ex"
        rp, rl = oracle.sort(chars, offs)
        assert np.array_equal(sp, rp) and np.array_equal(sl, rl), f"{name}: differs from the oracle"
        st = s5.stats()
        assert st["passes"] >= 1 and st["workspace_bytes"] <= s5.STATIC_SCRATCH_BYTES


def test_static_learned_mode():
    chars, offs = gen.workload("words_50M", 300_000)
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED)
    sp, sl, ep, el = _both(chars, offs, cfg)
    assert np.array_equal(sp, ep) and np.array_equal(sl, el)


def test_static_rejects_too_large():
    n = 2_000_000
    assert s5.workspace_bytes(n) > s5.STATIC_SCRATCH_BYTES
    chars, offs = gen.workload("random_1M", n)
    dc, do = to_dev(chars), to_dev(offs)
    sp = torch.full((n,), 7, dtype=torch.uint32, device=dc.device)
    sl = torch.full((n,), 7, dtype=torch.uint32, device=dc.device)
    assert s5.sort_static(dc, do, sp, sl) == s5.S5_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert bool((sp == 7).all()) and bool((sl == 7).all())  # nothing written


def test_static_empty_and_single():
    dc = to_dev(np.zeros(8, np.uint8))
    for n in (0, 1):
        do = to_dev(np.zeros(n, np.uint64))
        sp = torch.full((n,), 5, dtype=torch.uint32, device=dc.device)
        sl = torch.full((n,), 5, dtype=torch.uint32, device=dc.device)
        assert s5.sort_static(dc, do, sp, sl) == s5.S5_OK
        torch.cuda.synchronize()
        assert sp.cpu().tolist() == [0] * n and sl.cpu().tolist() == [0] * n
