"""C-ABI checks that need no GPU: the library loads and exports every entry
point that ``include/*.h`` declares; host-only calls behave as documented."""
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(s5_[a-z_]+)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_1305_1157_amd import s5
    if not os.path.exists(s5.LIB_PATH):
        from paper_1305_1157_amd import build
        build.build()
    return s5.load()


def test_every_declared_symbol_exported(lib):
    names = declared_functions()
    assert {"s5_sort", "s5_sort_ex", "s5_sort_batched", "s5_workspace_bytes", "s5_stats_get",
            "s5_strerror", "s5_release"} <= names
    for name in names:
        assert hasattr(lib, name), f"{name} not exported"


def test_strerror(lib):
    for rc in (0, -1, -2, -3, -4, -5):
        assert lib.s5_strerror(rc) and lib.s5_strerror(rc) != b"unknown status"
    assert lib.s5_strerror(-99) == b"unknown status"


def test_workspace_bytes(lib):
    from paper_1305_1157_amd import s5
    small = s5.workspace_bytes(1000)
    big = s5.workspace_bytes(1_000_000)
    assert 0 < small < big
    # about 26 B/string of work arrays plus bounded per-pass storage
    assert 26 * 1_000_000 < big < 64 * 1_000_000
    # invalid configurations are rejected (0 bytes)
    assert s5.workspace_bytes(1000, s5.make_config(splitters=100)) == 0
    assert s5.workspace_bytes(1000, s5.make_config(base_threshold=4096)) == 0
    assert s5.workspace_bytes(1000, s5.make_config(unroll=3)) == 0
    assert s5.workspace_bytes(1000, s5.make_config(splitters=1023, unroll=8)) > 0
    assert s5.workspace_bytes(1000, s5.make_config(distribution=2)) == 0
    # the two-pass distribution holds a second bucket-id array (2 bytes a string)
    two = s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS)
    assert s5.workspace_bytes(1_000_000, two) >= s5.workspace_bytes(1_000_000) + 2_000_000


def test_static_sort_size_limit_is_host_logic(lib):
    """s5_sort_static rejects a sort whose workspace exceeds its static array
    before any device work (the pointers are never touched, so this runs
    without a GPU)."""
    from paper_1305_1157_amd import s5
    n = 2_000_000
    assert s5.workspace_bytes(n) > s5.STATIC_SCRATCH_BYTES >= s5.workspace_bytes(1_000_000)
    fake = 4096  # never dereferenced: the size check comes first
    assert lib.s5_sort_static(fake, 0, fake, n, fake, fake, None, None) == s5.S5_ERR_TOO_LARGE
    cfg = s5.make_config(base_threshold=64)
    assert lib.s5_sort_static(fake, 0, fake, 1_000_000, fake, fake, cfg, None) == \
        s5.S5_ERR_TOO_LARGE
    assert lib.s5_sort_static(None, 0, None, 5, None, None, None, None) == s5.S5_ERR_INVALID


def test_batched_sorts_refuse_two_pass_distribution(lib):
    """The two-pass distribution is host-driven only; batched sorts reject the
    config before any device work (never-dereferenced pointers, no GPU)."""
    import ctypes
    from paper_1305_1157_amd import s5
    fake = 4096
    cfg = s5.make_config(distribution=s5.DISTRIBUTE_TWO_PASS)
    assert lib.s5_sort_batched(fake, 0, fake, fake, 1, fake, fake, ctypes.byref(cfg), None) == \
        s5.S5_ERR_INVALID
