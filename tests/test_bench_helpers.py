"""The benchmark's measurement helpers on the CPU: the distinguishing prefix D
that bench.py computes from a sort's output (torch ops) against the oracle's
explicit per-string definition, single and batched; the algorithmic byte
counts; the roofline parsed from a rocprofv3 summary."""
import os

import numpy as np
import torch

import bench
import oracle
from paper_1305_1157_amd import gen


def test_dist_prefix_matches_oracle():
    for name, n in (("url_10M", 30_000), ("dna_16M", 5_000), ("random_1M", 20_000)):
        chars, offs = gen.workload(name, n)
        p, l = oracle.sort(chars, offs)
        want = oracle.dist_prefix(chars, offs, p, l)
        for chunk in (1 << 30, 4093):  # the arena scanned whole and in chunks
            got = bench.dist_prefix(torch.from_numpy(chars), torch.from_numpy(offs),
                                    torch.from_numpy(p), torch.from_numpy(l), chunk=chunk)
            assert got == want


def test_dist_prefix_batched_matches_oracle():
    chars, offs, sb = gen.batched(25, 1, 4000, seed=9)
    p, l = oracle.sort_batched(chars, offs, sb)
    got = bench.dist_prefix(torch.from_numpy(chars), torch.from_numpy(offs), torch.from_numpy(p),
                            torch.from_numpy(l), torch.from_numpy(sb))
    want = sum(oracle.dist_prefix(chars, offs[int(sb[s]):int(sb[s + 1])], p[int(sb[s]):int(sb[s + 1])],
                                  l[int(sb[s]):int(sb[s + 1])])
               for s in range(sb.size - 1) if sb[s + 1] > sb[s])
    assert got == want


def test_hbm_figures():
    h = bench.hbm_figures(D=1000, n=10, moved=20, sec=1e-6, copy_gbps=4000.0)
    assert h["B_min_bytes"] == 1000 + 160 and h["B_alg_bytes"] == 1160 + 480
    assert abs(h["B_alg_GBps"] - 1640 / 1e-6 / 1e9) < 1e-9
    assert abs(h["B_alg_pct_peak"] - 100 * h["B_alg_GBps"] / 8000) < 1e-9
    assert abs(h["B_alg_pct_copy"] - 100 * h["B_alg_GBps"] / 4000) < 1e-9


def test_profile_roofline_parses_summary(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "k.txt").write_text(
        "# header\n"
        "kernel                          calls     total_us     avg_us\n"
        "k_scatter<true, false>             10       1000.0      100.0\n"
        "k_scatter<true, true>               2        500.0      250.0\n"
        "k_classify<4, true>                12        100.0        8.3\n"
        "sorts 2\n")
    src = tmp_path / "paper_1305_1157_amd" / "csrc"
    src.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        (src / name).write_text("x")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    r = bench.profile_roofline("k.txt", moved=600)
    assert r["launches_per_sort"] == 6 and abs(r["avg_launch_us"] - 125.0) < 1e-9
    assert abs(r["alg_bytes_per_launch"] - 24 * 600 / 6) < 1e-9
    assert abs(r["achieved"] - 2400 / 125e-6 / 1e9) < 1e-9
    assert r["profile_matches_kernel_source"] is False
    assert bench.profile_roofline("missing.txt", 1) is None
