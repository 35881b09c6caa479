#!/usr/bin/env python3
"""Benchmark of plain S^5 on one MI355X: strings/s and HBM GB/s.

One step = one complete sort (every distribution pass, the base case and the
LCP completion) of the URL-like workload: 10,000,000 synthetic strings
"http://" + host (Zipf s=1.1 over 50,000 hosts of 6-20 letters) + ".com" +
1-6 path segments of 3-12 [a-z0-9] characters, seeded, resident in HBM.  The
JSON line carries the roofline of the dominant kernel (the redistribution
pass, timed with HIP events inside the library on its launch stream) and the
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
DOMINANT = "scatter"          # library name of the dominant kernel
DOMINANT_SYMBOL = "k_scatter"  # its symbol in rocprofv3 traces
WORKLOAD_TEXT = {
    "url_10M": "10,000,000 URL-like strings: 'http://' + host (Zipf s=1.1 over 50,000 hosts "
               "of 6-20 lowercase letters) + '.com' + 1-6 path segments of 3-12 [a-z0-9] "
               "chars; uint64 offsets into one null-terminated arena",
    "random_1M": "1,000,000 random strings, length uniform in [8,20], bytes uniform 'a'..'z'",
    "dna_16M": "16,000,000 DNA reads of 100 bases, order-3 Markov chain, 10% exact duplicates",
    "words_50M": "50,000,000 words drawn Zipf(s=1.0) from a 1,000,000-word vocabulary",
}


def dist_prefix_from_output(chars, offs, perm, lcp):
    """D = sum over strings of min(|s|, max(lcp with sorted neighbours) + 1), |s| with the
    terminator (Section 2), evaluated on the sort's own output."""
    import numpy as np
    zeros = np.flatnonzero(chars == 0)
    lens = zeros[np.searchsorted(zeros, offs)] - offs.astype(np.int64)  # without terminator
    l = lcp.astype(np.int64)
    r = np.empty_like(l)
    r[:-1] = l[1:]
    r[-1] = 0
    m = np.maximum(l, r) + 1
    return int(np.minimum(m, lens[perm.astype(np.int64)] + 1).sum())


def cpu_baseline(name, n_sample, min_seconds=10.0):
    """The oracle, untuned, on one host core over the first ``n_sample`` strings of
    the same seeded recipe, repeated until at least ``min_seconds`` of CPU work."""
    import oracle
    from paper_1305_1157_amd import gen
    chars, offs = gen.workload(name, n_sample)
    reps, total = 0, 0.0
    while total < min_seconds and reps < 50:
        t0 = time.perf_counter()
        oracle.sort(chars, offs)
        total += time.perf_counter() - t0
        reps += 1
    return {"value": n_sample * reps / total, "unit": "strings/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample:,} strings of the same seeded {name} recipe, sorted "
                      f"{reps} times by the oracle (multikey quicksort + LCP pass), "
                      f"{total:.1f} s total on 1 host core"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="url_10M", choices=sorted(WORKLOAD_TEXT))
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="strings in the oracle's timed sample (0 = skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1305_1157_amd import gen, s5

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    chars, offs = gen.workload(args.workload)
    n = int(offs.size)
    d_chars = torch.from_numpy(chars).to(dev)
    d_offs = torch.from_numpy(offs).to(dev)
    perm = torch.empty(n, dtype=torch.uint32, device=dev)
    lcp = torch.empty(n, dtype=torch.uint32, device=dev)
    ws = torch.empty(s5.workspace_bytes(n), dtype=torch.uint8, device=dev)
    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        s5.sort(d_chars, d_offs, out_perm=perm, out_lcp=lcp, workspace=ws)
    torch.cuda.synchronize()
    s5.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s5.sort(d_chars, d_offs, out_perm=perm, out_lcp=lcp, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = s5.profile_read()
    s5.profile_enable(False)
    st = s5.stats()

    ms_per_step = dt * 1e3 / args.steps
    value = n * args.steps / dt
    h_perm, h_lcp = perm.cpu().numpy(), lcp.cpu().numpy()
    D = dist_prefix_from_output(chars, offs, h_perm, h_lcp)
    b_min = D + 16 * n
    b_alg = b_min + 24 * st["moved_M"]
    sec = ms_per_step / 1e3
    dom = prof[DOMINANT]
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = (dom["alg_bytes"] / dom["launches"]) / (avg_ms / 1e3) / 1e9
    kernels = {k: {"launches_per_step": v["launches"] / args.steps,
                   "ms_per_step": v["total_ms"] / args.steps,
                   "avg_launch_us": 1e3 * v["total_ms"] / v["launches"],
                   "alg_GBps": (v["alg_bytes"] / (v["total_ms"] / 1e3) / 1e9) if v["alg_bytes"] else None}
               for k, v in prof.items()}
    out = {
        "metric": "strings/s and HBM GB/s (% peak), plain vs learned-splitter vs batched S^5",
        "value": value,
        "unit": "strings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "name": args.workload, "n": n,
                   "arena_bytes": int(chars.size), "D": D, "variant": "plain S^5, sampled splitters",
                   "splitters_max": 255, "base_threshold": 1024},
        "hbm": {"B_min_bytes": b_min, "B_alg_bytes": b_alg, "moved_M": st["moved_M"],
                "passes": st["passes"], "B_min_GBps": b_min / sec / 1e9,
                "B_alg_GBps": b_alg / sec / 1e9,
                "B_alg_pct_peak": 100 * b_alg / sec / 1e9 / HBM_PEAK_GBPS},
        "roofline": {"kernel": DOMINANT_SYMBOL, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": None, "avg_launch_us": avg_ms * 1e3,
                     "launches_per_step": dom["launches"] / args.steps,
                     "alg_bytes_per_launch": dom["alg_bytes"] / dom["launches"]},
        "kernels": kernels,
        "stats": st,
    }
    if args.cpu_sample:
        out["cpu_baseline"] = cpu_baseline(args.workload, min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
