#!/usr/bin/env python3
"""Benchmark of S^5 on one MI355X: strings/s and HBM GB/s.

One step = one complete sort (every distribution pass, the base case and the
LCP completion) of the URL-like workload: 10,000,000 synthetic strings
"http://" + host (Zipf s=1.1 over 50,000 hosts of 6-20 letters) + ".com" +
1-6 path segments of 3-12 [a-z0-9] characters, seeded, resident in HBM.  The
JSON line carries the roofline of the dominant kernel (the redistribution
pass, timed with HIP events inside the library on its launch stream) and the
CPU oracle timed on a bounded sample of the same workload.

Beside it (skip with --no-extras): the learned splitter proposal against
sampled splitters on the DNA and word workloads (their outputs compared), and
the batched form (4,096 sets in one graph launch, autotuned per-set
parameters), each with its own strings/s.  Only the CPU baseline uses the
oracle; the full-size correctness checks are GPU tests.
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


def pmc_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    PMC summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is
    none for this workload or the kernels changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_{DOMINANT_SYMBOL}_{workload}.txt")
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 3 and parts[0] == "traffic_bytes_per_launch" and parts[1] == DOMINANT_SYMBOL:
            vals["traffic"] = float(parts[2])
        if len(parts) == 2 and parts[0] == "kernel_source_sha256":
            vals["sha"] = parts[1]
    src = os.path.join(ROOT, "paper_1305_1157_amd", "csrc", "s5_kernels.hip")
    now = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if "traffic" not in vals or vals.get("sha") != now:
        return None, f"{os.path.relpath(path, ROOT)} is stale (kernel source changed)"
    return vals["traffic"], os.path.relpath(path, ROOT)


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


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _timed_sorts(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def learned_extra(name, steps=3):
    """Learned vs sampled splitters on one workload (same output, checked)."""
    import torch
    from paper_1305_1157_amd import gen, s5
    chars, offs = gen.workload(name)
    n = int(offs.size)
    dc, do = torch.from_numpy(chars).cuda(), torch.from_numpy(offs).cuda()
    perm = torch.empty(n, dtype=torch.uint32, device="cuda")
    lcp = torch.empty_like(perm)
    res, ref = {"workload": WORKLOAD_TEXT[name], "name": name, "n": n}, None
    variants = [("sampled", s5.make_config()),
                ("learned", s5.make_config(splitter_mode=s5.SPLIT_LEARNED)),
                ("learned_no_fallback", s5.make_config(splitter_mode=s5.SPLIT_LEARNED,
                                                       imbalance_bound=1e9))]
    for label, cfg in variants:
        log(f"{name}: {label}")
        ws = torch.empty(s5.workspace_bytes(n, cfg), dtype=torch.uint8, device="cuda")
        run = lambda: s5.sort(dc, do, cfg=cfg, out_perm=perm, out_lcp=lcp, workspace=ws)  # noqa
        run()
        sec = _timed_sorts(run, steps)
        st = s5.stats()
        s5.profile_enable(True)
        run()
        torch.cuda.synchronize()
        prof = s5.profile_read()
        s5.profile_enable(False)
        if ref is None:
            ref = (perm.clone(), lcp.clone())
        same = bool(torch.equal(ref[0], perm) and torch.equal(ref[1], lcp))
        res[label] = {"value": n / sec, "ms": sec * 1e3, "passes": st["passes"],
                      "moved_M": st["moved_M"], "fallbacks": st["fallbacks"],
                      "entropy_bits_first_pass": st["entropy_bits"],
                      "max_bucket_first_pass": st["max_bucket"],
                      "learn_ms": prof.get("learn_splitters", {}).get("total_ms", 0.0),
                      "output_identical_to_sampled": same}
        del ws
    return res


def batched_extra(steps=3, learned=None):
    """The batched form on 4,096 sets in one graph launch (learned: only that
    variant, else all three)."""
    import numpy as np
    import torch
    from paper_1305_1157_amd import autotune, gen, s5
    spec = gen.BATCHED["sets_4096"]
    t0 = time.perf_counter()
    chars, offs, sb = gen.batched(**spec)
    gen_s = time.perf_counter() - t0
    n, sizes = int(offs.size), np.diff(sb).astype(np.int64)
    log(f"batched: generated {n:,} strings in {len(sizes)} sets ({gen_s:.1f} s)")
    dc, do, ds = (torch.from_numpy(chars).cuda(), torch.from_numpy(offs).cuda(),
                  torch.from_numpy(sb).cuda())
    perm = torch.empty(n, dtype=torch.uint32, device="cuda")
    lcp = torch.empty_like(perm)
    table = autotune.load_table()
    tuned = s5.make_tuning(autotune.tuning_for(sizes, table))
    res = {"workload": f"{spec['num_sets']:,} independent sets, sizes log-uniform in "
                       f"[{spec['min_size']:,}, {spec['max_size']:,}], each from one of the "
                       f"{'/'.join(spec['kinds'])} generators", "n": n, "sets": len(sizes),
           "arena_bytes": int(chars.size), "generate_s": gen_s, "tuning": table.get("source"),
           "unroll": table["unroll"], "launches": "one hipGraph per sort (host reads back "
           "set_begin ends and the final counters)"}
    variants = [("learned_tuned", s5.make_config(splitter_mode=s5.SPLIT_LEARNED,
                                                  unroll=table["unroll"]), tuned),
                ("sampled_tuned", s5.make_config(unroll=table["unroll"]), tuned),
                ("sampled_defaults", s5.make_config(), None)]
    if learned is not None:
        variants = [v for v in variants if v[0] == ("learned_tuned" if learned else "sampled_tuned")]
    for label, cfg, tun in variants:
        log(f"batched: {label}")
        run = lambda: s5.sort_batched(dc, do, ds, cfg=cfg, tuning=tun, out_perm=perm,  # noqa
                                      out_lcp=lcp)
        run()  # capture
        sec = _timed_sorts(run, steps)
        st = s5.stats()
        res[label] = {"value": n / sec, "ms": sec * 1e3, "passes": st["passes"],
                      "moved_M": st["moved_M"], "fallbacks": st["fallbacks"],
                      "segments": st["segments"], "base_items": st["base_items"]}
    res["check"] = ("tests/test_gpu_fullsize.py checks this workload at full size "
                    "(permutation per set, sampled neighbour pairs, whole small sets)")
    return res


def batched_main(args):
    """The batched workload as the main line: whole-job strings/s of one graph
    launch per sort (autotuned per-set parameters)."""
    res = batched_extra(steps=args.steps, learned=args.learned)
    label = "learned_tuned" if args.learned else "sampled_tuned"
    r = res[label]
    out = {
        "metric": "strings/s and HBM GB/s (% peak), plain vs learned-splitter vs batched S^5",
        "value": r["value"], "unit": "strings/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": r["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": res["workload"], "name": "sets_4096", "n": res["n"],
                   "sets": res["sets"], "arena_bytes": res["arena_bytes"],
                   "variant": "batched S^5 in one hipGraph, " +
                   ("learned splitters per set with sampled fallback" if args.learned
                    else "sampled splitters") + ", autotuned per-set parameters"},
        "roofline": None,
        "roofline_note": "kernels inside one graph launch are not bracketed by events; "
                         "per-kernel durations come from rocprofv3 (profiles/)",
        "batched": res,
    }
    print(json.dumps(out), flush=True)


def arg_parser():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="url_10M", choices=sorted(WORKLOAD_TEXT) + ["sets_4096"],
                    help="sets_4096: the batched form (one graph launch per sort) as the main line")
    ap.add_argument("--learned", action="store_true",
                    help="learned splitter proposal (with its sampled fallback) for the main line")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="strings in the oracle's timed sample (0 = skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run one plain device copy of this size (PMC calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the learned-splitter and batched measurements")
    return ap


def main():
    args = arg_parser().parse_args()
    if args.gpus != 1:
        print(f"bench.py: the sort runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1305_1157_amd import gen, s5

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.workload == "sets_4096":
        batched_main(args)
        return
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED if args.learned else s5.SPLIT_SAMPLED)
    chars, offs = gen.workload(args.workload)
    n = int(offs.size)
    d_chars = torch.from_numpy(chars).to(dev)
    d_offs = torch.from_numpy(offs).to(dev)
    perm = torch.empty(n, dtype=torch.uint32, device=dev)
    lcp = torch.empty(n, dtype=torch.uint32, device=dev)
    ws = torch.empty(s5.workspace_bytes(n, cfg), dtype=torch.uint8, device=dev)
    if args.copy_probe_mib:
        a = torch.empty(args.copy_probe_mib << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for _ in range(args.warmup):
        s5.sort(d_chars, d_offs, cfg=cfg, out_perm=perm, out_lcp=lcp, workspace=ws)
    torch.cuda.synchronize()
    # timed region: HIP events bracket only the dominant kernel's launches
    s5.profile_enable(True)
    s5.profile_only(DOMINANT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s5.sort(d_chars, d_offs, cfg=cfg, out_perm=perm, out_lcp=lcp, workspace=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof_dom = s5.profile_read()[DOMINANT]
    st = s5.stats()
    # per-kernel breakdown from a separate profiled run (every kernel timed)
    s5.profile_only(None)
    s5.profile_enable(True)
    for _ in range(3):
        s5.sort(d_chars, d_offs, cfg=cfg, out_perm=perm, out_lcp=lcp, workspace=ws)
    torch.cuda.synchronize()
    prof = s5.profile_read()
    s5.profile_enable(False)
    prof_steps = 3

    ms_per_step = dt * 1e3 / args.steps
    value = n * args.steps / dt
    h_perm, h_lcp = perm.cpu().numpy(), lcp.cpu().numpy()
    D = dist_prefix_from_output(chars, offs, h_perm, h_lcp)
    b_min = D + 16 * n
    b_alg = b_min + 24 * st["moved_M"]
    sec = ms_per_step / 1e3
    dom = prof_dom
    avg_ms = dom["total_ms"] / dom["launches"]
    achieved = (dom["alg_bytes"] / dom["launches"]) / (avg_ms / 1e3) / 1e9
    traffic, traffic_src = pmc_traffic(args.workload)
    kernels = {k: {"launches_per_step": v["launches"] / prof_steps,
                   "ms_per_step": v["total_ms"] / prof_steps,
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
                   "arena_bytes": int(chars.size), "D": D,
                   "variant": "S^5, learned splitter proposal with sampled fallback" if args.learned
                   else "plain S^5, sampled splitters",
                   "splitters_max": 255, "base_threshold": 1024},
        "hbm": {"B_min_bytes": b_min, "B_alg_bytes": b_alg, "moved_M": st["moved_M"],
                "passes": st["passes"], "B_min_GBps": b_min / sec / 1e9,
                "B_alg_GBps": b_alg / sec / 1e9,
                "B_alg_pct_peak": 100 * b_alg / sec / 1e9 / HBM_PEAK_GBPS},
        "roofline": {"kernel": DOMINANT_SYMBOL, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "traffic_source": traffic_src,
                     "avg_launch_us": avg_ms * 1e3,
                     "launches_per_step": dom["launches"] / args.steps,
                     "alg_bytes_per_launch": dom["alg_bytes"] / dom["launches"]},
        "kernels": kernels,
        "stats": st,
    }
    log(f"{args.workload}: {value / 1e9:.3f} G strings/s, {ms_per_step:.3f} ms per sort")
    if args.cpu_sample:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, min(args.cpu_sample, n))
    if not args.no_extras:
        del d_chars, d_offs, perm, lcp, ws
        torch.cuda.empty_cache()
        extras = {}
        for name in ("dna_16M", "words_50M"):
            try:
                extras[name] = learned_extra(name)
            except Exception as e:  # reported, never hides the main line
                extras[name] = {"error": repr(e)}
            torch.cuda.empty_cache()
        out["learned"] = extras
        try:
            out["batched"] = batched_extra()
        except Exception as e:
            out["batched"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
