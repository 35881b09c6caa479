#!/usr/bin/env python3
"""Benchmark of S^5 on one MI355X: strings/s and HBM GB/s.

One step = one complete sort (every distribution pass, the base case and the
LCP completion) of the URL-like workload: 10,000,000 synthetic strings
"http://" + host (Zipf s=1.1 over 50,000 hosts of 6-20 letters) + ".com" +
1-6 path segments of 3-12 [a-z0-9] characters, seeded, resident in HBM.  The
JSON line carries the roofline of the dominant kernel (the redistribution
pass, timed with HIP events inside the library on its launch stream) and the
CPU oracle timed on a bounded sample of the same workload.

Beside it (skip with --no-extras): plain S^5 on the random strings, the
learned splitter proposal against sampled splitters on the DNA and word
workloads (their outputs compared), and the batched form (4,096 sets in one
graph launch, autotuned per-set parameters), each with its strings/s, its
distinguishing prefix D and its algorithmic HBM bytes and rates (B_min, B_alg,
% of 8 TB/s and of a measured device copy).  Only the CPU baselines use the
oracle (one core for the main line, every core over whole sets for the
batched form); the full-size correctness checks are GPU tests.
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


# device sources of the library's kernels; a committed profile records their
# hash (kernel_source_sha256) and counts as stale once any of them changes
KERNEL_SOURCES = ("s5_kernels.hip", "s5_word.h", "s5_internal.h")


def kernel_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1305_1157_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def pmc_traffic(workload):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    PMC summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None if there is
    none for this workload or the kernels changed since it was taken."""
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
    if "traffic" not in vals or vals.get("sha") != kernel_source_sha256():
        return None, f"{os.path.relpath(path, ROOT)} is stale (kernel source changed)"
    return vals["traffic"], os.path.relpath(path, ROOT)


def dist_prefix(d_chars, d_offs, perm, lcp, d_sb=None, chunk=1 << 30):
    """D = sum over strings of min(|s|, max(lcp with sorted neighbours) + 1), |s| with the
    terminator (Section 2), evaluated on the sort's own output (device tensors;
    batched: set-local perm, lcp 0 at every set start, d_sb the set table)."""
    import torch
    # terminator positions, ascending (nonzero over chunks of the arena: one
    # call over more than 2^31 elements is not supported)
    zeros = torch.cat([torch.nonzero(d_chars[a:a + chunk] == 0).squeeze(1) + a
                       for a in range(0, d_chars.numel(), chunk)])
    offs = d_offs.view(torch.int64)
    lens = zeros[torch.searchsorted(zeros, offs)] - offs  # bytes before the terminator
    del zeros
    p = perm.view(torch.int32).to(torch.int64)
    if d_sb is not None:
        sb = d_sb.view(torch.int64)
        p += torch.repeat_interleave(sb[:-1], sb[1:] - sb[:-1], output_size=p.numel())
    l = lcp.view(torch.int32).to(torch.int64)
    r = torch.zeros_like(l)
    r[:-1] = l[1:]
    m = torch.maximum(l, r) + 1
    return int(torch.minimum(m, lens[p] + 1).sum())


def hbm_figures(D, n, moved, sec, copy_gbps):
    """Algorithmic bytes of one sort and the rates they give: B_min = D + 16 n
    (offset read, perm and lcp written, distinguishing prefixes), B_alg = B_min +
    24 M (key and index read and written per string per distribution pass)."""
    b_min = D + 16 * n
    b_alg = b_min + 24 * moved
    g_min, g_alg = b_min / sec / 1e9, b_alg / sec / 1e9
    out = {"D": D, "moved_M": moved, "B_min_bytes": b_min, "B_alg_bytes": b_alg,
           "B_min_GBps": g_min, "B_alg_GBps": g_alg,
           "B_min_pct_peak": 100 * g_min / HBM_PEAK_GBPS,
           "B_alg_pct_peak": 100 * g_alg / HBM_PEAK_GBPS}
    if copy_gbps:
        out["B_alg_pct_copy"] = 100 * g_alg / copy_gbps
    return out


def host_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "usable_cores": len(os.sched_getaffinity(0))}


def copy_bandwidth(dev, mib=1024, reps=10):
    """A plain device copy (torch copy_) of ``mib`` MiB, timed with events on the
    stream it runs on: bytes read + written per second."""
    import torch
    a = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbps = 2 * (mib << 20) / (ms / 1e3) / 1e9
    del a, b
    return {"GBps": gbps, "pct_of_peak": 100 * gbps / HBM_PEAK_GBPS, "bytes_per_copy": 2 * (mib << 20),
            "how": f"torch copy_ of a {mib} MiB device buffer, {reps} copies timed with HIP events"}


def profile_roofline(profile, moved, sorts_key="sorts"):
    """Roofline of the redistribution kernel (every instantiation) from a
    committed rocprofv3 summary: average launch duration there, and 24 B per
    string moved per sort spread over that profile's launches per sort."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    calls, total_us, sorts, sha = 0, 0.0, None, None
    for line in open(path):
        parts = [x for x in line.strip().split("  ") if x]
        if line.startswith(DOMINANT_SYMBOL + "<") and len(parts) >= 3:
            calls += int(parts[1])
            total_us += float(parts[2])
        if line.startswith(sorts_key + " "):
            sorts = int(line.split()[1])
        if line.startswith("kernel_source_sha256 "):
            sha = line.split()[1]
    if not calls or not sorts:
        return None
    fresh = sha == kernel_source_sha256()
    per_sort = calls / sorts
    alg = 24.0 * moved / per_sort
    avg_us = total_us / calls
    achieved = alg / (avg_us / 1e6) / 1e9
    return {"kernel": DOMINANT_SYMBOL, "bound": "hbm", "achieved": achieved,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
            "traffic": None, "avg_launch_us": avg_us, "launches_per_sort": per_sort,
            "alg_bytes_per_launch": alg, "source": f"profiles/{profile} (rocprofv3)",
            "profile_matches_kernel_source": fresh}


def cpu_baseline_sets(chars, offs, sb, min_seconds=8.0):
    """The oracle, untuned, on every usable host core: whole sets of the batched
    workload handed to worker threads (the oracle's C code runs without the
    interpreter lock), sets taken in a seeded order until the wall clock passes
    ``min_seconds``."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    order = np.random.default_rng(5).permutation(sb.size - 1)
    done_sets, done_strings = 0, 0
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        for lo in range(0, order.size, 4 * cores):
            chunk = order[lo:lo + 4 * cores]
            futs = [ex.submit(oracle.sort, chars, offs[int(sb[s]):int(sb[s + 1])]) for s in chunk]
            for f in futs:
                f.result()
            done_sets += chunk.size
            done_strings += int((sb[chunk + 1] - sb[chunk]).sum())
            if time.perf_counter() - t0 >= min_seconds:
                break
    wall = time.perf_counter() - t0
    info = host_info()
    return {"value": done_strings / wall, "unit": "strings/s", "cores": cores, "kind": "oracle",
            "sample": f"{done_sets} of {sb.size - 1} sets ({done_strings:,} strings) of the same "
                      f"seeded batched workload, each sorted by the oracle (multikey quicksort + "
                      f"LCP pass) on one of {cores} worker threads, {wall:.1f} s wall",
            "cpu_model": info["cpu_model"], "nproc": info["nproc"]}


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
    info = host_info()
    return {"value": n_sample * reps / total, "unit": "strings/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample:,} strings of the same seeded {name} recipe, sorted "
                      f"{reps} times by the oracle (multikey quicksort + LCP pass), "
                      f"{total:.1f} s total on 1 host core",
            "cpu_model": info["cpu_model"], "nproc": info["nproc"]}


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


def learned_extra(name, copy_gbps=None, steps=3):
    """Learned vs sampled splitters on one workload (same output, checked), each
    with the metric's HBM figures."""
    import torch
    from paper_1305_1157_amd import gen, s5
    chars, offs = gen.workload(name)
    n = int(offs.size)
    dc, do = torch.from_numpy(chars).cuda(), torch.from_numpy(offs).cuda()
    perm = torch.empty(n, dtype=torch.uint32, device="cuda")
    lcp = torch.empty_like(perm)
    res, ref, D = {"workload": WORKLOAD_TEXT[name], "name": name, "n": n}, None, None
    variants = [("sampled", s5.make_config()),
                ("sampled_equal", s5.make_config(classifier=s5.CLASSIFY_EQUAL)),
                ("sampled_jump", s5.make_config(classifier=s5.CLASSIFY_JUMP)),
                ("sampled_packed", s5.make_config(alphabet=s5.ALPHABET_AUTO)),
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
            D = dist_prefix(dc, do, perm, lcp)
        same = bool(torch.equal(ref[0], perm) and torch.equal(ref[1], lcp))
        res[label] = {"value": n / sec, "ms": sec * 1e3, "passes": st["passes"],
                      "moved_M": st["moved_M"], "fallbacks": st["fallbacks"],
                      "entropy_bits_first_pass": st["entropy_bits"],
                      "max_bucket_first_pass": st["max_bucket"],
                      "learn_ms": prof.get("learn_splitters", {}).get("total_ms", 0.0),
                      "learned_proposals": st["learned_proposals"],
                      "sample_imbalance_mean": st["imbalance_mean"],
                      "sample_imbalance_max": st["imbalance_max"],
                      "classify_ms": prof.get("classify", {}).get("total_ms", 0.0),
                      "base_ms": prof.get("base_sort", {}).get("total_ms", 0.0),
                      "char_bits": st["char_bits"],
                      "hbm": hbm_figures(D, n, st["moved_M"], sec, copy_gbps),
                      "output_identical_to_sampled": same}
        del ws
    return res


def plain_extra(name, copy_gbps=None, steps=10):
    """Plain S^5 with sampled splitters on another workload: strings/s and the
    metric's HBM figures."""
    import torch
    from paper_1305_1157_amd import gen, s5
    chars, offs = gen.workload(name)
    n = int(offs.size)
    dc, do = torch.from_numpy(chars).cuda(), torch.from_numpy(offs).cuda()
    perm = torch.empty(n, dtype=torch.uint32, device="cuda")
    lcp = torch.empty_like(perm)
    ws = torch.empty(s5.workspace_bytes(n), dtype=torch.uint8, device="cuda")
    run = lambda: s5.sort(dc, do, out_perm=perm, out_lcp=lcp, workspace=ws)  # noqa
    for _ in range(3):
        run()
    sec = _timed_sorts(run, steps)
    st = s5.stats()
    D = dist_prefix(dc, do, perm, lcp)
    return {"workload": WORKLOAD_TEXT[name], "name": name, "n": n, "value": n / sec,
            "ms": sec * 1e3, "steps": steps, "passes": st["passes"],
            "hbm": hbm_figures(D, n, st["moved_M"], sec, copy_gbps)}


BATCHED_PROFILES = {"sampled_tuned": "kernels_sets_4096.txt",
                    "learned_tuned": "kernels_sets_4096_learned.txt"}


def batched_extra(steps=3, learned=None, copy_gbps=None, cpu_sample=True):
    """The batched form on 4,096 sets in one graph launch (learned: only that
    variant, else all three), with the metric's HBM figures, the redistribution
    kernel's roofline from the committed rocprofv3 summary of the same workload,
    and the oracle on every host core over a sample of the sets."""
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
           "unroll": table["unroll"], "classifier": table.get("classifier", "unroll"),
           "launches": "one hipGraph per sort (host reads back "
           "set_begin ends and the final counters)"}
    variants = [("learned_tuned", autotune.launch_config(table, splitter_mode=s5.SPLIT_LEARNED),
                 tuned),
                ("sampled_tuned", autotune.launch_config(table), tuned),
                ("sampled_defaults", s5.make_config(), None)]
    if learned is not None:
        variants = [v for v in variants if v[0] == ("learned_tuned" if learned else "sampled_tuned")]
    D = None
    for label, cfg, tun in variants:
        log(f"batched: {label}")
        run = lambda: s5.sort_batched(dc, do, ds, cfg=cfg, tuning=tun, out_perm=perm,  # noqa
                                      out_lcp=lcp)
        run()  # capture
        sec = _timed_sorts(run, steps)
        st = s5.stats()
        if D is None:
            D = dist_prefix(dc, do, perm, lcp, ds)
        res[label] = {"value": n / sec, "ms": sec * 1e3, "passes": st["passes"],
                      "moved_M": st["moved_M"], "fallbacks": st["fallbacks"],
                      "segments": st["segments"], "base_items": st["base_items"],
                      "hbm": hbm_figures(D, n, st["moved_M"], sec, copy_gbps)}
        if label in BATCHED_PROFILES:
            res[label]["roofline"] = profile_roofline(BATCHED_PROFILES[label], st["moved_M"])
    res["check"] = ("tests/test_gpu_fullsize.py checks this workload at full size "
                    "(permutation per set and every neighbour pair, whole small sets)")
    if cpu_sample:
        log("batched: cpu baseline (oracle, all cores)")
        res["cpu_baseline"] = cpu_baseline_sets(chars, offs, sb)
    return res


def batched_main(args):
    """The batched workload as the main line: whole-job strings/s of one graph
    launch per sort (autotuned per-set parameters)."""
    import torch
    copy = copy_bandwidth(torch.device("cuda:0"))
    res = batched_extra(steps=args.steps, learned=args.learned, copy_gbps=copy["GBps"],
                        cpu_sample=bool(args.cpu_sample))
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
        "hbm": r["hbm"],
        "roofline": r.get("roofline"),
        "roofline_note": "kernels inside one graph launch are not bracketed by events; the "
                         "redistribution kernel's average duration comes from the committed "
                         "rocprofv3 summary of this workload",
        "copy_bandwidth": copy,
        "host": host_info(),
        "batched": res,
    }
    if "cpu_baseline" in res:
        out["cpu_baseline"] = res["cpu_baseline"]
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
    copy = None if args.copy_probe_mib else copy_bandwidth(dev)
    copy_gbps = copy["GBps"] if copy else None

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
    D = dist_prefix(d_chars, d_offs, perm, lcp)
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
        "hbm": dict(hbm_figures(D, n, st["moved_M"], sec, copy_gbps), passes=st["passes"]),
        "roofline": {"kernel": DOMINANT_SYMBOL, "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "traffic_source": traffic_src,
                     "avg_launch_us": avg_ms * 1e3,
                     "launches_per_step": dom["launches"] / args.steps,
                     "alg_bytes_per_launch": dom["alg_bytes"] / dom["launches"]},
        "kernels": kernels,
        "stats": st,
        "copy_bandwidth": copy,
        "host": host_info(),
    }
    log(f"{args.workload}: {value / 1e9:.3f} G strings/s, {ms_per_step:.3f} ms per sort")
    if not args.no_extras:
        # the other classification variants (Section 3.1; appendix A jump
        # tables) on the same workload
        names = {s5.CLASSIFY_UNROLL: "unroll", s5.CLASSIFY_EQUAL: "equal",
                 s5.CLASSIFY_JUMP: "jump"}
        out["classifier_variants"] = {
            names[cfg.classifier]: {"ms": ms_per_step, "value": value,
                                   "classify_ms": kernels.get("classify", {}).get("ms_per_step")}}
        for other in names:
            if other == cfg.classifier:
                continue
            c2 = s5.make_config(splitter_mode=cfg.splitter_mode, classifier=other)
            ws2 = torch.empty(s5.workspace_bytes(n, c2), dtype=torch.uint8, device=dev)
            run2 = lambda: s5.sort(d_chars, d_offs, cfg=c2, out_perm=perm, out_lcp=lcp,  # noqa
                                   workspace=ws2)
            run2()
            sec2 = _timed_sorts(run2, args.steps)
            s5.profile_enable(True)
            run2()
            torch.cuda.synchronize()
            cl2 = s5.profile_read().get("classify", {}).get("total_ms", 0.0)
            s5.profile_enable(False)
            out["classifier_variants"][names[other]] = {"ms": sec2 * 1e3, "value": n / sec2,
                                                        "classify_ms": cl2}
            del ws2
        # the two-pass distribution (appendix A, multipass data distribution)
        out["distribution_variants"] = {
            "one_pass": {"ms": ms_per_step, "value": value,
                         "scatter_ms": kernels.get("scatter", {}).get("ms_per_step")}}
        c2 = s5.make_config(splitter_mode=cfg.splitter_mode,
                            distribution=s5.DISTRIBUTE_TWO_PASS)
        ws2 = torch.empty(s5.workspace_bytes(n, c2), dtype=torch.uint8, device=dev)
        run2 = lambda: s5.sort(d_chars, d_offs, cfg=c2, out_perm=perm, out_lcp=lcp,  # noqa
                               workspace=ws2)
        run2()
        sec2 = _timed_sorts(run2, args.steps)
        s5.profile_enable(True)
        run2()
        torch.cuda.synchronize()
        pr2 = s5.profile_read()
        s5.profile_enable(False)
        out["distribution_variants"]["two_pass"] = {
            "ms": sec2 * 1e3, "value": n / sec2,
            "scatter_ms": pr2.get("scatter", {}).get("total_ms"),
            "scatter_launches": pr2.get("scatter", {}).get("launches"),
            "digit_counts_ms": pr2.get("digit_counts", {}).get("total_ms")}
        del ws2
    if args.cpu_sample:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.workload, min(args.cpu_sample, n))
    if not args.no_extras:
        del d_chars, d_offs, perm, lcp, ws
        torch.cuda.empty_cache()
        try:
            out["plain"] = {"random_1M": plain_extra("random_1M", copy_gbps)}
        except Exception as e:  # reported, never hides the main line
            out["plain"] = {"error": repr(e)}
        torch.cuda.empty_cache()
        extras = {}
        for name in ("dna_16M", "words_50M"):
            try:
                extras[name] = learned_extra(name, copy_gbps)
            except Exception as e:
                extras[name] = {"error": repr(e)}
            torch.cuda.empty_cache()
        out["learned"] = extras
        try:
            out["batched"] = batched_extra(copy_gbps=copy_gbps, cpu_sample=bool(args.cpu_sample))
        except Exception as e:
            out["batched"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
