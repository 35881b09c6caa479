"""Autotuner for batched S^5.

The paper fixes its thresholds by hand for its machines (Section 3.1,
"Implementation Details": splitter tree size, base-case thresholds).  Here the
same parameters are measured on the device instead: for every class of set
sizes the tuner times the HIP sort on a synthetic probe batch of that class
and keeps the fastest splitter count v, base-case threshold T and tile, by
coordinate descent from the defaults; the table is kept only if it also wins
on a batch that mixes all classes, and the interleaved descents per lane U
and the classification variant (Unroll or Equal, Section 3.1, or Unroll with
a jump table, appendix A; one value of each per launch) are tuned last on that
batch.  The
result is a JSON table; ``tuning_for`` maps set sizes to per-set parameters
for ``s5.sort_batched(..., tuning=...)``.

Run on a GPU:  ``python -m paper_1305_1157_amd.autotune --out table.json``.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "tune_table.json")

# [lo, hi) strings per set
SIZE_CLASSES = [(100, 1_000), (1_000, 10_000), (10_000, 100_000), (100_000, 1_000_001)]
CANDIDATES = {
    "splitters": [63, 255, 1023],
    "base_threshold": [256, 512, 1024, 2048],
    "tile": [1024, 2048, 4096],
}
UNROLLS = [2, 4, 8]
CLASSIFIERS = {"unroll": 0, "equal": 1, "jump": 2}  # s5.CLASSIFY_UNROLL / _EQUAL / _JUMP
DEFAULT = {"splitters": 255, "base_threshold": 1024, "tile": 2048}
DEFAULT_UNROLL = 4
DEFAULT_CLASSIFIER = "unroll"


def default_table() -> dict:
    return {"classes": [dict(lo=lo, hi=hi, **DEFAULT) for lo, hi in SIZE_CLASSES],
            "unroll": DEFAULT_UNROLL, "classifier": DEFAULT_CLASSIFIER, "source": "defaults"}


def launch_config(table: dict, **kw):
    """The launch-wide s5 config of a table: its U and classification variant."""
    from . import s5
    return s5.make_config(unroll=table.get("unroll", DEFAULT_UNROLL),
                          classifier=CLASSIFIERS[table.get("classifier", DEFAULT_CLASSIFIER)], **kw)


def load_table(path: str = TABLE_PATH) -> dict:
    """The tuned table, or the defaults if none has been written."""
    if not os.path.exists(path):
        return default_table()
    with open(path) as f:
        return json.load(f)


def class_of(size: int, table: dict) -> dict:
    for c in table["classes"]:
        if c["lo"] <= size < c["hi"]:
            return c
    return table["classes"][0] if size < table["classes"][0]["lo"] else table["classes"][-1]


def tuning_for(set_sizes, table: dict):
    """Per-set rows (splitters, base_threshold, tile) from the table."""
    rows = []
    for sz in np.asarray(set_sizes, dtype=np.int64):
        c = class_of(int(sz), table)
        rows.append((c["splitters"], c["base_threshold"], c["tile"]))
    return rows


def pick_clearly_faster(ms: dict, default):
    """The fastest choice from {choice: ms}, but the default unless another is
    clearly (2 %) faster, as for the other parameters."""
    best = min(ms, key=ms.get)
    return best if ms[best] < ms[default] * 0.98 else default


def pick_unroll(ms: dict) -> int:
    return pick_clearly_faster(ms, DEFAULT_UNROLL)


def pick_classifier(ms: dict) -> str:
    return pick_clearly_faster(ms, DEFAULT_CLASSIFIER)


def apply_mix_check(table: dict, table_ms: float, defaults_ms: float) -> dict:
    """Keep the per-class choices only if the whole table is clearly (2 %)
    faster than the defaults on the mixed batch; otherwise every class goes
    back to the defaults.  Records both times in ``table["mix_check"]``."""
    kept = table_ms < defaults_ms * 0.98
    table["mix_check"] = {"table_ms": table_ms, "defaults_ms": defaults_ms, "kept": kept}
    if not kept:
        for c in table["classes"]:
            c.update(DEFAULT)
    return table


# ---------------------------------------------------------------------------
# measurement (needs the GPU)

def _probe(lo, hi, kinds, target, seed):
    from . import gen
    mean = (hi - lo) / max(np.log(hi / lo), 1e-9)  # mean of log-uniform sizes
    nsets = int(max(2, min(4096, round(target / mean))))
    return gen.batched(nsets, lo, hi - 1, kinds=kinds, seed=seed)


class _Batch:
    def __init__(self, chars, offs, sb):
        import torch
        self.sizes = np.diff(sb).astype(np.int64)
        self.n = int(offs.size)
        self.chars = torch.from_numpy(chars).cuda()
        self.offs = torch.from_numpy(offs).cuda()
        self.sb = torch.from_numpy(sb).cuda()
        self.perm = torch.empty(self.n, dtype=torch.uint32, device="cuda")
        self.lcp = torch.empty(self.n, dtype=torch.uint32, device="cuda")

    reps = 3  # timed sorts per measurement (the median is kept)

    def time(self, rows, unroll, reps=None, classifier=DEFAULT_CLASSIFIER):
        """Median wall time (ms) of the batched sort with per-set rows."""
        import torch

        from . import s5
        cfg = s5.make_config(unroll=unroll, classifier=CLASSIFIERS[classifier])
        tun = s5.make_tuning(rows)
        s5.sort_batched(self.chars, self.offs, self.sb, cfg=cfg, tuning=tun, out_perm=self.perm,
                        out_lcp=self.lcp)  # capture / warm-up
        ts = []
        for _ in range(reps or self.reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            s5.sort_batched(self.chars, self.offs, self.sb, cfg=cfg, tuning=tun,
                            out_perm=self.perm, out_lcp=self.lcp)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t) * 1e3)
        return float(np.median(ts))


def _descend(batch: _Batch, start: dict, unroll: int, rounds: int, log):
    best = dict(start)
    best_t = batch.time([tuple(best[k] for k in ("splitters", "base_threshold", "tile"))] *
                        len(batch.sizes), unroll)
    trials = [(dict(best), best_t)]
    for _ in range(rounds):
        changed = False
        for key, values in CANDIDATES.items():
            for v in values:
                if v == best[key]:
                    continue
                cand = dict(best, **{key: v})
                row = tuple(cand[k] for k in ("splitters", "base_threshold", "tile"))
                t = batch.time([row] * len(batch.sizes), unroll)
                trials.append((cand, t))
                log(f"    {cand} -> {t:.3f} ms")
                if t < best_t * 0.98:  # keep a change only if it is clearly faster
                    best, best_t, changed = cand, t, True
        if not changed:
            break
    return best, best_t, trials


def tune(kinds=("random", "url", "dna"), target=3_000_000, rounds=2, seed=0x70E, log=print):
    """Measure and return a table (see the module docstring)."""
    import torch

    table = {"classes": [], "kinds": list(kinds), "probe_strings": target,
             "device": torch.cuda.get_device_name(0), "source": "measured"}
    for ci, (lo, hi) in enumerate(SIZE_CLASSES):
        b = _Batch(*_probe(lo, hi, kinds, target, seed + ci))
        log(f"class [{lo}, {hi}): {len(b.sizes)} sets, {b.n} strings")
        best, t, trials = _descend(b, DEFAULT, DEFAULT_UNROLL, rounds, log)
        t0 = trials[0][1]
        log(f"  best {best}: {t:.3f} ms (defaults {t0:.3f} ms)")
        table["classes"].append(dict(lo=lo, hi=hi, **best, ms=t, default_ms=t0, sets=len(b.sizes),
                                     strings=b.n))
        del b
    # the table must also win on a batch mixing every class, else the defaults stay
    mix = _Batch(*_probe(SIZE_CLASSES[0][0], SIZE_CLASSES[-1][1], kinds, target, seed + 99))
    rows = tuning_for(mix.sizes, table)
    t_tab = mix.time(rows, DEFAULT_UNROLL)
    t_def = mix.time(tuning_for(mix.sizes, default_table()), DEFAULT_UNROLL)
    log(f"mixed batch: table {t_tab:.3f} ms, defaults {t_def:.3f} ms")
    apply_mix_check(table, t_tab, t_def)
    rows = tuning_for(mix.sizes, table)
    # one unroll for the launch, on the same batch
    ut = {u: mix.time(rows, u) for u in UNROLLS}
    table["unroll"] = pick_unroll(ut)
    table["unroll_ms"] = ut
    log(f"unroll: {ut} -> {table['unroll']}")
    # one classification variant for the launch, on the same batch
    ct = {c: mix.time(rows, table["unroll"], classifier=c) for c in CLASSIFIERS}
    table["classifier"] = pick_classifier(ct)
    table["classifier_ms"] = ct
    log(f"classifier: {ct} -> {table['classifier']}")
    return table


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--target", type=int, default=3_000_000, help="strings per probe batch")
    ap.add_argument("--rounds", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3, help="timed sorts per measurement")
    a = ap.parse_args()
    _Batch.reps = a.reps
    t = tune(target=a.target, rounds=a.rounds, log=lambda s: print(s, flush=True))
    with open(a.out, "w") as f:
        json.dump(t, f, indent=1)
    print(f"wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
