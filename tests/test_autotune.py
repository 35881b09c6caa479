"""Host logic of the autotuner: table defaults, size classes, per-set rows
that the C-ABI accepts (no GPU needed)."""
import json

import numpy as np

from paper_1305_1157_amd import autotune


def _valid_row(v, t, tile):
    return v in (7, 15, 31, 63, 127, 255, 511, 1023) and 64 <= t <= 2048 and tile % 64 == 0 \
        and 64 <= tile <= 1 << 20


def test_defaults_cover_every_size():
    t = autotune.default_table()
    assert t["classes"][0]["lo"] <= 100 and t["classes"][-1]["hi"] > 1_000_000
    for a, b in zip(t["classes"][:-1], t["classes"][1:]):
        assert a["hi"] == b["lo"]
    rows = autotune.tuning_for([1, 100, 999, 1000, 99_999, 100_000, 1_000_000, 5_000_000], t)
    assert len(rows) == 8 and all(_valid_row(*r) for r in rows)


def test_class_boundaries(tmp_path):
    t = autotune.default_table()
    for i, c in enumerate(t["classes"]):
        c["splitters"] = [63, 127, 255, 1023][i]
    rows = autotune.tuning_for([100, 999, 1000, 9999, 10_000, 100_000, 1_000_000], t)
    assert [r[0] for r in rows] == [63, 63, 127, 127, 255, 1023, 1023]
    p = tmp_path / "t.json"
    p.write_text(json.dumps(t))
    assert autotune.load_table(str(p)) == t
    assert autotune.load_table(str(tmp_path / "missing.json"))["source"] == "defaults"


def test_committed_table_is_valid():
    t = autotune.load_table()
    assert t["unroll"] in (1, 2, 4, 8)
    for c in t["classes"]:
        assert _valid_row(c["splitters"], c["base_threshold"], c["tile"])
    sizes = np.random.default_rng(0).integers(100, 1_000_000, size=1000)
    assert all(_valid_row(*r) for r in autotune.tuning_for(sizes, t))


def test_unroll_needs_a_clear_win():
    # a faster U replaces the default only when it wins by 2 %
    assert autotune.pick_unroll({2: 1.0, 4: 1.01, 8: 1.02}) == 4
    assert autotune.pick_unroll({2: 0.9, 4: 1.0, 8: 1.0}) == 2
    assert autotune.pick_unroll({2: 1.1, 4: 1.0, 8: 0.985}) == 4


def test_mix_check_keeps_only_a_clear_win():
    def table():
        t = autotune.default_table()
        t["classes"][1].update(splitters=63, base_threshold=512)
        return t
    won = autotune.apply_mix_check(table(), 0.95, 1.0)
    assert won["mix_check"]["kept"] and won["classes"][1]["splitters"] == 63
    lost = autotune.apply_mix_check(table(), 0.99, 1.0)
    assert not lost["mix_check"]["kept"]
    assert [(c["splitters"], c["base_threshold"], c["tile"]) for c in lost["classes"]] == \
        [(c["splitters"], c["base_threshold"], c["tile"]) for c in autotune.default_table()["classes"]]
    assert lost["mix_check"] == {"table_ms": 0.99, "defaults_ms": 1.0, "kept": False}


def test_committed_table_passed_its_mix_check():
    t = autotune.load_table()
    mc = t["mix_check"]
    defaults = autotune.default_table()["classes"]
    if not mc["kept"]:
        assert [(c["splitters"], c["base_threshold"], c["tile"]) for c in t["classes"]] == \
            [(c["splitters"], c["base_threshold"], c["tile"]) for c in defaults]
    else:
        assert mc["table_ms"] < 0.98 * mc["defaults_ms"]


def test_launch_choices_need_a_clear_win():
    assert autotune.pick_unroll({2: 1.0, 4: 1.01, 8: 1.1}) == 4
    assert autotune.pick_unroll({2: 0.9, 4: 1.0, 8: 1.1}) == 2
    assert autotune.pick_classifier({"unroll": 1.0, "equal": 0.99}) == "unroll"
    assert autotune.pick_classifier({"unroll": 1.0, "equal": 0.97}) == "equal"
    t = autotune.default_table()
    assert t["classifier"] in autotune.CLASSIFIERS
    assert autotune.load_table().get("classifier", "unroll") in autotune.CLASSIFIERS
