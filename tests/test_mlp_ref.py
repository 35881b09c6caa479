"""Pins of the fp64 reference for the learned splitter proposal (CPU only).

* splitmix64 against the generator's published first outputs;
* backpropagation against central finite differences (a closed form);
* forward / Adam / quantile selection against closed forms;
* entropy of bucket sizes against log2(k) for k equal buckets.
"""
import os

import numpy as np
import pytest

from oracle import mlp_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_outputs():
    vals = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64.txt"))
            if l.strip() and not l.startswith("#")]
    state = 0
    for v in vals:
        assert mlp_ref.splitmix64(state) == v
        state = (state + 0x9E3779B97F4A7C15) & mlp_ref.MASK64


def test_init_params_ranges():
    p = mlp_ref.init_params(7)
    q = mlp_ref.unpack(p)
    assert p.shape == (1377,)
    assert np.all(q["b1"] == 0) and np.all(q["b2"] == 0) and q["b3"][0] == 0
    assert np.abs(q["W1"]).max() <= np.sqrt(6 / 8) and np.abs(q["W2"]).max() <= np.sqrt(6 / 32)
    assert np.abs(q["w3"]).max() <= 0.1 * np.sqrt(6 / 32)
    assert not np.array_equal(p, mlp_ref.init_params(8))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_grad_vs_finite_differences(seed):
    rng = np.random.default_rng(seed)
    keys = np.sort(rng.integers(0, 2**63, size=24, dtype=np.uint64))
    x = mlp_ref.features(keys)
    t = mlp_ref.cdf_targets(len(keys))
    p = mlp_ref.init_params(seed) + rng.normal(0, 0.05, size=1377)
    g = mlp_ref.grad(p, x, t)
    idx = rng.choice(1377, size=60, replace=False)
    idx = np.concatenate([idx, [1376, 1344, 288, 0]])
    h = 1e-6
    for i in idx:
        e = np.zeros(1377)
        e[i] = h
        fd = (mlp_ref.loss(p + e, x, t) - mlp_ref.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(fd), (i, fd, g[i])


def test_forward_closed_forms():
    x = mlp_ref.features(np.array([0, 2**64 - 1, 12345], dtype=np.uint64))
    assert np.allclose(x[1], 1.0) and np.allclose(x[0], 0.0)
    p = np.zeros(1377)
    y, _ = mlp_ref.forward(p, x)
    assert np.allclose(y, 0.5)
    p[1376] = 2.0
    y, _ = mlp_ref.forward(p, x)
    assert np.allclose(y, 1 / (1 + np.exp(-2.0)))


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    p = rng.normal(size=1377)
    g = rng.normal(size=1377)
    p1, _, _ = mlp_ref.adam_step(p, g, np.zeros(1377), np.zeros(1377), 1, 0.01)
    # bias-corrected moments of the first step are g and g^2
    assert np.allclose(p1 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-12)


def test_quantile_splitters_closed_form():
    m, v = 1000, 15
    keys = np.arange(m, dtype=np.uint64) * np.uint64(3)
    spl = mlp_ref.quantile_splitters(mlp_ref.cdf_targets(m), keys, v)
    want = [keys[int(np.ceil(j * m / (v + 1) - 0.5))] for j in range(1, v + 1)]
    assert spl.tolist() == [int(w) for w in want]
    # a non-monotone CDF is made monotone first; a constant CDF maps every
    # splitter to the first key reaching the quantile, or to the last key
    cdf = np.full(m, 0.2)
    spl = mlp_ref.quantile_splitters(cdf, keys, v)
    assert np.all(spl[: 3] == keys[0]) and np.all(spl[3:] == keys[-1])


def test_training_lowers_loss():
    rng = np.random.default_rng(4)
    keys = np.sort(rng.integers(0, 2**63, size=512, dtype=np.uint64))
    p, losses = mlp_ref.train(keys, steps=40, lr=0.02, seed=3)
    assert losses[-1] < 0.25 * losses[0]


def test_entropy_and_imbalance():
    assert mlp_ref.entropy_bits(np.full(64, 10)) == pytest.approx(6.0)
    assert mlp_ref.entropy_bits(np.array([0, 50, 0])) == 0.0
    sizes = np.array([10, 0, 10, 0, 100])
    assert mlp_ref.imbalanced(sizes, v=2, size=120, beta=2.0)
    assert not mlp_ref.imbalanced(sizes, v=2, size=120, beta=3.0)


def test_feature_range_and_features():
    # byte-wise range written out per byte, against hand-computed values
    k = np.array([0x6161610000000000, 0x6162790000000000, 0x6163620000000000], dtype=np.uint64)
    lo, hi = mlp_ref.feature_range(k)
    assert lo == 0x6161610000000000 and hi == 0x6163790000000000
    f = mlp_ref.features(k, lo, hi)
    assert np.allclose(f[:, 0], 0) and np.allclose(f[:, 3:], 0)  # shared bytes -> 0
    assert np.allclose(f[:, 1], [0, 0.5, 1.0])                    # 0x61, 0x62, 0x63 over [0x61, 0x63]
    assert np.allclose(f[:, 2], [0, (0x79 - 0x61) / 0x18, (0x62 - 0x61) / 0x18])
    # default range is the plain byte / 255 encoding
    g = mlp_ref.features(np.array([0x00FF7F0102030405], dtype=np.uint64))
    assert np.allclose(g[0] * 255, [0x00, 0xFF, 0x7F, 1, 2, 3, 4, 5])
    # each feature of the sample lies in [0, 1] and reaches both ends where bytes vary
    rng = np.random.default_rng(3)
    s = rng.integers(0, 2**64 - 1, size=500, dtype=np.uint64, endpoint=True)
    fs = mlp_ref.features(s, *mlp_ref.feature_range(s))
    assert fs.min() == 0.0 and fs.max() == 1.0
    assert np.all(fs.min(axis=0) == 0) and np.all(fs.max(axis=0) == 1)


def test_sample_imbalance_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(20):
        k = np.sort(rng.integers(0, 50, size=200).astype(np.uint64))
        s = np.sort(rng.choice(k, size=7))
        brute = []
        edges = [None] + list(s) + [None]
        for a, b in zip(edges[:-1], edges[1:]):
            brute.append(sum(1 for x in k if (a is None or x > a) and (b is None or x < b)))
        assert mlp_ref.sample_imbalance(s, k) == max(brute)




def test_heavy_keys_by_hand():
    k = np.array([1, 1, 2, 3, 3, 3, 4, 5, 5], dtype=np.uint64)
    # v = 7: at most 3 heavy hitters, and there are exactly 3 runs of >= 2
    assert mlp_ref.heavy_keys(k, 7).tolist() == [1, 3, 5]
    # v = 3: at most 1, so only runs of >= 3 (the single longest run) count
    assert mlp_ref.heavy_keys(k, 3).tolist() == [3]
    assert mlp_ref.heavy_keys(np.arange(10, dtype=np.uint64), 7).size == 0
    assert mlp_ref.heavy_keys(np.full(10, 7, dtype=np.uint64), 7).tolist() == [7]
    # two runs of 4, two of 2, cap 1: no length admits a single run except > 4
    k2 = np.array([1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 4, 4], dtype=np.uint64)
    assert mlp_ref.heavy_keys(k2, 3).size == 0
    assert mlp_ref.heavy_keys(k2, 5).tolist() == [1, 2]


def test_heavy_keys_brute_force():
    """The definition counted out: for every L >= 2 the runs of length >= L, the
    smallest L with at most v // 2 of them, and the keys of those runs."""
    rng = np.random.default_rng(8)
    for _ in range(50):
        m = int(rng.integers(1, 300))
        k = np.sort(rng.integers(0, int(rng.integers(1, 200)), size=m).astype(np.uint64))
        v = int(rng.choice([7, 15, 31, 63]))
        counts = {}
        for x in k.tolist():
            counts[x] = counts.get(x, 0) + 1
        L = 2
        while sum(1 for c in counts.values() if c >= L) > v // 2:
            L += 1
        want = sorted(x for x, c in counts.items() if c >= L)
        got = mlp_ref.heavy_keys(k, v)
        assert got.tolist() == want
        assert got.size <= v // 2


def test_propose_from_cdf_by_hand():
    # distinct keys, ideal CDF: quantiles 1/4, 1/2, 3/4 land on keys 4, 8, 12
    keys = np.arange(16, dtype=np.uint64)
    cdf = ((np.arange(16) + 0.5) / 16).astype(np.float32)
    assert mlp_ref.propose_from_cdf(cdf, keys, 3).tolist() == [4, 8, 12]
    # a run of three 20s is a heavy hitter (cap 1); the two quantiles 1/3 and
    # 2/3 land on positions 3 (a 20) and 5 (key 40); the union keeps both 20s
    keys = np.array([10, 20, 20, 20, 30, 40, 50, 60], dtype=np.uint64)
    cdf = ((np.arange(8) + 0.5) / 8).astype(np.float32)
    assert mlp_ref.propose_from_cdf(cdf, keys, 3).tolist() == [20, 20, 40]
    # the quantile thresholds are float32 divisions: F = 1/3 in float32 reaches
    # the first quantile exactly
    keys = np.arange(3, dtype=np.uint64)
    cdf = np.array([0.0, np.float32(1) / np.float32(3), 1.0], dtype=np.float32)
    assert mlp_ref.quantile_splitters(cdf, keys, 2).tolist() == [1, 2]
