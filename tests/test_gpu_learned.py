"""Learned splitter proposal on the GPU: model parity with the fp64 reference and
bit-exact sorting in learned mode (the model never changes the output)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import assert_parity, to_dev  # noqa: E402
from oracle import mlp_ref  # noqa: E402
from paper_1305_1157_amd import gen, s5  # noqa: E402

LEARNED = s5.make_config(splitter_mode=s5.SPLIT_LEARNED)


def sample_keys(name, m, seed=0):
    chars, offs = gen.workload(name, 20000)
    rng = np.random.default_rng(seed)
    keys = s5.prefix_keys(to_dev(chars), to_dev(offs), 0).cpu().numpy()
    return np.sort(keys[rng.integers(0, keys.size, size=m)])


def test_forward_matches_reference():
    rng = np.random.default_rng(1)
    p = mlp_ref.init_params(5) + rng.normal(0, 0.2, size=1377)
    keys = np.concatenate([rng.integers(0, 2**64 - 1, size=3000, dtype=np.uint64, endpoint=True),
                           np.array([0, 2**64 - 1], dtype=np.uint64)])
    ranges = [(0, 2**64 - 1), mlp_ref.feature_range(keys[:100]),
              (0x6100000000000000, 0x7A7A7A7A00000000)]
    for lo, hi in ranges:
        got = s5.mlp_eval(to_dev(p.astype(np.float32)), to_dev(keys), lo, hi).cpu().numpy()
        want, _ = mlp_ref.forward(p.astype(np.float32).astype(np.float64),
                                  mlp_ref.features(keys, lo, hi))
        # keys outside the range give features far outside [0, 1]: relative bound
        assert np.all(np.abs(got - want) < 2e-5 * np.maximum(1.0, np.abs(want)) + 2e-5)


@pytest.mark.parametrize("name", ["dna_16M", "words_50M", "url_10M"])
def test_gradient_matches_reference(name):
    keys = sample_keys(name, 512)
    p = mlp_ref.init_params(9).astype(np.float32)
    got = s5.mlp_grad(to_dev(p), to_dev(keys)).cpu().numpy().astype(np.float64)
    x = mlp_ref.features(keys, *mlp_ref.feature_range(keys))
    want = mlp_ref.grad(p.astype(np.float64), x, mlp_ref.cdf_targets(512))
    scale = np.max(np.abs(want))
    assert np.all(np.abs(got - want) <= 1e-4 * scale + 1e-3 * np.abs(want))


def test_first_adam_step_matches_reference():
    keys = sample_keys("words_50M", 1024, seed=2)
    got = s5.mlp_train(to_dev(keys), 1, 0.01, 11).cpu().numpy().astype(np.float64)
    x, t = mlp_ref.features(keys, *mlp_ref.feature_range(keys)), mlp_ref.cdf_targets(1024)
    p0 = mlp_ref.init_params(11)
    g = mlp_ref.grad(p0, x, t)
    want, _, _ = mlp_ref.adam_step(p0, g, np.zeros(1377), np.zeros(1377), 1, 0.01)
    big = np.abs(g) > 1e-3 * np.max(np.abs(g))
    assert np.all(np.abs(got - want)[big] < 1e-5)
    assert np.all(np.abs(got - p0) <= 0.01 * 1.0001 + 1e-6)


@pytest.mark.parametrize("name", ["dna_16M", "words_50M"])
def test_training_tracks_reference(name):
    keys = sample_keys(name, 4096, seed=3)
    steps, lr, seed = 64, 0.03, 5
    got = s5.mlp_train(to_dev(keys), steps, lr, seed).cpu().numpy().astype(np.float64)
    x, t = mlp_ref.features(keys, *mlp_ref.feature_range(keys)), mlp_ref.cdf_targets(4096)
    _, losses = mlp_ref.train(keys, steps, lr, seed)
    got_loss = mlp_ref.loss(got, x, t)
    # the exact trajectory is not pinned (FP32 sums); the loss reached is
    assert got_loss <= 1.25 * losses[-1] + 1e-4
    assert got_loss < 0.5 * losses[0]


def _proposal_vs_reference(params, keys, v, beta):
    """The kernel's proposal against the reference on the kernel's own float32
    model outputs (both sides take the quantile decisions in float32 from the
    same values); the outputs themselves against the fp64 forward pass."""
    spl, y, rej = s5.mlp_propose(params, to_dev(keys), v, beta)
    torch.cuda.synchronize()
    yg = y.cpu().numpy()
    p64 = params.cpu().numpy().astype(np.float64)
    y_ref, _ = mlp_ref.forward(p64, mlp_ref.features(keys, *mlp_ref.feature_range(keys)))
    assert np.all(np.abs(yg - y_ref) <= 3e-5)
    want = mlp_ref.propose_from_cdf(yg, keys, v)
    got = spl.cpu().numpy()
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"v={v}: splitters differ at {bad[:8]}"
    want_rej = mlp_ref.sample_imbalanced(want, keys, v, beta)
    assert int(rej.item()) == int(want_rej)
    return want, mlp_ref.sample_imbalance(want, keys) / (keys.size / (v + 1))


@pytest.mark.parametrize("name", ["dna_16M", "words_50M", "url_10M"])
def test_proposal_matches_reference(name):
    """The learned splitter proposal (monotone CDF, heavy hitters, quantiles,
    merge, sample check) bit-exact against the reference, for a model trained
    by the GPU on the workload's own sample, at the v the sort uses."""
    keys = sample_keys(name, 4096, seed=4)
    params = s5.mlp_train(to_dev(keys), 64, 0.03, 5)
    for v in (127, 255, 1023):
        for beta in (4.0, 1e9):
            spl, ratio = _proposal_vs_reference(params, keys, v, beta)
            print(f"{name} v={v} beta={beta}: heavy {mlp_ref.heavy_keys(keys, v).size}, "
                  f"largest sample range bucket {ratio:.2f} x ideal", flush=True)


def test_proposal_hand_cases():
    """Heavy hitters from planted duplicate runs, a sample of one repeated key,
    the smallest sample (m = 256) and untrained weights."""
    rng = np.random.default_rng(8)
    p0 = to_dev(mlp_ref.init_params(3).astype(np.float32))
    base = rng.integers(0, 2**63, size=4096, dtype=np.uint64)
    runs = np.repeat(rng.integers(0, 2**63, size=40, dtype=np.uint64),
                     rng.integers(2, 60, size=40))  # 40 runs, at most 2360 keys
    planted = np.sort(np.concatenate([base[:4096 - runs.size], runs]))
    cases = [planted, np.full(4096, 0x4142434445464748, dtype=np.uint64),
             np.sort(base[:256]), np.sort(rng.integers(0, 4, size=512).astype(np.uint64))]
    for keys in cases:
        for v in (1, 7, 63, 255, 1023):
            _proposal_vs_reference(p0, keys, v, 4.0)


@pytest.mark.parametrize("name,n", [("dna_16M", 200_000), ("words_50M", 400_000),
                                    ("url_10M", 200_000), ("random_1M", 300_000)])
def test_learned_sort_parity(name, n):
    chars, offs = gen.workload(name, n)
    st = assert_parity(chars, offs, LEARNED, label=f"learned {name}")
    assert st["passes"] >= 1


def test_learned_jump_tables_parity():
    # learned trees build their jump tables in the proposal kernel
    chars, offs = gen.workload("words_50M", 300_000)
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED, imbalance_bound=1e9,
                         classifier=s5.CLASSIFY_JUMP)
    st = assert_parity(chars, offs, cfg, label="learned jump")
    assert st["fallbacks"] == 0


def test_forced_fallback_parity():
    chars, offs = gen.workload("words_50M", 300_000)
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED, imbalance_bound=1e-6)
    st = assert_parity(chars, offs, cfg, label="forced fallback")
    assert st["fallbacks"] >= st["learned_proposals"] >= 1


def test_never_fallback_parity():
    # whatever the model proposes is used; the output is still exact
    chars, offs = gen.workload("dna_16M", 150_000)
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED, imbalance_bound=1e9, base_threshold=64)
    st = assert_parity(chars, offs, cfg, label="never fallback")
    assert st["fallbacks"] == 0


def test_sample_imbalance_statistics():
    """The statistics report each proposal's largest range bucket on its own
    sample (keys equal to a splitter are not in one), relative to m / (v + 1):
    positive, the maximum at least the mean; with no bound nothing is replaced."""
    chars, offs = gen.workload("words_50M", 300_000)
    for bound in (1e9, 4.0):
        cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED, imbalance_bound=bound)
        st = assert_parity(chars, offs, cfg, label=f"imbalance stats, bound {bound}")
        assert st["learned_proposals"] >= 1
        assert 0.0 < st["imbalance_mean"] <= st["imbalance_max"] + 1e-9
        if bound == 1e9:
            assert st["fallbacks"] == 0
    sampled = s5.make_config()
    st = assert_parity(chars, offs, sampled, label="sampled, no proposals")
    assert st["learned_proposals"] == 0 and st["imbalance_max"] == 0.0


def test_learned_two_pass_parity():
    # learned trees (some rejected on the exact histogram and redone) with two moves per level
    chars, offs = gen.workload("words_50M", 300_000)
    cfg = s5.make_config(splitter_mode=s5.SPLIT_LEARNED, distribution=s5.DISTRIBUTE_TWO_PASS)
    assert_parity(chars, offs, cfg, label="learned two-pass")


def test_batched_learned_parity():
    chars, offs, sb = gen.batched(6, 70_000, 150_000, kinds=("random", "url", "dna"), seed=21)
    perm, lcp = s5.sort_batched(to_dev(chars), to_dev(offs), to_dev(sb), cfg=LEARNED)
    torch.cuda.synchronize()
    import oracle
    rp, rl = oracle.sort_batched(chars, offs, sb)
    assert np.array_equal(perm.cpu().numpy(), rp) and np.array_equal(lcp.cpu().numpy(), rl)
