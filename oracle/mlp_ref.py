"""Reference (fp64, NumPy) for the learned splitter proposal -- test infrastructure only.

Only ``tests/`` may use this module; the HIP library shares no code with it.

The paper suggests adapting S^5 to the input by inspecting the sample and
measures what a set of splitters gains by the entropy of the bucket sizes
(appendix A, "Adaptivity").  The learned proposal here models the sample's
distribution function with a small network and places splitters at its
quantiles; classification stays the exact key comparison of Section 3.1, so the
sort's output never depends on the model.

Model (fixed by the build, see the design notes): 8 input features, one per
key byte (most significant first), each scaled by the range that byte takes
over the training sample: x_b = (c_b - lo_b) / max(hi_b - lo_b, 1) with lo_b
and hi_b the smallest and largest value of byte b among the sampled keys (so a
byte every sampled key shares is a constant 0, and lo = 0, hi = 255 gives the
plain c_b / 255); two hidden layers of 32 ReLU units; one sigmoid output, the
estimated CDF.  1377 parameters in this order: W1 (32x8, row major), b1 (32),
W2 (32x32), b2 (32), w3 (32), b3 (1).

Initialisation draws uniform numbers from splitmix64 (Steele, Lea and Flood,
2014) used as a counter-based generator: u_i = top 24 bits of
splitmix64(seed + i + 1) / 2^24, parameter i gets (2 u_i - 1) * a_i with
a = sqrt(6 / fan_in) for W1, W2 and 0.1 * sqrt(6 / 32) for w3; biases start at 0.

Training: full-batch mean squared error against the empirical CDF of the sorted
sample, t_i = (i + 0.5) / m, optimised with Adam (Kingma and Ba, 2015).

Proposal (all comparisons in float32, the precision the kernels decide in):
F_i = running maximum of the model's float32 outputs over the sorted sample (a
monotone CDF).  Heavy hitters first: every run of at least two equal sample keys
is a candidate; with c(L) the number of runs of length >= L and cap = v // 2,
the keys of the runs of length >= L* = min{L >= 2 : c(L) <= cap} become
splitters of their own (equality buckets, Section 3.1).  The other
vq = v - |heavy| splitters are model quantiles: splitter j (1 <= j <= vq) is the
sample key at the first i with F_i >= float32(j) / float32(vq + 1), or the last
sample key if there is none.  The proposal is the sorted union of both lists.
"""
from __future__ import annotations

import numpy as np

N_PARAMS = 1377
H = 32
SLICES = {  # name -> (offset, shape)
    "W1": (0, (H, 8)),
    "b1": (256, (H,)),
    "W2": (288, (H, H)),
    "b2": (1312, (H,)),
    "w3": (1344, (H,)),
    "b3": (1376, (1,)),
}
MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One output of splitmix64 for state x (the state advance is included)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def init_params(seed: int) -> np.ndarray:
    p = np.zeros(N_PARAMS, dtype=np.float64)
    bounds = np.zeros(N_PARAMS)
    bounds[0:256] = np.sqrt(6.0 / 8)
    bounds[288:1312] = np.sqrt(6.0 / H)
    bounds[1344:1376] = 0.1 * np.sqrt(6.0 / H)
    for i in range(N_PARAMS):
        if bounds[i] == 0:
            continue
        u = (splitmix64((seed + i + 1) & MASK64) >> 40) / float(1 << 24)
        p[i] = (2.0 * u - 1.0) * bounds[i]
    return p


def unpack(p: np.ndarray):
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in SLICES.items()}


def key_bytes(keys: np.ndarray) -> np.ndarray:
    """(n, 8) bytes of big-endian 64-bit keys, most significant first."""
    keys = np.asarray(keys, dtype=np.uint64)
    shifts = np.arange(56, -8, -8, dtype=np.uint64)
    return ((keys[:, None] >> shifts[None, :]) & np.uint64(0xFF)).astype(np.int64)


def pack_bytes(b) -> int:
    return int(sum(int(v) << (56 - 8 * i) for i, v in enumerate(b)))


def feature_range(sample_keys: np.ndarray):
    """(lo, hi): byte-wise minimum and maximum over the sample, each packed
    into a 64-bit word like the keys."""
    b = key_bytes(sample_keys)
    return pack_bytes(b.min(axis=0)), pack_bytes(b.max(axis=0))


def features(keys: np.ndarray, lo: int = 0, hi: int = MASK64) -> np.ndarray:
    """(n, 8) features: byte b of every key minus byte b of lo, divided by
    max(byte b of hi - byte b of lo, 1)."""
    c = key_bytes(keys).astype(np.float64)
    lb = key_bytes(np.array([lo], dtype=np.uint64))[0].astype(np.float64)
    hb = key_bytes(np.array([hi], dtype=np.uint64))[0].astype(np.float64)
    return (c - lb) / np.maximum(hb - lb, 1.0)


def forward(p: np.ndarray, x: np.ndarray):
    q = unpack(p)
    z1 = x @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ q["w3"] + q["b3"][0]
    y = 1.0 / (1.0 + np.exp(-z3))
    return y, (x, z1, h1, z2, h2, y)


def loss(p: np.ndarray, x: np.ndarray, t: np.ndarray) -> float:
    y, _ = forward(p, x)
    return float(np.mean((y - t) ** 2))


def grad(p: np.ndarray, x: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Gradient of the mean squared error by backpropagation."""
    q = unpack(p)
    y, (x, z1, h1, z2, h2, _) = forward(p, x)
    m = x.shape[0]
    d3 = (2.0 / m) * (y - t) * y * (1.0 - y)          # dL/dz3, (m,)
    g = np.zeros_like(p)
    gq = unpack(g)
    gq["w3"][:] = d3 @ h2
    gq["b3"][0] = d3.sum()
    d2 = np.outer(d3, q["w3"]) * (z2 > 0)              # dL/dz2, (m, 32)
    gq["W2"][:] = d2.T @ h1
    gq["b2"][:] = d2.sum(axis=0)
    d1 = (d2 @ q["W2"]) * (z1 > 0)                     # dL/dz1, (m, 32)
    gq["W1"][:] = d1.T @ x
    gq["b1"][:] = d1.sum(axis=0)
    return g


def adam_step(p, g, m1, m2, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mh = m1 / (1 - b1 ** step)
    vh = m2 / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def cdf_targets(m: int) -> np.ndarray:
    return (np.arange(m, dtype=np.float64) + 0.5) / m


def train(sorted_keys: np.ndarray, steps: int, lr: float, seed: int):
    """Full-batch Adam on the empirical CDF of a sorted sample; returns
    (params, losses) with losses[s] the loss before step s+1 and a final one."""
    x = features(sorted_keys, *feature_range(sorted_keys))
    t = cdf_targets(len(sorted_keys))
    p = init_params(seed)
    m1 = np.zeros_like(p)
    m2 = np.zeros_like(p)
    losses = []
    for s in range(1, steps + 1):
        losses.append(loss(p, x, t))
        p, m1, m2 = adam_step(p, grad(p, x, t), m1, m2, s, lr)
    losses.append(loss(p, x, t))
    return p, np.array(losses)


def quantile_splitters(cdf: np.ndarray, sorted_keys: np.ndarray, v: int) -> np.ndarray:
    """v splitters from float32 CDF values over the sorted sample: running
    maximum, then for each j the sample key at the first index whose value
    reaches float32(j) / float32(v + 1) (compared in float32)."""
    f = np.maximum.accumulate(np.asarray(cdf, dtype=np.float32))
    q = np.arange(1, v + 1, dtype=np.float32) / np.float32(v + 1)
    idx = np.searchsorted(f, q, side="left")
    idx = np.minimum(idx, len(sorted_keys) - 1)
    return np.asarray(sorted_keys, dtype=np.uint64)[idx]


def heavy_keys(sorted_keys: np.ndarray, v: int) -> np.ndarray:
    """Keys of the runs of >= L* equal sample keys, ascending, where L* is the
    smallest L >= 2 for which at most v // 2 runs are that long (so the heavy
    hitters take at most half of the v splitters)."""
    k = np.asarray(sorted_keys, dtype=np.uint64)
    if k.size == 0:
        return k
    starts = np.flatnonzero(np.concatenate([[True], k[1:] != k[:-1]]))
    lengths = np.diff(np.concatenate([starts, [k.size]]))
    cap = v // 2
    L = 2
    while np.count_nonzero(lengths >= L) > cap:
        L += 1
    return k[starts[lengths >= L]]


def propose_from_cdf(cdf: np.ndarray, sorted_keys: np.ndarray, v: int) -> np.ndarray:
    """v splitters (sorted, may repeat): the heavy hitters of the sample, then
    model quantiles for the remaining slots (float32 CDF values given)."""
    heavy = heavy_keys(sorted_keys, v)
    quant = quantile_splitters(cdf, sorted_keys, v - heavy.size)
    return np.sort(np.concatenate([heavy, quant]))


def propose(p: np.ndarray, sorted_keys: np.ndarray, v: int) -> np.ndarray:
    """The proposal of model p for its own training sample (float32 model
    outputs of the fp64 forward pass)."""
    y, _ = forward(p, features(sorted_keys, *feature_range(sorted_keys)))
    return propose_from_cdf(y.astype(np.float32), sorted_keys, v)


def sample_imbalance(splitters: np.ndarray, sorted_keys: np.ndarray) -> int:
    """Largest number of sample keys strictly between two consecutive splitters
    (or below the first, or above the last): the range buckets the proposal
    would make, counted on the sample itself."""
    s = np.asarray(splitters, dtype=np.uint64)
    k = np.asarray(sorted_keys, dtype=np.uint64)
    lower = np.searchsorted(k, s, side="left")   # keys < s_j
    upper = np.searchsorted(k, s, side="right")  # keys <= s_j
    gaps = np.concatenate([[lower[0]], lower[1:] - upper[:-1], [len(k) - upper[-1]]])
    return int(np.max(np.maximum(gaps, 0)))


def sample_imbalanced(splitters: np.ndarray, sorted_keys: np.ndarray, v: int, beta: float) -> bool:
    """The proposal is rejected before classification if a range bucket of the
    sample alone holds more than beta times the ideal share m / (v + 1)
    (beta as a float32, the product in double)."""
    b = float(np.float32(beta))
    return sample_imbalance(splitters, sorted_keys) > b * len(sorted_keys) / (v + 1)


def imbalanced(bucket_sizes: np.ndarray, v: int, size: int, beta: float) -> bool:
    """True if some range bucket (even index) holds more than beta times the
    ideal share |S| / (v + 1): the learned splitters are then replaced by
    sampled ones."""
    return bool(np.max(np.asarray(bucket_sizes)[0::2]) > beta * size / (v + 1))


def entropy_bits(bucket_sizes: np.ndarray) -> float:
    """sum_i (|b_i| / n) log2(n / |b_i|) over non-empty buckets (appendix A)."""
    b = np.asarray(bucket_sizes, dtype=np.float64)
    b = b[b > 0]
    n = b.sum()
    return float(np.sum(b / n * np.log2(n / b)))
