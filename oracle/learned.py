"""FP64 CPU oracle of the learned partitioner (test infrastructure only).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this module; the HIP library never does.

The paper builds its kernel matrix from exact neighbour sets and leaves the
neighbour search itself open; it notes that finding nearest neighbours in high
dimension is a hard problem of its own (Section 4, computational cost). The
learned partitioner is the approximate search used for the largest sample
sets: a balanced partition taught to an MLP by the neighbour-histogram recipe
of Neural LSH (Dong, Indyk, Razenshteyn and Wagner, "Learning Space
Partitions for Nearest Neighbor Search", ICLR 2020). What this module defines,
in plain numpy:

  * ``splitmix64`` -- the SplitMix64 generator (Steele, Lea and Flood, OOPSLA
    2014; constants as published by Vigna), in counter form: output c of seed s
    is the mix of s + (c + 1) * 0x9E3779B97F4A7C15.
  * ``teacher_labels`` -- balanced median splits: in round l each node v is
    projected on its own random direction u(l, v) (components uniform in
    [-1, 1) with 24 random bits), the projection summed in float64 in column
    order and rounded to float32; the node's samples ordered by (projection,
    index) give their lower half (floor) to child 2v and the rest to 2v + 1.
  * ``forward`` / ``backward`` -- the MLP m -> h1 -> h2 -> nb with ReLU and the
    batch-mean soft-target cross-entropy, in float64, with optional rounding
    to bfloat16 (round to nearest even at 8 significant bits) at the points
    where the GPU path stores BF16: the input rows, the weights, the ReLU
    outputs, and the gradients of the logits and hidden layers before they
    enter a product.
  * ``adam_step`` -- Adam (Kingma and Ba, ICLR 2015) with bias correction.
  * ``recall`` -- mean fraction of exact neighbours found.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters) -> np.ndarray:
    """Outputs number c (0-based) of the SplitMix64 sequence started at seed."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (c + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def teacher_direction(seed: int, level: int, node: int, m: int) -> np.ndarray:
    """u(level, node) in [-1, 1)^m, float64 (exact float32 values)."""
    ctr = (np.uint64(level) << np.uint64(40)) | (np.uint64(node) << np.uint64(20)) | np.arange(m, dtype=np.uint64)
    bits = splitmix64(seed, ctr) >> np.uint64(40)
    return bits.astype(np.float64) / 8388608.0 - 1.0


def float32_order(x32: np.ndarray) -> np.ndarray:
    """Unsigned integers ordered like the float32 values (negative zero first)."""
    b = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    neg = (b & np.uint64(0x80000000)) != 0
    return np.where(neg, (~b) & np.uint64(0xFFFFFFFF), b | np.uint64(0x80000000))


def teacher_labels(X: np.ndarray, levels: int, seed: int) -> np.ndarray:
    """Bucket label in [0, 2^levels) of every row of X [ns, m] float32."""
    X64 = np.asarray(X, dtype=np.float32).astype(np.float64)
    ns, m = X64.shape
    node = np.zeros(ns, dtype=np.int64)
    for level in range(levels):
        proj = np.zeros(ns, dtype=np.float64)
        dirs = np.stack([teacher_direction(seed, level, v, m) for v in range(1 << level)])
        U = dirs[node]                     # [ns, m] direction of each sample's node
        for c in range(m):                 # column order, one rounding per product and sum
            proj = proj + X64[:, c] * U[:, c]
        key = float32_order(proj.astype(np.float32))
        order = np.lexsort((np.arange(ns), key, node))
        new = np.empty_like(node)
        sorted_nodes = node[order]
        starts = np.searchsorted(sorted_nodes, np.arange((1 << level) + 1))
        for v in range(1 << level):
            members = order[starts[v]:starts[v + 1]]
            half = len(members) // 2
            new[members[:half]] = 2 * v
            new[members[half:]] = 2 * v + 1
        node = new
    return node.astype(np.int32)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest value with 8 significant bits, ties to even
    (bfloat16 for normal numbers), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    mant, expo = np.frexp(x)              # x = mant 2^expo, 0.5 <= |mant| < 1
    return np.ldexp(np.round(mant * 256.0) / 256.0, expo)


def init_params(m: int, h1: int, h2: int, nb: int, seed: int, bias_scale: float = 0.1) -> list[np.ndarray]:
    """Seeded test parameters (W1, b1, W2, b2, W3, b3), He-scaled, float32 values."""
    rng = np.random.default_rng(seed)
    out = []
    for fan_in, fan_out in ((m, h1), (h1, h2), (h2, nb)):
        out.append((rng.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)).astype(np.float32))
        out.append((rng.standard_normal(fan_out) * bias_scale).astype(np.float32))
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def unflatten(flat: np.ndarray, m: int, h1: int, h2: int, nb: int) -> list[np.ndarray]:
    shapes = [(h1, m), (h1,), (h2, h1), (h2,), (nb, h2), (nb,)]
    out, o = [], 0
    for s in shapes:
        cnt = int(np.prod(s))
        out.append(np.asarray(flat[o:o + cnt], dtype=np.float64).reshape(s))
        o += cnt
    return out


def soft_targets(nbr_labels: np.ndarray, nb: int) -> np.ndarray:
    """t[i, b] = fraction of row i's neighbour labels equal to b."""
    B, ks = nbr_labels.shape
    T = np.zeros((B, nb), dtype=np.float64)
    np.add.at(T, (np.repeat(np.arange(B), ks), nbr_labels.ravel()), 1.0)
    return T / ks


def forward(params, X: np.ndarray, cast: bool = True) -> dict:
    c = bf16_round if cast else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, dtype=np.float64) for p in params)
    Xb = c(X)
    H1 = np.maximum(Xb @ c(W1).T + b1, 0.0)
    H1b = c(H1)
    H2 = np.maximum(H1b @ c(W2).T + b2, 0.0)
    H2b = c(H2)
    Z = H2b @ c(W3).T + b3
    return {"Xb": Xb, "H1": H1, "H1b": H1b, "H2": H2, "H2b": H2b, "Z": Z}


def loss_of_logits(Z: np.ndarray, T: np.ndarray) -> float:
    """Batch mean of logsumexp(z) - sum_b t_b z_b."""
    zmax = Z.max(axis=1, keepdims=True)
    lse = zmax[:, 0] + np.log(np.exp(Z - zmax).sum(axis=1))
    return float(np.mean(lse - (T * Z).sum(axis=1)))


def backward(params, X: np.ndarray, nbr_labels: np.ndarray, cast: bool = True):
    """(loss, [dW1, db1, dW2, db2, dW3, db3]) of the batch-mean soft-target
    cross-entropy. Without casts this is the exact gradient."""
    c = bf16_round if cast else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = (np.asarray(p, dtype=np.float64) for p in params)
    f = forward(params, X, cast)
    Z = f["Z"]
    B, nb = Z.shape
    T = soft_targets(nbr_labels, nb)
    loss = loss_of_logits(Z, T)
    zmax = Z.max(axis=1, keepdims=True)
    Pm = np.exp(Z - zmax)
    Pm /= Pm.sum(axis=1, keepdims=True)
    dZ = (Pm - T) / B
    dZb = c(dZ)
    dW3 = dZb.T @ f["H2b"]
    db3 = dZ.sum(axis=0)
    dH2 = (dZb @ c(W3)) * (f["H2"] > 0)
    dH2b = c(dH2)
    dW2 = dH2b.T @ f["H1b"]
    db2 = dH2.sum(axis=0)
    dH1 = (dH2b @ c(W2)) * (f["H1"] > 0)
    dH1b = c(dH1)
    dW1 = dH1b.T @ f["Xb"]
    db1 = dH1.sum(axis=0)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


def adam_step(p, g, m1, m2, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step counts from 1); returns (p, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    mhat = m1 / (1 - b1 ** step)
    vhat = m2 / (1 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m1, m2


def top_buckets(Z: np.ndarray, P: int) -> np.ndarray:
    """The P largest logits of each row, descending, ties to the smaller id."""
    nb = Z.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(nb), Z.shape), -Z), axis=1)
    return order[:, :P].astype(np.int32)


def recall(idx_found: np.ndarray, idx_exact: np.ndarray) -> float:
    """Mean over rows of |found & exact| / k."""
    n, k = idx_exact.shape
    hits = 0
    for i in range(n):
        hits += len(np.intersect1d(idx_found[i], idx_exact[i], assume_unique=True))
    return hits / float(n * k)
