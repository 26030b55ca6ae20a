"""Pins of the learned-partitioner oracle (CPU only).

* SplitMix64 reproduces the reference outputs published with the generator.
* The teacher partition is balanced (recursive floor/ceil halving), every
  split separates the two halves along that node's direction, and one level
  reduces to a plain median split by sorting.
* The float64 MLP gradient matches central finite differences (no casts).
* The soft-target loss reduces to -log softmax for one-hot targets, and its
  logit gradient sums to zero per row.
* The bfloat16 rounding is round-to-nearest-even at 8 significant bits.
"""
import numpy as np
import pytest

from oracle import learned as OL


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 seeded with 1234567 (Vigna's reference code)
    got = OL.splitmix64(1234567, np.arange(5))
    want = np.array([6457827717110365317, 3203168211198807973, 9817491932198370423,
                     4593380528125082431, 16408922859458223821], dtype=np.uint64)
    assert np.array_equal(got, want)


def _sizes(ns, levels):
    sizes = [ns]
    for _ in range(levels):
        sizes = [s for t in sizes for s in (t // 2, t - t // 2)]
    return sizes


@pytest.mark.parametrize("ns,m,levels", [(1000, 3, 4), (777, 16, 5), (64, 1, 6)])
def test_teacher_balanced_and_separating(ns, m, levels):
    rng = np.random.default_rng(ns)
    X = rng.standard_normal((ns, m)).astype(np.float32)
    lab = OL.teacher_labels(X, levels, seed=5)
    counts = np.bincount(lab, minlength=1 << levels)
    assert counts.tolist() == _sizes(ns, levels)
    # every level: inside each parent node, the left child's projections lie
    # at or below the right child's along the parent's direction
    X64 = X.astype(np.float64)
    for level in range(levels):
        shift = levels - level
        parent = lab >> shift
        child = (lab >> (shift - 1)) & 1
        for v in range(1 << level):
            u = OL.teacher_direction(5, level, v, m)
            sel = parent == v
            p = (X64[sel] @ u).astype(np.float32)
            left, right = p[child[sel] == 0], p[child[sel] == 1]
            assert left.max() <= right.min()


def test_teacher_one_level_is_a_median_split():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((501, 4)).astype(np.float32)
    u = OL.teacher_direction(9, 0, 0, 4)
    p = (X.astype(np.float64) @ u).astype(np.float32)
    order = np.argsort(p, kind="stable")
    want = np.zeros(501, dtype=np.int32)
    want[order[250:]] = 1
    assert np.array_equal(OL.teacher_labels(X, 1, seed=9), want)


def test_teacher_direction_range_and_exactness():
    u = OL.teacher_direction(1, 3, 5, 1000)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    assert abs(u.mean()) < 0.1


def test_bf16_round_to_nearest_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, 1 + 2 ** -8 + 2 ** -20, -3.0 - 2 ** -7,
                  2.0 ** -100, 0.0])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, 1 + 2 ** -7, -3.0, 2.0 ** -100, 0.0])
    assert np.array_equal(OL.bf16_round(x), want)


def test_mlp_gradient_matches_finite_differences():
    m, h1, h2, nb, B, ks = 5, 7, 6, 9, 4, 3
    params = [p.astype(np.float64) for p in OL.init_params(m, h1, h2, nb, seed=2, bias_scale=0.3)]
    rng = np.random.default_rng(4)
    X = rng.standard_normal((B, m))
    lab = rng.integers(0, nb, size=(B, ks))
    loss, grads = OL.backward(params, X, lab, cast=False)
    flat = OL.flatten(params)
    g = OL.flatten(grads)
    T = OL.soft_targets(lab, nb)
    h = 1e-6
    for j in range(flat.size):
        fp, fm = flat.copy(), flat.copy()
        fp[j] += h
        fm[j] -= h
        lp = OL.loss_of_logits(OL.forward(OL.unflatten(fp, m, h1, h2, nb), X, False)["Z"], T)
        lm = OL.loss_of_logits(OL.forward(OL.unflatten(fm, m, h1, h2, nb), X, False)["Z"], T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 + 1e-5 * abs(fd), (j, fd, g[j])
    assert abs(loss - OL.loss_of_logits(OL.forward(params, X, False)["Z"], T)) < 1e-15


def test_soft_target_loss_special_cases():
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((6, 10))
    lab = rng.integers(0, 10, size=(6, 1))
    T = OL.soft_targets(lab, 10)
    logp = Z - np.log(np.exp(Z).sum(axis=1, keepdims=True))
    assert abs(OL.loss_of_logits(Z, T) - np.mean(-logp[np.arange(6), lab[:, 0]])) < 1e-14
    # targets are distributions; the logit gradient (softmax - t)/B sums to zero per row
    lab4 = rng.integers(0, 10, size=(6, 4))
    T4 = OL.soft_targets(lab4, 10)
    assert np.allclose(T4.sum(axis=1), 1.0)
    Pm = np.exp(Z) / np.exp(Z).sum(axis=1, keepdims=True)
    assert np.allclose(((Pm - T4) / 6).sum(axis=1), 0.0, atol=1e-16)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    p, m1, m2 = OL.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-5)


def test_top_buckets_ties_and_order():
    Z = np.array([[0.0, 2.0, 2.0, 1.0, -1.0], [5.0, 5.0, 5.0, 5.0, 5.0]])
    assert OL.top_buckets(Z, 3).tolist() == [[1, 2, 3], [0, 1, 2]]


def test_recall_definition():
    a = np.array([[0, 1, 2, 3], [4, 5, 6, 7]])
    b = np.array([[0, 1, 9, 8], [4, 5, 6, 7]])
    assert OL.recall(b, a) == pytest.approx(6 / 8)
