"""Pins of the oracle's exact k-NN and ad-hoc bandwidth (CPU only).

The oracle's neighbour lists follow the ordering I(x, k) of Section 2.1 with
I(x^(i), 0) = i: row i is i itself, then the k-1 nearest j != i, ties broken by
the smaller index. Pins: an independent dense numpy brute force, integer
lattices whose distances are exact in every precision (ties everywhere), and
the closed-form bandwidths of those lattices (bandwidth eq., Section 2.1).
"""
import numpy as np
import pytest

import oracle
import workloads


def numpy_knn(X, k):
    """Dense float64 distance matrix, then a lexicographic (distance, index)
    sort of every row with the row's own index removed."""
    X64 = X.astype(np.float64)
    n = len(X64)
    diff = X64[:, None, :] - X64[None, :, :]
    D = np.einsum("ijc,ijc->ij", diff, diff)
    idx = np.empty((n, k), dtype=np.int64)
    d2 = np.empty((n, k))
    cols = np.arange(n)
    for i in range(n):
        order = np.lexsort((cols, D[i]))
        order = order[order != i][: k - 1]
        idx[i, 0], d2[i, 0] = i, 0.0
        idx[i, 1:], d2[i, 1:] = order, D[i, order]
    return idx, d2


@pytest.mark.parametrize("n,m,k,seed", [(300, 1, 7, 0), (500, 3, 32, 1), (600, 16, 20, 2),
                                        (400, 64, 9, 3), (700, 3, 64, 4), (257, 5, 257, 5)])
def test_knn_matches_dense_bruteforce(n, m, k, seed):
    X = workloads.gaussian_iid(n, m, seed=seed)
    ref_i, ref_d = numpy_knn(X, k)
    idx, d2 = oracle.knn(X, k)
    np.testing.assert_array_equal(idx, ref_i)
    np.testing.assert_allclose(d2, ref_d, rtol=1e-13, atol=0)


def test_knn_duplicate_points_tie_break_by_index():
    rng = np.random.default_rng(11)
    base = rng.standard_normal((40, 3)).astype(np.float32)
    X = np.ascontiguousarray(np.repeat(base, 5, axis=0)[rng.permutation(200)])
    ref_i, _ = numpy_knn(X, 12)
    idx, d2 = oracle.knn(X, 12)
    np.testing.assert_array_equal(idx, ref_i)
    # every row: self first with distance 0, the 4 copies next (distance 0, index order)
    assert (idx[:, 0] == np.arange(200)).all()
    assert (d2[:, 1:5] == 0).all()
    assert (np.diff(idx[:, 1:5], axis=1) > 0).all()


def test_chain_lattice_rows():
    X = workloads.chain_lattice(50)
    idx, d2 = oracle.knn(X, 9)
    for i in range(4, 46):
        exp = [i, i - 1, i + 1, i - 2, i + 2, i - 3, i + 3, i - 4, i + 4]
        assert idx[i].tolist() == exp
        assert d2[i].tolist() == [0, 1, 1, 4, 4, 9, 9, 16, 16]
    assert idx[0].tolist() == list(range(9))
    assert idx[49].tolist() == [49] + list(range(48, 40, -1))


def test_cubic_lattice_shells():
    side = 5
    X = workloads.cubic_lattice(side)
    idx, d2 = oracle.knn(X, 19)
    c = 2 * 25 + 2 * 5 + 2          # the centre point (2, 2, 2)
    pts = X.astype(int)
    shell1 = sorted(j for j in range(len(X)) if ((pts[j] - pts[c]) ** 2).sum() == 1)
    shell2 = sorted(j for j in range(len(X)) if ((pts[j] - pts[c]) ** 2).sum() == 2)
    assert len(shell1) == 6 and len(shell2) == 12
    assert idx[c].tolist() == [c] + shell1 + shell2
    assert d2[c].tolist() == [0] + [1] * 6 + [2] * 12


def test_knn_degenerate_cases():
    X = np.zeros((30, 2), dtype=np.float32)       # all points identical
    idx, d2 = oracle.knn(X, 10)
    for i in range(30):
        assert idx[i].tolist() == [i] + [j for j in range(30) if j != i][:9]
    assert (d2 == 0).all()
    X2 = workloads.gaussian_iid(2, 3, seed=1)     # n = k = 2
    idx, d2 = oracle.knn(X2, 2)
    assert idx.tolist() == [[0, 1], [1, 0]]
    assert d2[0, 1] == d2[1, 1] > 0
    idx, _ = oracle.knn(workloads.gaussian_iid(9, 4, seed=2), 9)   # k = n: every row is a permutation
    assert all(sorted(r) == list(range(9)) for r in idx.tolist())


def test_knn_row_ranges_and_samples_agree():
    X = workloads.torus(3000, seed=3)
    full_i, full_d = oracle.knn(X, 16)
    part_i, part_d = oracle.knn(X, 16, rows=slice(1000, 1400))
    np.testing.assert_array_equal(part_i, full_i[1000:1400])
    rows = np.array([2999, 0, 1777, 5])
    s_i, s_d = oracle.knn_sampled(X, 16, rows)
    np.testing.assert_array_equal(s_i, full_i[rows])
    np.testing.assert_array_equal(s_d, full_d[rows])


def test_adhoc_bandwidth_closed_forms():
    X = workloads.chain_lattice(60)
    _, d2 = oracle.knn(X, 12)
    b = oracle.adhoc_bandwidth(d2, 8)
    # interior: 2 (1 + 4 + 9 + 16) = 60; first point: 1 + 4 + ... + 64 = 204
    assert b[30] ** 2 == pytest.approx(60.0, rel=1e-15)
    assert b[0] ** 2 == pytest.approx(204.0, rel=1e-15)
    # Z^3 interior: six neighbours at distance 1, then two at sqrt(2)
    Z = workloads.cubic_lattice(5)
    _, dz = oracle.knn(Z, 19)
    bz = oracle.adhoc_bandwidth(dz, 8)
    assert bz[62] ** 2 == pytest.approx(10.0, rel=1e-15)
