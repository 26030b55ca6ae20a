"""GPU k-NN parity against the FP64 oracle (run on an MI355X).

Every case calls kvb_knn through the C ABI on seeded inputs and compares with
the oracle's exact (distance, index) neighbour lists (Section 2.1 ordering).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import check_knn_rows, knn_reference, say

pytestmark = pytest.mark.gpu


def run_knn(kvb, X, k, margin, mode="f32", ctx=None):
    Xd = torch.from_numpy(X).cuda()
    idx, d2, flags = kvb.knn(Xd, k, mode=mode, margin=margin, ctx=ctx)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), d2.cpu().numpy(), flags.cpu().numpy()


CASES = [
    # (name, n, m, k, margin, seed)
    ("tiny_n1", 1, 3, 1, 0, 0),
    ("n2_k2", 2, 3, 2, 0, 1),
    ("n3_k3_m1", 3, 1, 3, 4, 2),
    ("n63_k9", 63, 3, 9, 8, 3),
    ("n64_k64", 64, 2, 64, 32, 4),
    ("n65_k33", 65, 3, 33, 32, 5),
    ("n1037_k32_m3", 1037, 3, 32, 32, 6),
    ("n1037_k32_m3_margin0", 1037, 3, 32, 0, 7),
    ("n2049_k64_m5", 2049, 5, 64, 32, 8),
    ("n1500_k128_m8", 1500, 8, 128, 32, 9),
    ("n1000_k200_m4", 1000, 4, 200, 56, 10),
    ("n700_k16_m12", 700, 12, 16, 16, 11),
    ("n900_k40_m16", 900, 16, 40, 32, 12),
    ("n500_k20_m64", 500, 64, 20, 8, 13),
    ("n3000_k64_m1", 3000, 1, 64, 32, 14),
]


@pytest.mark.parametrize("name,n,m,k,margin,seed", CASES, ids=[c[0] for c in CASES])
def test_knn_random(gpu_lib, name, n, m, k, margin, seed):
    say(f"[knn] {name}: n={n} m={m} k={k} margin={margin} seed={seed}")
    X = workloads.gaussian_iid(n, m, seed=seed)
    gi, gd, fl = run_knn(gpu_lib, X, k, margin)
    ri, rd = knn_reference(X, k)
    ties = check_knn_rows(gi, gd, ri, rd, k, np.arange(n))
    say(f"[knn] {name}: ok, near-tie rows {ties}, fallback rows {int(((fl & 2) > 0).sum())}")


@pytest.mark.parametrize("margin", [0, 4, 32])
def test_knn_chain_lattice_bitwise(gpu_lib, margin):
    say(f"[knn] chain lattice margin={margin}")
    X = workloads.chain_lattice(300)
    gi, gd, fl = run_knn(gpu_lib, X, 9, margin)
    ri, rd = oracle.knn(X, 9)
    np.testing.assert_array_equal(gi, ri)
    np.testing.assert_array_equal(gd, rd.astype(np.float32))


@pytest.mark.parametrize("margin", [0, 32])
def test_knn_cubic_lattice_bitwise(gpu_lib, margin):
    say(f"[knn] cubic lattice margin={margin}")
    X = workloads.cubic_lattice(9)
    gi, gd, fl = run_knn(gpu_lib, X, 19, margin)
    ri, rd = oracle.knn(X, 19)
    np.testing.assert_array_equal(gi, ri)
    np.testing.assert_array_equal(gd, rd.astype(np.float32))


def test_knn_duplicates_and_identical_points(gpu_lib):
    say("[knn] duplicates")
    rng = np.random.default_rng(11)
    base = rng.standard_normal((40, 3)).astype(np.float32)
    X = np.ascontiguousarray(np.repeat(base, 5, axis=0)[rng.permutation(200)])
    for margin in (0, 4, 32):
        gi, gd, fl = run_knn(gpu_lib, X, 12, margin)
        ri, rd = oracle.knn(X, 12)
        np.testing.assert_array_equal(gi, ri)
    say("[knn] identical points")
    Z = np.zeros((300, 3), dtype=np.float32)
    gi, gd, fl = run_knn(gpu_lib, Z, 10, 16)
    ri, rd = oracle.knn(Z, 10)
    np.testing.assert_array_equal(gi, ri)
    assert (gd == 0).all()
    assert ((fl & 2) > 0).all(), "every row of identical points needs the exact fallback"


def test_knn_forced_fallback_matches(gpu_lib):
    say("[knn] forced fallback on the sphere")
    from paper_2104_15124_amd import kvb
    X = workloads.sphere2(2000, seed=0)
    ctx = kvb.Context()
    ctx.set_option(kvb.OPT_FORCE_FALLBACK, 3)
    gi, gd, fl = run_knn(gpu_lib, X, 32, 32, ctx=ctx)
    assert kvb.knn_fallback_rows(ctx) == len(range(0, 2000, 3))
    ri, rd = knn_reference(X, 32)
    check_knn_rows(gi, gd, ri, rd, 32, np.arange(2000))
    assert ((fl[::3] & 2) > 0).all()
    ctx.close()


@pytest.mark.parametrize("mode,m", [("f32", 3), ("f32", 16), ("bf16", 64), ("bf16", 128), ("f32", 200)])
def test_knn_forced_fallback_duplicates(gpu_lib, mode, m):
    """Every row through the exact fallback: 1500 copies of one point (their
    bounded-pass buffers overflow, so they take the full scan) among 700
    distinct points (finished by the bounded pass); ties ranked by index."""
    from paper_2104_15124_amd import kvb
    say(f"[knn] forced fallback with 1500 duplicates, mode={mode} m={m}")
    rng = np.random.default_rng(17)
    X = rng.standard_normal((2200, m)).astype(np.float32)
    X[rng.permutation(2200)[:1500]] = X[0]
    ctx = kvb.Context()
    ctx.set_option(kvb.OPT_FORCE_FALLBACK, 1)
    gi, gd, fl = run_knn(gpu_lib, X, 24, 16, mode=mode, ctx=ctx)
    assert kvb.knn_fallback_rows(ctx) == 2200
    ctx.close()
    ri, rd = oracle.knn(X, 24)
    np.testing.assert_array_equal(gi, ri)
    np.testing.assert_array_equal(gd, rd.astype(np.float32))


def test_knn_sphere_n2000_k32(gpu_lib):
    say("[knn] sphere2 n=2000 k=32 (full oracle)")
    X = workloads.make("sphere2_n2000", seed=0)
    gi, gd, fl = run_knn(gpu_lib, X, 32, 32)
    ri, rd = knn_reference(X, 32)
    check_knn_rows(gi, gd, ri, rd, 32, np.arange(len(X)))


def test_knn_torus_n100k_k64_full(gpu_lib):
    """The measured workload at full size, in the launch configuration the
    benchmark times, against the oracle on every row."""
    say("[knn] torus n=100000 k=64 (full oracle)")
    X = workloads.make("torus_n100k", seed=0)
    gi, gd, fl = run_knn(gpu_lib, X, 64, 32)
    ri, rd = knn_reference(X, 64)
    ties = check_knn_rows(gi, gd, ri, rd, 64, np.arange(len(X)))
    say(f"[knn] torus: ok, near-tie rows {ties}, fallback rows {int(((fl & 2) > 0).sum())}")


def test_knn_deterministic(gpu_lib):
    say("[knn] determinism")
    X = workloads.torus(20000, seed=5)
    a = run_knn(gpu_lib, X, 64, 32)
    b = run_knn(gpu_lib, X, 64, 32)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)


def test_knn_invalid_arguments(gpu_lib):
    from paper_2104_15124_amd import kvb
    X = torch.zeros((10, 3), device="cuda")
    with pytest.raises(kvb.KvbError) as e:
        kvb.knn(X, 11)                       # k > n
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.knn(X, 5, margin=-1)
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.knn(torch.zeros((300, 3), device="cuda"), 200, margin=100)   # k + margin > 256
    assert e.value.code == kvb.E_UNSUPPORTED


# ---------------------------------------------------------------- matrix-core tiles
def _gen(kind, n, m, seed):
    if kind == "gauss":
        return workloads.gaussian_iid(n, m, seed=seed)
    if kind == "nonlinear5":
        return workloads.nonlinear5(n, seed=seed)
    if kind == "sphere3":
        return workloads.sphere3_lifted(n, seed=seed, m=m)
    if kind == "gmm":
        return workloads.gaussian_mixture(n, seed=seed, m=m)
    raise ValueError(kind)


MFMA_CASES = [
    # (name, kind, n, m, k, margin, mode, split, seed)
    ("f32_gauss_m9", "gauss", 1500, 9, 32, 32, "f32", 3, 21),
    ("f32_gmm_m16", "gmm", 3001, 16, 64, 32, "f32", 3, 22),
    ("f32_nl5_m64", "nonlinear5", 2500, 64, 64, 32, "f32", 3, 23),
    ("f32_s3_m128_k128", "sphere3", 2049, 128, 128, 32, "f32", 3, 24),
    ("bf16x3_gmm_m16", "gmm", 3001, 16, 64, 32, "bf16", 3, 25),
    ("bf16x3_nl5_m64", "nonlinear5", 2500, 64, 64, 32, "bf16", 3, 26),
    ("bf16x3_s3_m128_k128", "sphere3", 2049, 128, 128, 32, "bf16", 3, 27),
    ("bf16x6_gmm_m16", "gmm", 3001, 16, 64, 32, "bf16", 6, 28),
    ("bf16x6_nl5_m40", "gauss", 1100, 40, 20, 16, "bf16", 6, 29),
    ("bf16x1_nl5_m64", "nonlinear5", 1200, 64, 32, 32, "bf16", 1, 30),
    ("bf16x3_tiny_n33", "gauss", 33, 20, 9, 4, "bf16", 3, 31),
    ("bf16x3_k1", "gauss", 100, 16, 1, 0, "bf16", 3, 32),
    # rows of odd length (no float4 reads in the re-rank)
    ("f32_gauss_m37", "gauss", 1300, 37, 24, 16, "f32", 3, 33),
    ("bf16x3_gauss_m150", "gauss", 900, 150, 16, 16, "bf16", 3, 34),
]


@pytest.mark.parametrize("name,kind,n,m,k,margin,mode,split,seed", MFMA_CASES, ids=[c[0] for c in MFMA_CASES])
def test_knn_matrix_core_tiles(gpu_lib, name, kind, n, m, k, margin, mode, split, seed):
    from paper_2104_15124_amd import kvb
    say(f"[knn-mfma] {name}: n={n} m={m} k={k} margin={margin} mode={mode} split={split}")
    X = _gen(kind, n, m, seed)
    ctx = kvb.Context()
    ctx.set_option(kvb.OPT_BF16_SPLIT, split)
    gi, gd, fl = run_knn(gpu_lib, X, k, margin, mode=mode, ctx=ctx)
    nfb = kvb.knn_fallback_rows(ctx)
    ctx.close()
    ri, rd = knn_reference(X, k)
    ties = check_knn_rows(gi, gd, ri, rd, k, np.arange(n))
    say(f"[knn-mfma] {name}: ok, near-tie rows {ties}, fallback rows {nfb} of {n}")
    if split >= 3 and kind != "gauss":
        assert nfb <= n // 20, "the split-BF16 error bound should certify almost every row"


def test_knn_bf16_lattice_and_duplicates(gpu_lib):
    from paper_2104_15124_amd import kvb
    say("[knn-mfma] lattice in R^16 and duplicates, BF16")
    Z = workloads.cubic_lattice(7)
    X = np.zeros((len(Z), 16), dtype=np.float32)
    X[:, :3] = Z
    gi, gd, fl = run_knn(gpu_lib, X, 19, 8, mode="bf16")
    ri, rd = oracle.knn(X, 19)
    np.testing.assert_array_equal(gi, ri)
    rng = np.random.default_rng(3)
    base = rng.standard_normal((50, 24)).astype(np.float32)
    D = np.ascontiguousarray(np.repeat(base, 4, axis=0)[rng.permutation(200)])
    gi, gd, fl = run_knn(gpu_lib, D, 10, 4, mode="bf16")
    ri, rd = oracle.knn(D, 10)
    np.testing.assert_array_equal(gi, ri)


def test_knn_nonlinear5_n1m_sampled_rows(gpu_lib):
    """The BF16 workload at full size (n = 1e6, m = 64, k = 64, margin 32),
    timed launch configuration; 256 sampled rows checked against the oracle,
    all rows checked for the row invariants."""
    from paper_2104_15124_amd import kvb
    w = workloads.WORKLOADS["nonlinear5_n1m"]
    say(f"[knn-mfma] {w.name}: n={w.n} m={w.m} k={w.k} (sampled oracle rows)")
    X = workloads.make(w.name, seed=0)
    ctx = kvb.Context()
    gi, gd, fl = run_knn(gpu_lib, X, w.k, w.margin, mode="bf16", ctx=ctx)
    nfb = kvb.knn_fallback_rows(ctx)
    pairs = kvb.knn_pairs(ctx)
    ctx.close()
    say(f"[knn-mfma] {w.name}: fallback rows {nfb}, candidate pairs {pairs:.4g} of {float(w.n) ** 2:.4g}")
    # five intrinsic dimensions: the curve-ordered scan skips tiles
    assert pairs < 0.5 * float(w.n) ** 2
    assert (gi[:, 0] == np.arange(w.n)).all()
    assert (np.diff(gd, axis=1) >= 0).all()
    rows = np.random.default_rng(7).choice(w.n, 256, replace=False)
    ri, rd = knn_reference(X, w.k, rows=rows)
    check_knn_rows(gi[rows], gd[rows], ri, rd, w.k, rows)
    assert nfb <= w.n // 100


LARGE_CASES = [("sphere3_n4m", "bf16"), ("gmm_n8m", "f32"), ("gmm_n8m", "bf16")]


@pytest.mark.parametrize("name,mode", LARGE_CASES, ids=[f"{c[0]}_{c[1]}" for c in LARGE_CASES])
def test_knn_large_workloads_sampled_rows(gpu_lib, name, mode):
    """The two largest workloads at full size in the exact modes the benchmark
    times (the lifted 3-sphere: n = 4e6, m = 128, k = 128; the mixture:
    n = 8e6, m = 16, k = 64; margin 32, curve order): 256 sampled rows
    against the oracle's exact rows, every row against the row invariants."""
    from paper_2104_15124_amd import kvb
    w = workloads.WORKLOADS[name]
    say(f"[knn-large] {name}: n={w.n} m={w.m} k={w.k} mode={mode} (sampled oracle rows)")
    X = workloads.make(w.name, seed=0)
    ctx = kvb.Context()
    gi, gd, fl = run_knn(gpu_lib, X, w.k, w.margin, mode=mode, ctx=ctx)
    nfb = kvb.knn_fallback_rows(ctx)
    pairs = kvb.knn_pairs(ctx)
    ctx.close()
    say(f"[knn-large] {name}: fallback rows {nfb}, candidate pairs {pairs:.4g} ({pairs / float(w.n) ** 2:.3%} of n^2)")
    assert (gi[:, 0] == np.arange(w.n)).all()
    assert (gd[:, 0] == 0).all() and (np.diff(gd, axis=1) >= 0).all()
    assert ((gi >= 0) & (gi < w.n)).all()
    rows = np.random.default_rng(11).choice(w.n, 256, replace=False)
    ri, rd = knn_reference(X, w.k, rows=rows)
    ties = check_knn_rows(gi[rows], gd[rows], ri, rd, w.k, rows)
    say(f"[knn-large] {name}: 256 sampled rows match the oracle (near-tie rows {ties})")
    assert nfb <= w.n // 100


EXACT_ROWS_CASES = [("n3000_m3_k32", 3000, 3, 32, 1), ("n2000_m64_k64", 2000, 64, 64, 2), ("n500_m7_k1", 500, 7, 1, 3)]


@pytest.mark.parametrize("name,n,m,k,seed", EXACT_ROWS_CASES, ids=[c[0] for c in EXACT_ROWS_CASES])
def test_knn_exact_rows(gpu_lib, name, n, m, k, seed):
    say(f"[knn-exact-rows] {name}")
    X = workloads.gaussian_iid(n, m, seed=seed)
    rng = np.random.default_rng(seed)
    rows = rng.choice(n, size=min(n, 300), replace=False).astype(np.int32)
    gi, gd = gpu_lib.knn_exact_rows(torch.from_numpy(X).cuda(), k, torch.from_numpy(rows).cuda())
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    ri, rd = knn_reference(X, k, rows)
    check_knn_rows(gi, gd, ri, rd, k, rows)
    # an id outside [0, n) gives a row of -1
    bad = torch.tensor([0, n, -1], dtype=torch.int32, device="cuda")
    bi, bd = gpu_lib.knn_exact_rows(torch.from_numpy(X).cuda(), k, bad)
    bi = bi.cpu().numpy()
    assert bi[0, 0] == 0 and (bi[1] == -1).all() and (bi[2] == -1).all()


# ------------------------------------------------ curve order and box pruning
CURVE_CASES = [
    # (name, kind, n, m, k, margin, mode, split, seed)
    ("nl5_m64_bf16", "nonlinear5", 20000, 64, 64, 32, "bf16", 3, 41),
    ("s3_m128_f32", "sphere3", 12000, 128, 32, 16, "f32", 3, 42),
    ("gmm_m16_bf16x6", "gmm", 15001, 16, 64, 32, "bf16", 6, 43),
    ("gauss_m24_f32", "gauss", 5000, 24, 16, 8, "f32", 3, 44),
    ("s3_m8_bf16", "sphere3", 9000, 8, 48, 16, "bf16", 3, 45),
]


@pytest.mark.parametrize("name,kind,n,m,k,margin,mode,split,seed", CURVE_CASES, ids=[c[0] for c in CURVE_CASES])
def test_knn_curve_order_matches_plain_scan(gpu_lib, name, kind, n, m, k, margin, mode, split, seed):
    """The curve-ordered scans with projected-box pruning (Morton order, and
    Morton order with median splits inside 4096-tile groups) return the same
    exact neighbour lists as the scan of every tile; on samples of low
    intrinsic dimension they evaluate fewer candidate pairs."""
    from paper_2104_15124_amd import kvb
    say(f"[knn-curve] {name}: n={n} m={m} k={k} margin={margin} mode={mode} split={split}")
    X = _gen(kind, n, m, seed)
    out = {}
    for curve in (2, 1, 0):
        ctx = kvb.Context()
        ctx.set_option(kvb.OPT_BF16_SPLIT, split)
        ctx.set_option(kvb.OPT_CURVE_ORDER, curve)
        gi, gd, fl = run_knn(gpu_lib, X, k, margin, mode=mode, ctx=ctx)
        out[curve] = (gi, gd, kvb.knn_pairs(ctx), kvb.knn_fallback_rows(ctx))
        ctx.close()
    pi, pd, ppairs, pfb = out[0]
    assert ppairs == float(n) * n
    rows = np.random.default_rng(seed).choice(n, 200, replace=False)
    ri, rd = knn_reference(X, k, rows=rows)
    for curve in (2, 1):
        ci, cd, cpairs, cfb = out[curve]
        say(f"[knn-curve] {name}: order {curve}: pairs {cpairs:.4g} (plain {ppairs:.4g}), "
            f"fallback rows {cfb} / {pfb}")
        np.testing.assert_array_equal(cd, pd)
        # indices may differ only among neighbours at exactly equal distances
        for r in np.nonzero((ci != pi).any(axis=1))[0]:
            for p in np.nonzero(ci[r] != pi[r])[0]:
                assert (cd[r] == cd[r][p]).sum() > 1 or cd[r][p] == cd[r][-1], f"row {r} position {p}"
        check_knn_rows(ci[rows], cd[rows], ri, rd, k, rows)
        assert cpairs <= ppairs


def test_knn_median_splits_score_fewer_pairs(gpu_lib):
    """On the 4-dimensional mixture (the 8M workload's recipe at n = 500k) the
    median splits inside the curve's 4096-tile groups give tighter tile boxes:
    the exact scan scores at most 80% of the Morton order's pairs, with the
    same neighbour distances."""
    from paper_2104_15124_amd import kvb
    X = workloads.make("gmm_n8m", seed=3, n=500_000)
    out = {}
    for curve in (1, 2):
        ctx = kvb.Context()
        ctx.set_option(kvb.OPT_CURVE_ORDER, curve)
        gi, gd, fl = run_knn(gpu_lib, X, 64, 32, mode="f32", ctx=ctx)
        out[curve] = (gd, kvb.knn_pairs(ctx))
        ctx.close()
    say(f"[knn-curve] mixture n=500k: pairs Morton {out[1][1]:.4g}, with median splits {out[2][1]:.4g}")
    np.testing.assert_array_equal(out[1][0], out[2][0])
    assert out[2][1] <= 0.8 * out[1][1]


def test_knn_curve_rank_deficient_and_small(gpu_lib):
    """Covariance of rank below the projection dimension (zero basis columns),
    a single tile, and n not a multiple of the tile height."""
    from paper_2104_15124_amd import kvb
    say("[knn-curve] rank-deficient and small cases")
    rng = np.random.default_rng(5)
    for n, m, k, r in ((31, 12, 7, 2), (97, 40, 20, 1), (2500, 32, 32, 3), (777, 10, 64, 10)):
        B = rng.standard_normal((r, m)).astype(np.float32)
        X = np.ascontiguousarray((rng.standard_normal((n, r)).astype(np.float32) @ B).astype(np.float32))
        for mode in ("f32", "bf16"):
            say(f"[knn-curve] n={n} m={m} k={k} rank={r} mode={mode}")
            gi, gd, fl = run_knn(gpu_lib, X, k, 8, mode=mode)
            ri, rd = knn_reference(X, k)
            check_knn_rows(gi, gd, ri, rd, k, np.arange(n))
