"""GPU parity of threshold truncation (run on an MI355X).

Section 4: Algorithm 1 stores an entry only when its kernel value exceeds the
sparsity tolerance delta_tol, which gives rows of varying length.
kvb_truncate_csr keeps the entries with exp(-d2/(e rho_i rho_j)) > delta; the
keep/drop decision is an integer taken from floating point, so the oracle
(oracle.truncate) takes it with the same operations in the same precision and
the kept patterns must agree bit for bit on the same inputs. In the whole
truncated build the decisions depend on the bandwidths b and rho, which the GPU
computes in float32; there the oracle's truncation is fed the GPU's b and rho
(its own values differ in the last places and would move entries that sit
exactly at the threshold), and every value is compared within the entry
tolerance of the untruncated path.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import spectral
from parity import check_entries, say

pytestmark = pytest.mark.gpu


def f64(t):
    return t.cpu().numpy().astype(np.float64)


def pair_ids(p):
    rows = np.repeat(np.arange(p.n, dtype=np.int64), np.diff(p.rowptr))
    return rows * (p.n + 1) + p.col


def check_same_pattern(g, r, what):
    np.testing.assert_array_equal(g.rowptr.cpu().numpy(), r.rowptr, err_msg=f"{what}: rowptr")
    np.testing.assert_array_equal(g.col.cpu().numpy(), r.col, err_msg=f"{what}: col")
    np.testing.assert_array_equal(f64(g.d2), r.dist2, err_msg=f"{what}: d2")


def gpu_base(g, idx, d2, pattern):
    """The GPU's base pattern, checked (rowptr, col) against the oracle's
    construction from the GPU's k-NN, then used with the GPU's distances as
    the oracle's input array (a pair stored in both rows may carry distances
    that differ in the last place, where one row rechecked it in FP64)."""
    ref = oracle.Pattern.from_knn(idx, d2) if pattern == "knn" else spectral.union_pattern(idx, d2)
    np.testing.assert_array_equal(g.base.rowptr.cpu().numpy(), ref.rowptr)
    np.testing.assert_array_equal(g.base.col.cpu().numpy(), ref.col)
    return oracle.Pattern(g.base.rowptr.cpu().numpy(), g.base.col.cpu().numpy(), f64(g.base.d2))


@pytest.mark.parametrize("delta", [0.3, 1e-2, 1e-6])
@pytest.mark.parametrize("union", [False, True])
def test_truncate_matches_oracle(gpu_lib, delta, union):
    kvb = gpu_lib
    n, k = 3000, 32
    say(f"[truncate] n={n} k={k} delta={delta} union={union}")
    X = workloads.sphere2(n, seed=5)
    idx, d2 = oracle.knn(X, k)
    d2f = d2.astype(np.float32)
    gi, gd = torch.from_numpy(idx).cuda(), torch.from_numpy(d2f).cuda()
    if union:
        gpat = kvb.union_pattern(gi, gd)
        rpat = spectral.union_pattern(idx, d2f.astype(np.float64))
    else:
        gpat = kvb.knn_pattern(gi, gd)
        rpat = oracle.Pattern.from_knn(idx, d2f.astype(np.float64))
    rng = np.random.default_rng(3)
    rho = (0.05 + 0.1 * rng.random(n)).astype(np.float32)
    e = 0.2
    g = kvb.truncate_csr(gpat, torch.from_numpy(rho).cuda(), e, delta)
    r = oracle.truncate(rpat, rho.astype(np.float64), e, delta)
    check_same_pattern(g, r, f"delta {delta}")
    assert 0 < g.nnz < gpat.nnz
    say(f"[truncate] kept {g.nnz} of {gpat.nnz}")


def test_truncate_limits_and_ragged(gpu_lib):
    """delta tiny keeps every entry, delta near 1 only the diagonal; n = 1 and
    a ragged row count; an invalid delta is rejected."""
    kvb = gpu_lib
    for n, k in ((1, 1), (777, 9)):
        X = np.random.default_rng(n).standard_normal((n, 3)).astype(np.float32)
        idx, d2 = oracle.knn(X, k)
        gpat = kvb.knn_pattern(torch.from_numpy(idx).cuda(), torch.from_numpy(d2.astype(np.float32)).cuda())
        rho = torch.ones(n, dtype=torch.float32, device="cuda")
        full = kvb.truncate_csr(gpat, rho, 0.1, 1e-300)
        assert torch.equal(full.col, gpat.col) and torch.equal(full.rowptr, gpat.rowptr)
        diag = kvb.truncate_csr(gpat, rho, 0.1, 1 - 1e-12)
        assert diag.col.cpu().tolist() == list(range(n))
    with pytest.raises(kvb.KvbError, match="delta"):
        kvb.truncate_csr(gpat, rho, 0.1, 1.0)


@pytest.mark.parametrize("pattern", ["knn", "union"])
def test_truncated_build_matches_oracle(gpu_lib, pattern):
    """The build with the paper's sparsity tolerance 1e-2 (Section 5 sets
    density-kernel entries below 1e-2 to zero) on the 2-sphere workload."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    n, delta = len(X), 1e-2
    say(f"[truncate] build, pattern {pattern}")
    g = kvb.build_truncated_matrix(torch.from_numpy(X).cuda(), w.k, w.k0, float(w.d), w.alpha, w.beta, delta,
                                   w.e_min, w.e_max, w.G, pattern=pattern)
    idx, d2 = g.idx.cpu().numpy(), f64(g.d2)
    base = gpu_base(g, idx, d2, pattern)
    ref = oracle.truncated_build(base, d2, w.k0, float(w.d), w.alpha, w.beta, delta, w.e_min, w.e_max, w.G)
    np.testing.assert_allclose(f64(g.b), ref["b"], rtol=2e-6)
    assert g.tune_a.e_star == pytest.approx(ref["ta"].e_star, rel=1e-13)
    e_a = g.tune_a.e_star
    # density stage: the decisions taken with the GPU's b
    pa = oracle.truncate(base, f64(g.b), e_a, delta)
    check_same_pattern(g.density_pattern, pa, "density pattern")
    # with the oracle's own b only entries at the threshold may move
    moved = len(np.setxor1d(pair_ids(pa), pair_ids(ref["pa"])))
    assert moved <= 1e-4 * len(pa.col) + 2
    psi_r, rho_r = oracle.density(pa, ref["b"], e_a, float(w.d), w.beta)
    np.testing.assert_allclose(f64(g.psi), psi_r, rtol=5e-6)
    np.testing.assert_allclose(f64(g.rho), rho_r, rtol=5e-6)
    assert g.scale_b == ref["s"]
    assert g.tune_b.e_star == pytest.approx(ref["tb"].e_star, rel=1e-13)
    e_b = g.tune_b.e_star
    # operator stage: the decisions taken with the GPU's rho
    rho_g = f64(g.rho)
    pb = oracle.truncate(base, rho_g, e_b, delta)
    check_same_pattern(g.pattern, pb, "operator pattern")
    val_r, q, P, D = oracle.normalize(pb, rho_g, e_b, w.alpha, float(w.d))
    rows = np.repeat(np.arange(n), np.diff(pb.rowptr))
    x = pb.dist2 / (e_b * rho_g[rows] * rho_g[pb.col])
    rowmax = np.maximum.reduceat(val_r, pb.rowptr[:-1])[rows]
    worst = check_entries(f64(g.val), val_r, x, rowmax, f"truncated {pattern} entries")
    np.testing.assert_allclose(g.D.cpu().numpy(), D, rtol=2e-5)
    rs = np.add.reduceat(f64(g.val), pb.rowptr[:-1])
    assert np.abs(rs - 1).max() < 2e-6
    assert (x < -np.log(delta) * (1 + 1e-12)).all()
    say(f"[truncate] {pattern}: kept {len(pb.col)} of {len(base.col)} entries, worst rel err {worst:.3g}")


def test_truncated_build_torus_n100k(gpu_lib):
    """The measured workload's size, the union pattern, delta 1e-2: the
    operator pattern bit for bit and every value, against the oracle fed the
    GPU's k-NN and rho."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["torus_n100k"]
    X = workloads.make(w.name, seed=0)
    n, delta = len(X), 1e-2
    say("[truncate] torus n=100000 union delta=1e-2")
    g = kvb.build_truncated_matrix(torch.from_numpy(X).cuda(), w.k, w.k0, float(w.d), w.alpha, w.beta, delta,
                                   w.e_min, w.e_max, w.G, pattern="union")
    idx, d2 = g.idx.cpu().numpy(), f64(g.d2)
    base = gpu_base(g, idx, d2, "union")
    rho_g = f64(g.rho)
    pb = oracle.truncate(base, rho_g, g.tune_b.e_star, delta)
    check_same_pattern(g.pattern, pb, "operator pattern")
    val_r, q, P, D = oracle.normalize(pb, rho_g, g.tune_b.e_star, w.alpha, float(w.d))
    rows = np.repeat(np.arange(n), np.diff(pb.rowptr))
    x = pb.dist2 / (g.tune_b.e_star * rho_g[rows] * rho_g[pb.col])
    rowmax = np.maximum.reduceat(val_r, pb.rowptr[:-1])[rows]
    check_entries(f64(g.val), val_r, x, rowmax, "torus truncated entries")
    say(f"[truncate] torus: kept {len(pb.col)} of {len(base.col)}")


@pytest.mark.parametrize("pattern", ["knn", "union"])
def test_single_call_truncated_build(gpu_lib, pattern):
    """kvb_build with a sparsity tolerance enqueues the truncated build without
    a host round trip. On the union pattern it matches the separate calls bit
    for bit (the tuning sums to rounding); on the k-NN pattern its rows are in
    column order, so the kept sets agree and the values to rounding."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["torus_n100k"]
    X = torch.from_numpy(workloads.torus(20000, seed=6)).cuda()
    delta = 1e-2
    say(f"[truncate] single call, pattern {pattern}")
    a = kvb.build_truncated_matrix(X, w.k, w.k0, float(w.d), w.alpha, w.beta, delta, w.e_min, w.e_max, w.G,
                                   pattern=pattern)
    b = kvb.build(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, pattern=pattern, delta=delta)
    assert a.tune_a.e_star == b.tune_a.e_star and a.tune_b.e_star == b.tune_b.e_star
    # the k-NN rows are summed in another order here, so rho and the
    # operator-stage sums agree to rounding only
    np.testing.assert_allclose(b.tune_b.chi, a.tune_b.chi, rtol=1e-12 if pattern == "union" else 1e-6)
    if pattern == "union":
        assert torch.equal(a.pattern.rowptr, b.rowptr)
        assert torch.equal(a.pattern.col, b.col)
        for f in ("rho", "psi", "val", "P", "D"):
            assert torch.equal(getattr(a, f), getattr(b, f)), f
    else:
        # the row sums run in another order, so rho may move an entry that
        # sits exactly at the threshold; such rows are counted, not compared
        n = X.shape[0]
        ra, rb = a.pattern.rowptr.cpu().numpy(), b.rowptr.cpu().numpy()
        same = np.diff(ra) == np.diff(rb)
        assert (~same).sum() <= 3
        ca, va = a.pattern.col.cpu().numpy(), a.val.cpu().numpy().astype(np.float64)
        cb, vb = b.col.cpu().numpy(), b.val.cpu().numpy().astype(np.float64)
        for i in np.nonzero(same)[0][::97]:
            oa = np.argsort(ca[ra[i]:ra[i + 1]])
            np.testing.assert_array_equal(ca[ra[i]:ra[i + 1]][oa], cb[rb[i]:rb[i + 1]])
            np.testing.assert_allclose(va[ra[i]:ra[i + 1]][oa], vb[rb[i]:rb[i + 1]], rtol=1e-6)
        torch.testing.assert_close(a.rho, b.rho, rtol=1e-6, atol=0)


def test_truncated_build_gmm_n8m_sampled_rows(gpu_lib):
    """The largest workload (n = 8e6, k = 64) built in one call with the
    sparsity tolerance 1e-2: the operator pattern's rows of 48 sampled samples
    against the keep rule x = (d2 (1 / (e rho_i))) / rho_j < -ln(delta),
    evaluated in float64 with the same operations on the GPU's rho and e_B,
    bit for bit; the rows are the k-NN rows in column order."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["gmm_n8m"]
    X = workloads.make(w.name, seed=0)
    n, k, delta = len(X), w.k, 1e-2
    say(f"[truncate] gmm_n8m: n={n} k={k} delta={delta}")
    g = kvb.build(torch.from_numpy(X).cuda(), k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G,
                  mode="bf16", margin=w.margin, delta=delta)
    rho = f64(g.rho)
    e_b = g.tune_b.e_star
    L = -np.log(delta)
    rowptr = g.rowptr.cpu().numpy()
    rng = np.random.default_rng(13)
    for i in np.sort(rng.choice(n, 48, replace=False)):
        order = np.argsort(g.idx[i].cpu().numpy(), kind="stable")
        cols = g.idx[i].cpu().numpy()[order]
        dd = g.d2[i].cpu().numpy()[order].astype(np.float64)
        x = dd * (1.0 / (e_b * rho[i])) / rho[cols]
        keep = x < L
        lo, hi = rowptr[i], rowptr[i + 1]
        assert g.col[lo:hi].cpu().numpy().tolist() == cols[keep].tolist(), i
    kept = int(rowptr[-1])
    assert kept == g.col.numel() and 0 < kept < n * k
    say(f"[truncate] gmm_n8m: kept {kept} of {n * k} entries ({kept / (n * k):.3f})")
