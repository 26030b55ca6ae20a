"""GPU parity of the union pattern E u E^T and of the passes over it (run on an MI355X).

The paper's kernel matrix is symmetric (Section 4, Algorithm 1 stores K_ij and
K_ji together). kvb_union_pattern builds E u E^T of the directed k-NN pattern
on the device; kvb_density_csr, kvb_tune_eps_csr and kvb_normalize_csr run the
density, tuning and normalisation passes of Sections 2.1-2.3 over it. Each is
compared with the FP64 oracle (oracle.spectral.union_pattern and the oracle's
CSR passes) on the same seeded samples: the pattern bit for bit, the values
within the entry tolerance of the directed path.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import workloads
from oracle import spectral
from parity import D2_RTOL, check_entries, check_knn_rows, knn_reference, say

pytestmark = pytest.mark.gpu


def near_tie(slope):
    s = np.sort(slope)
    return (s[-1] - s[-2]) <= 1e-5 * abs(s[-1])


def check_pattern(gpat, rpat, what):
    rowptr = gpat.rowptr.cpu().numpy()
    col = gpat.col.cpu().numpy()
    np.testing.assert_array_equal(rowptr, rpat.rowptr, err_msg=f"{what}: rowptr")
    np.testing.assert_array_equal(col, rpat.col, err_msg=f"{what}: col")
    gd = gpat.d2.cpu().numpy().astype(np.float64)
    err = np.abs(gd - rpat.dist2)
    assert (err <= D2_RTOL * rpat.dist2 + 1e-30).all(), f"{what}: d2 max rel err " \
        f"{np.max(err / np.maximum(rpat.dist2, 1e-30))}"


def oracle_union_build(idx, d2, w, out_kind=oracle.MARKOV):
    """The oracle's passes in the order of the build, every row sum over E u E^T."""
    pat = spectral.union_pattern(idx, d2)
    b = oracle.adhoc_bandwidth(d2, w.k0)
    ta = oracle.chi(pat, b, w.e_min, w.e_max, w.G)
    psi, rho = oracle.density(pat, b, ta.e_star, float(w.d), w.beta)
    s = oracle.grid_scale(b, rho)
    tb = oracle.chi(pat, rho, w.e_min * s, w.e_max * s, w.G)
    val, q, P, D = oracle.normalize(pat, rho, tb.e_star, w.alpha, float(w.d), out_kind)
    return dict(pat=pat, b=b, ta=ta, psi=psi, rho=rho, s=s, tb=tb, val=val, P=P, D=D)


def compare_union_build(kvb, name, X, w, oracle_knn=True):
    n, k = len(X), w.k
    say(f"[union] {name}: n={n} m={X.shape[1]} k={k}")
    Xd = torch.from_numpy(X).cuda()
    g = kvb.build_union_matrix(Xd, k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, mode="f32",
                               margin=w.margin)
    torch.cuda.synchronize()
    gi, gd = g.idx.cpu().numpy(), g.d2.cpu().numpy()
    if oracle_knn:
        ri, rd = knn_reference(X, k)
        assert check_knn_rows(gi, gd, ri, rd, k, np.arange(n)) == 0
        idx, d2 = ri[:, :k], rd[:, :k]
    else:
        # the GPU's exact k-NN (checked by the k-NN parity tests) as the input array
        idx, d2 = gi, gd.astype(np.float64)
    ref = oracle_union_build(idx, d2, w)
    check_pattern(g.pattern, ref["pat"], name)
    np.testing.assert_allclose(g.b.cpu().numpy(), ref["b"], rtol=2e-6)
    np.testing.assert_allclose(g.tune_a.chi, ref["ta"].chi, rtol=2e-5)
    assert not near_tie(ref["ta"].slope), "the oracle's two best slopes tie: pick another seed"
    assert g.tune_a.e_star == pytest.approx(ref["ta"].e_star, rel=1e-13)
    np.testing.assert_allclose(g.psi.cpu().numpy(), ref["psi"], rtol=5e-6)
    np.testing.assert_allclose(g.rho.cpu().numpy(), ref["rho"], rtol=5e-6)
    assert g.scale_b == ref["s"]
    np.testing.assert_allclose(g.tune_b.chi, ref["tb"].chi, rtol=2e-5)
    assert not near_tie(ref["tb"].slope)
    assert g.tune_b.e_star == pytest.approx(ref["tb"].e_star, rel=1e-13)
    pat = ref["pat"]
    e_b = ref["tb"].e_star
    rows = np.repeat(np.arange(n), np.diff(pat.rowptr))
    x = pat.dist2 / (e_b * ref["rho"][rows] * ref["rho"][pat.col])
    rowmax = np.maximum.reduceat(ref["val"], pat.rowptr[:-1])[rows]
    val = g.val.cpu().numpy().astype(np.float64)
    worst = check_entries(val, ref["val"], x, rowmax, f"{name} union Markov entries")
    np.testing.assert_allclose(g.P.cpu().numpy(), ref["P"], rtol=1e-7)
    np.testing.assert_allclose(g.D.cpu().numpy(), ref["D"], rtol=2e-5)
    rs = np.add.reduceat(val, pat.rowptr[:-1])
    assert np.abs(rs - 1).max() < 2e-6
    say(f"[union] {name}: ok, nnz={len(pat.col)} ({len(pat.col) / (n * k):.3f} n k), "
        f"worst entry rel err {worst:.3g}")
    return g, ref


def test_union_build_sphere_n2000(gpu_lib):
    w = workloads.WORKLOADS["sphere2_n2000"]
    compare_union_build(gpu_lib, "sphere2_n2000", workloads.make(w.name, seed=0), w)


def test_union_build_torus_n100k_full(gpu_lib):
    """The measured workload's size; the GPU's exact k-NN is the oracle's input."""
    w = workloads.WORKLOADS["torus_n100k"]
    compare_union_build(gpu_lib, "torus_n100k", workloads.make(w.name, seed=0), w, oracle_knn=False)


@pytest.mark.parametrize("n,m,k", [(1, 3, 1), (7, 2, 7), (1001, 3, 17), (3000, 3, 200), (5000, 16, 100),
                                   (50, 4, 1)])
def test_union_pattern_shapes(gpu_lib, n, m, k):
    """Ragged sizes, one- and three-slot rows, k = n (the union is the
    directed pattern) and k = 1 (only the diagonal)."""
    say(f"[union] pattern n={n} m={m} k={k}")
    rng = np.random.default_rng(n * 7 + k)
    X = rng.standard_normal((n, m)).astype(np.float32)
    idx, d2 = oracle.knn(X, k)
    gpat = gpu_lib.union_pattern(torch.from_numpy(idx).cuda(), torch.from_numpy(d2.astype(np.float32)).cuda())
    check_pattern(gpat, spectral.union_pattern(idx, d2.astype(np.float32).astype(np.float64)), f"n{n} k{k}")
    if k == n:
        assert gpat.nnz == n * n
    if k == 1:
        assert gpat.nnz == n


def hub_pattern(n, k):
    """Every row lists the k-1 lowest other indices: rows 0..k-1 of the union
    hold (almost) all n samples; the squared distance is symmetric in (i, j)."""
    idx = np.empty((n, k), dtype=np.int32)
    for i in range(n):
        idx[i] = [i] + [j for j in range(k + 1) if j != i][:k - 1]
    ii = np.repeat(np.arange(n), k).reshape(n, k)
    d2 = (0.001 * (ii + idx + 1) * (ii != idx)).astype(np.float32)
    return idx, d2


def test_union_reverse_segment_lengths(gpu_lib):
    """Reverse segments of 1-64, 65-256 and over 256 entries (the three sort
    paths) in one pattern: rows 0, 1, 2 are listed by 50, 200 and 1000 other
    rows that they do not list themselves."""
    n, k = 3000, 8
    idx = np.empty((n, k), dtype=np.int32)
    for i in range(n):
        row = [i]
        hub = 0 if 100 <= i < 150 else 1 if 200 <= i < 400 else 2 if 1000 <= i < 2000 else -1
        if hub >= 0:
            row.append(hub)
        j = i + 3
        while len(row) < k:
            c = j % n
            if c not in row and c > 2:
                row.append(c)
            j += 1
        idx[i] = row
    d2 = (np.arange(n * k).reshape(n, k) % 97 * 0.01).astype(np.float32)
    d2[:, 0] = 0
    say("[union] reverse segments of 50, 200 and 1000 entries")
    gpat = gpu_lib.union_pattern(torch.from_numpy(idx).cuda(), torch.from_numpy(d2).cuda())
    # the distance of a pair stored in both directions differs here, so only
    # the pattern is compared, and the distances of the hub rows' reverse entries
    rpat = spectral.union_pattern(idx, d2.astype(np.float64))
    np.testing.assert_array_equal(gpat.rowptr.cpu().numpy(), rpat.rowptr)
    np.testing.assert_array_equal(gpat.col.cpu().numpy(), rpat.col)
    lens = np.diff(rpat.rowptr)[:3]
    assert lens.tolist() == [k + 50, k + 200, k + 1000]
    gd = gpat.d2.cpu().numpy()
    for h in range(3):
        for t in range(rpat.rowptr[h], rpat.rowptr[h + 1]):
            c = rpat.col[t]
            if c not in idx[h]:   # a reverse entry: its distance comes from row c
                r = int(np.nonzero(idx[c] == h)[0][0])
                assert gd[t] == d2[c, r], (h, c)


def test_union_hub_rows_and_csr_passes(gpu_lib):
    """Rows far longer than k (in-degree n) through the pattern build and all
    three CSR passes, against the oracle's passes on the same pattern."""
    n, k = 6000, 24
    idx, d2 = hub_pattern(n, k)
    say(f"[union] hub rows n={n} k={k}")
    gpat = gpu_lib.union_pattern(torch.from_numpy(idx).cuda(), torch.from_numpy(d2).cuda())
    rpat = spectral.union_pattern(idx, d2.astype(np.float64))
    check_pattern(gpat, rpat, "hub")
    assert int(np.diff(rpat.rowptr).max()) >= n - 1
    rng = np.random.default_rng(5)
    b = (0.5 + rng.random(n)).astype(np.float32)
    bd = torch.from_numpy(b).cuda()
    tg = gpu_lib.tune_eps_csr(gpat, bd, 1e-3, 1e1, 64)
    tr = oracle.chi(rpat, b.astype(np.float64), 1e-3, 1e1, 64)
    np.testing.assert_allclose(tg.chi, tr.chi, rtol=2e-5)
    e = 0.05
    rho, psi = gpu_lib.density_csr(gpat, bd, e, 2.0, -0.5)
    psi_r, rho_r = oracle.density(rpat, b.astype(np.float64), e, 2.0, -0.5)
    np.testing.assert_allclose(psi.cpu().numpy(), psi_r, rtol=5e-6)
    np.testing.assert_allclose(rho.cpu().numpy(), rho_r, rtol=5e-6)
    for kind in (oracle.MARKOV, oracle.GENERATOR, oracle.SYMMETRIC):
        val, P, D = gpu_lib.normalize_csr(gpat, rho, 0.2, -0.5, 2.0, kind)
        vr, q, Pr, Dr = oracle.normalize(rpat, rho.cpu().numpy().astype(np.float64), 0.2, -0.5, 2.0, kind)
        v = val.cpu().numpy().astype(np.float64)
        scale = np.abs(vr).max()
        err = np.abs(v - vr)
        assert (err <= 1e-5 * np.abs(vr) + 1e-6 * scale).all(), (kind, float(np.max(err / (np.abs(vr) + scale))))
        np.testing.assert_allclose(D.cpu().numpy(), Dr, rtol=2e-5)


@pytest.mark.parametrize("out_kind", [1, 2])
def test_union_output_kinds_and_spectrum(gpu_lib, out_kind):
    """Generator and symmetric conjugate on the union pattern. The conjugate is
    symmetric up to float32 rounding and similar to L, so both give the
    oracle's leading eigenvalues (Section 2.2; they approach -l(l+1) on the
    sphere, Section 5.2)."""
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    n = len(X)
    say(f"[union] output kind {out_kind}")
    g = gpu_lib.build_union_matrix(torch.from_numpy(X).cuda(), w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min,
                                   w.e_max, w.G, out_kind=out_kind)
    ref = oracle_union_build(*oracle.knn(X, w.k), w, out_kind=out_kind)
    val = g.val.cpu().numpy().astype(np.float64)
    scale = np.abs(ref["val"]).max()
    err = np.abs(val - ref["val"])
    assert (err <= 1e-5 * np.abs(ref["val"]) + 1e-6 * scale).all(), float(np.max(err / (np.abs(ref["val"]) + scale)))
    pat = ref["pat"]
    A = sp.csr_matrix((val, pat.col, pat.rowptr), shape=(n, n)).toarray()
    if out_kind == 2:
        assert np.abs(A - A.T).max() <= 2e-6 * scale
        wg = np.sort(np.linalg.eigvalsh(0.5 * (A + A.T)))[::-1][:9]
    else:
        wg = np.sort(np.linalg.eigvals(A).real)[::-1][:9]
    wr = np.sort(np.linalg.eigvalsh(spectral.union_operator(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min,
                                                            w.e_max, w.G)[0].toarray()))[::-1][:9]
    # entries within 1e-5 relative move these eigenvalues by about 1e-4 relative
    np.testing.assert_allclose(wg[1:], wr[1:], rtol=5e-4)
    assert abs(wg[0]) <= 5e-4 * abs(wr[1])
    # the l = 1 cluster (three eigenvalues; -2 in the limit, biased low in
    # magnitude by the tuned bandwidth at k = 32) stands apart from l = 2
    assert -2.2 < wr[3] < wr[1] < -1.1 and wr[4] < -3.0
    say(f"[union] kind {out_kind}: leading eigenvalues {np.round(wg[:9], 4).tolist()}")


def test_union_rejects_invalid_rows_and_patterns(gpu_lib):
    kvb = gpu_lib
    n, k = 100, 5
    rng = np.random.default_rng(0)
    X = rng.standard_normal((n, 3)).astype(np.float32)
    idx, d2 = oracle.knn(X, k)
    d2t = torch.from_numpy(d2.astype(np.float32)).cuda()
    bad = idx.copy()
    bad[7, 3] = bad[7, 2]                       # a repeated column
    with pytest.raises(kvb.KvbError, match="column"):
        kvb.union_pattern(torch.from_numpy(bad).cuda(), d2t)
    bad = idx.copy()
    bad[9, 1] = n                               # a column outside [0, n)
    with pytest.raises(kvb.KvbError, match="column"):
        kvb.union_pattern(torch.from_numpy(bad).cuda(), d2t)
    gpat = kvb.union_pattern(torch.from_numpy(idx).cuda(), d2t)
    rho = torch.ones(n, dtype=torch.float32, device="cuda")
    broken = kvb.CsrPattern(gpat.rowptr.clone(), gpat.col, gpat.d2)
    broken.rowptr[5] = broken.rowptr[7] + 1     # rowptr decreases
    with pytest.raises(kvb.KvbError, match="rowptr"):
        kvb.tune_eps_csr(broken, rho, 1e-3, 1e1, 64)
    broken = kvb.CsrPattern(gpat.rowptr, gpat.col.clone(), gpat.d2)
    broken.col[3] = -1
    with pytest.raises(kvb.KvbError, match="col"):
        kvb.normalize_csr(broken, rho, 0.1, -0.5, 2.0)
    # the context still works afterwards
    val, P, D = kvb.normalize_csr(gpat, rho, 0.1, -0.5, 2.0)
    assert torch.isfinite(val).all()


def test_union_deterministic(gpu_lib):
    w = workloads.WORKLOADS["torus_n100k"]
    X = torch.from_numpy(workloads.torus(30000, seed=9)).cuda()
    a = gpu_lib.build_union_matrix(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
    b = gpu_lib.build_union_matrix(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
    for f in ("rowptr", "col", "d2"):
        assert torch.equal(getattr(a.pattern, f), getattr(b.pattern, f)), f
    for f in ("rho", "psi", "val", "P", "D"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f


@pytest.mark.parametrize("out_kind", [0, 1, 2])
def test_single_call_union_build_matches_separate_calls(gpu_lib, out_kind):
    """kvb_build with the union pattern enqueues the same passes without a host
    round trip (its transpose sort runs over all n k slots); only the block
    partition of the tuning sums differs, so those agree to rounding and every
    other result bit for bit."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["torus_n100k"]
    X = torch.from_numpy(workloads.torus(20000, seed=3)).cuda()
    say(f"[union] single call, kind {out_kind}")
    a = kvb.build_union_matrix(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, out_kind=out_kind)
    b = kvb.build(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, out_kind=out_kind,
                  pattern="union")
    assert torch.equal(a.pattern.rowptr, b.rowptr)
    assert torch.equal(a.pattern.col, b.col)
    np.testing.assert_allclose(b.tune_a.chi, a.tune_a.chi, rtol=1e-12)
    np.testing.assert_allclose(b.tune_b.chi, a.tune_b.chi, rtol=1e-12)
    assert a.tune_a.e_star == b.tune_a.e_star and a.tune_b.e_star == b.tune_b.e_star
    assert a.scale_b == b.scale_b
    for f in ("b", "rho", "psi", "val", "P", "D"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f


def test_union_async_builds_back_to_back(gpu_lib):
    """Enqueued union builds (no host round trip) into the same arrays give the
    synchronous result; the directed build on the same context is unchanged."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["torus_n100k"]
    X = torch.from_numpy(workloads.torus(30000, seed=4)).cuda()
    ref = kvb.build(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, pattern="union")
    out = kvb.build(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, pattern="union", sync=False)
    for _ in range(3):
        out = kvb.build(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, pattern="union",
                        sync=False, out=out)
    ta, s, tb, fb = kvb.build_info(w.G)
    nnz = int(out.rowptr[-1].item())
    assert nnz == ref.col.numel()
    assert torch.equal(out.col[:nnz], ref.col) and torch.equal(out.val[:nnz], ref.val)
    assert ta.e_star == ref.tune_a.e_star and tb.e_star == ref.tune_b.e_star
    d = kvb.build(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
    assert d.col.numel() == X.shape[0] * w.k
    assert torch.equal(d.rowptr, torch.arange(X.shape[0] + 1, device="cuda", dtype=torch.int64) * w.k)


def test_union_pattern_gmm_n8m_sampled_rows(gpu_lib):
    """The largest workload (n = 8e6, k = 64, matrix-core k-NN, as bench.py
    times it): the union rows of 48 sampled samples against the set definition
    (the row's own list plus every row that lists it), bit for bit, with each
    reverse entry's distance taken from the row that lists it."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["gmm_n8m"]
    X = workloads.make(w.name, seed=0)
    n, k = len(X), w.k
    say(f"[union] gmm_n8m: n={n} k={k}")
    idx_g, d2_g, _ = kvb.knn(torch.from_numpy(X).cuda(), k, mode="bf16", margin=w.margin)
    pat = kvb.union_pattern(idx_g, d2_g)
    idx, d2 = idx_g.cpu().numpy(), d2_g.cpu().numpy()
    rowptr = pat.rowptr.cpu().numpy()
    rng = np.random.default_rng(12)
    R = np.sort(rng.choice(n, 48, replace=False)).astype(np.int32)
    flat = idx.ravel()
    pos = np.searchsorted(R, flat)
    hit = np.nonzero((pos < len(R)) & (R[np.minimum(pos, len(R) - 1)] == flat))[0]
    src_row = hit // k
    for q, i in enumerate(R):
        own = dict(zip(idx[i].tolist(), d2[i].tolist()))
        rev = {int(s): float(d2.ravel()[p]) for s, p in zip(src_row[flat[hit] == i], hit[flat[hit] == i])}
        want = dict(rev)
        want.update(own)                                  # a pair the row stores keeps its own distance
        lo, hi = rowptr[i], rowptr[i + 1]
        cols = pat.col[lo:hi].cpu().numpy()
        dd = pat.d2[lo:hi].cpu().numpy()
        assert cols.tolist() == sorted(want), i
        assert [float(v) for v in dd] == [want[c] for c in cols.tolist()], i
    assert rowptr[-1] == pat.nnz and np.all(np.diff(rowptr) >= k)
    say(f"[union] gmm_n8m: {pat.nnz} entries ({pat.nnz / (n * k):.4f} n k), 48 rows checked")
