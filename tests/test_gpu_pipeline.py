"""GPU kernel-matrix parity against the FP64 oracle (run on an MI355X).

The whole build (k-NN, ad-hoc bandwidth, e tuning on the density kernel,
density and rho, e tuning on the operator kernel, q / Kt / D, CSR) runs through
the C ABI and is compared step by step with the oracle run on the same seeded
samples (Sections 2.1-2.3 and 4).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import check_entries, check_knn_rows, knn_reference, say

pytestmark = pytest.mark.gpu


def gpu_build(kvb, X, w, out_kind=0, mode="f32", entry="calls"):
    """The build through the separate entry points (kvb_knn, kvb_bandwidth,
    kvb_tune_eps, kvb_grid_scale, kvb_assemble_csr) or through the single call
    kvb_build."""
    Xd = torch.from_numpy(X).cuda()
    fn = kvb.build_kernel_matrix if entry == "calls" else kvb.build
    r = fn(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G,
           mode=mode, margin=w.margin, out_kind=out_kind)
    torch.cuda.synchronize()
    return r


def near_tie(slope):
    s = np.sort(slope)
    return (s[-1] - s[-2]) <= 1e-5 * abs(s[-1])


def compare_pipeline(kvb, name, X, w, mode="f32", entry="calls"):
    say(f"[pipeline] {name}: n={len(X)} m={X.shape[1]} k={w.k} mode={mode} entry={entry}")
    g = gpu_build(kvb, X, w, mode=mode, entry=entry)
    ref = oracle.pipeline(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
    n, k = len(X), w.k
    # k-NN
    ri, rd = knn_reference(X, k)
    ties = check_knn_rows(g.idx.cpu().numpy(), g.d2.cpu().numpy(), ri, rd, k, np.arange(n))
    assert ties == 0, "the workloads have no near-tie rows at these seeds"
    # ad-hoc bandwidth
    b = g.b.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(b, ref.b, rtol=2e-6)
    # tuning, density stage: same grid point (unless the oracle's top slopes tie)
    np.testing.assert_allclose(g.tune_a.chi, ref.tune_a.chi, rtol=2e-5)
    assert not near_tie(ref.tune_a.slope), "the oracle's two best slopes tie: pick another seed"
    assert g.tune_a.e_star == pytest.approx(ref.tune_a.e_star, rel=1e-13)
    assert g.tune_a.dim == pytest.approx(ref.tune_a.dim, rel=1e-3)
    e_a = g.tune_a.e_star
    # density and rho
    psi = g.psi.cpu().numpy().astype(np.float64)
    rho = g.rho.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(psi, ref.psi, rtol=5e-6)
    np.testing.assert_allclose(rho, ref.rho, rtol=5e-6)
    assert g.scale_b == ref.scale_b
    np.testing.assert_allclose(g.tune_b.chi, ref.tune_b.chi, rtol=2e-5)
    assert g.tune_b.e_star == pytest.approx(ref.tune_b.e_star, rel=1e-13)
    e_b = ref.tune_b.e_star
    # CSR
    rowptr = g.rowptr.cpu().numpy()
    col = g.col.cpu().numpy()
    val = g.val.cpu().numpy().astype(np.float64)
    assert (rowptr == np.arange(n + 1) * k).all()
    np.testing.assert_array_equal(col, ref.col)
    # exponent of every entry from the oracle's own values
    pat = oracle.Pattern.from_knn(ref.idx, ref.d2)
    xs = pat.dist2 / (e_b * ref.rho[np.repeat(np.arange(n), k)] * ref.rho[pat.col])
    _, x = oracle.sort_rows_by_col(pat.col, xs, k)   # exponents in CSR order
    rowmax = np.repeat(ref.val.reshape(n, k).max(axis=1), k)
    worst = check_entries(val, ref.val, x, rowmax, f"{name} Markov entries")
    np.testing.assert_allclose(g.P.cpu().numpy(), ref.P, rtol=5e-6)     # P = rho / 2 of the float32 rho
    np.testing.assert_allclose(g.D.cpu().numpy(), ref.D, rtol=2e-5)
    rs = val.reshape(n, k).sum(axis=1)
    assert np.abs(rs - 1).max() < 2e-6
    say(f"[pipeline] {name}: ok, e_A={e_a:.6g} e_B={e_b:.6g} dimA={g.tune_a.dim:.4f} "
        f"dimB={g.tune_b.dim:.4f} worst entry rel err {worst:.3g}")
    return g, ref


def test_pipeline_sphere_n2000(gpu_lib):
    w = workloads.WORKLOADS["sphere2_n2000"]
    compare_pipeline(gpu_lib, "sphere2_n2000", workloads.make(w.name, seed=0), w)


def test_pipeline_sphere_other_seeds(gpu_lib):
    w = workloads.WORKLOADS["sphere2_n2000"]
    for seed in (1, 2):
        compare_pipeline(gpu_lib, f"sphere2_n2000_seed{seed}", workloads.make(w.name, seed=seed), w)


def test_pipeline_torus_n100k_full(gpu_lib):
    """Full-size measured workload, every row and entry compared."""
    w = workloads.WORKLOADS["torus_n100k"]
    compare_pipeline(gpu_lib, "torus_n100k", workloads.make(w.name, seed=0), w)


def test_pipeline_torus_n100k_single_call(gpu_lib):
    """The entry point the benchmark times (kvb_build, one call, intermediate
    values on the device) at the torus workload's full size, every row and
    entry against the oracle."""
    w = workloads.WORKLOADS["torus_n100k"]
    compare_pipeline(gpu_lib, "torus_n100k", workloads.make(w.name, seed=0), w, entry="build")


def test_pipeline_k128_lifted_sphere(gpu_lib):
    """The lifted 3-sphere recipe (m = 128, k = 128, d = 3) at n = 20000 through
    kvb_build with BF16 matrix-core tiles: the k > 64 forms of the density,
    tuning, q and assembly passes (two row slices per lane) against the oracle."""
    import dataclasses
    w = dataclasses.replace(workloads.WORKLOADS["sphere3_n4m"], n=20000, mode="bf16")
    compare_pipeline(gpu_lib, "sphere3_n20k_k128", workloads.make(w.name, seed=0, n=w.n), w, mode="bf16",
                     entry="build")


@pytest.mark.parametrize("entry", ["calls", "build"])
def test_pipeline_mixture_k64_curve_rows(gpu_lib, entry):
    """The mixture recipe at its own m = 16, k = 64 (n = 20000), every row and
    entry against the oracle. Through the single call the passes run on the
    curve-ordered rows (the row pass, the row sums of 64 rows per wavefront,
    the assembly's 32-bit-key row sort writing rows by sample id); through the
    separate entry points they run in sample order."""
    import dataclasses
    w = dataclasses.replace(workloads.WORKLOADS["gmm_n8m"], n=20000, mode="f32")
    compare_pipeline(gpu_lib, f"gmm_n20000_k64_{entry}", workloads.make(w.name, seed=3, n=w.n), w, mode="f32",
                     entry=entry)


@pytest.mark.parametrize("entry", ["calls", "build"])
def test_pipeline_k200_mixture(gpu_lib, entry):
    """k = 200 (margin 56, k + margin = 256: the largest list) on the mixture
    recipe at n = 5000: the widest form of the passes (four row slices per
    lane) against the oracle, through both entry forms."""
    import dataclasses
    w = dataclasses.replace(workloads.WORKLOADS["gmm_n8m"], n=5000, k=200, margin=56, mode="f32")
    compare_pipeline(gpu_lib, f"gmm_n5000_k200_{entry}", workloads.make(w.name, seed=1, n=w.n), w, mode="f32",
                     entry=entry)


@pytest.mark.parametrize("out_kind", [1, 2])
@pytest.mark.parametrize("k", [128, 200])
def test_output_kinds_wide_rows(gpu_lib, out_kind, k):
    """The generator and the symmetric conjugate at k > 64."""
    import dataclasses
    w = dataclasses.replace(workloads.WORKLOADS["gmm_n8m"], n=3000, k=k, margin=256 - k, mode="f32")
    X = workloads.make(w.name, seed=2, n=w.n)
    say(f"[pipeline] output kind {out_kind}, k={k}")
    g = gpu_build(gpu_lib, X, w, out_kind=out_kind, entry="build")
    ref = oracle.pipeline(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, out_kind=out_kind)
    assert g.tune_b.e_star == pytest.approx(ref.tune_b.e_star, rel=1e-13)
    val = g.val.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(g.col.cpu().numpy(), ref.col)
    scale = np.abs(ref.val).max()
    err = np.abs(val - ref.val)
    assert (err <= 1e-5 * np.abs(ref.val) + 1e-6 * scale).all(), float(np.max(err / (np.abs(ref.val) + scale)))


@pytest.mark.parametrize("out_kind", [1, 2])
def test_output_kinds(gpu_lib, out_kind):
    from paper_2104_15124_amd import kvb
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    say(f"[pipeline] output kind {out_kind}")
    g = gpu_build(kvb, X, w, out_kind=out_kind)
    ref = oracle.pipeline(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, out_kind=out_kind)
    n, k = len(X), w.k
    val = g.val.cpu().numpy().astype(np.float64)
    np.testing.assert_array_equal(g.col.cpu().numpy(), ref.col)
    scale = np.abs(ref.val).max()
    # the diagonal entries carry the -1 (or -1/P^2) shift; compare with an
    # absolute floor relative to the largest entry of the matrix
    err = np.abs(val - ref.val)
    assert (err <= 1e-5 * np.abs(ref.val) + 1e-6 * scale).all(), float(np.max(err / (np.abs(ref.val) + scale)))
    if out_kind == 1:
        rs = val.reshape(n, k).sum(axis=1)
        assert np.abs(rs).max() <= 1e-5 * scale


def test_pipeline_deterministic(gpu_lib):
    w = workloads.WORKLOADS["torus_n100k"]
    X = workloads.torus(30000, seed=9)
    a = gpu_build(gpu_lib, X, w)
    b = gpu_build(gpu_lib, X, w)
    for f in ("idx", "d2", "b", "rho", "psi", "rowptr", "col", "val", "P", "D"):
        assert torch.equal(getattr(a, f), getattr(b, f)), f
    assert (a.tune_a.chi == b.tune_a.chi).all() and (a.tune_b.chi == b.tune_b.chi).all()


def test_pass_argument_errors(gpu_lib):
    from paper_2104_15124_amd import kvb
    idx = torch.zeros((10, 4), dtype=torch.int32, device="cuda")
    d2 = torch.zeros((10, 4), device="cuda")
    rho = torch.ones(10, device="cuda")
    with pytest.raises(kvb.KvbError) as e:
        kvb.bandwidth_adhoc(d2, 4)               # k0 must be < k
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.tune_eps(idx, d2, rho, 1.0, 0.5, 64)  # e_min > e_max
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.tune_eps(idx, d2, rho, 1e-3, 1.0, 2)  # G < 3
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.assemble_csr(idx, d2, rho, -1.0, -0.5, 2.0)
    assert e.value.code == kvb.E_INVALID


@pytest.mark.parametrize("out_kind", [0, 1, 2])
def test_single_call_build_matches_separate_calls(gpu_lib, out_kind):
    """kvb_build keeps every intermediate on the device; its results must equal
    the separate entry points' bit for bit."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make("sphere2_n2000", seed=3)
    Xd = torch.from_numpy(X).cuda()
    a = kvb.build_kernel_matrix(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G,
                                mode="f32", margin=w.margin, out_kind=out_kind)
    b = kvb.build(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G,
                  mode="f32", margin=w.margin, out_kind=out_kind)
    torch.cuda.synchronize()
    for name in ("idx", "d2", "b", "rho", "psi", "rowptr", "col", "val", "P", "D"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
    assert a.scale_b == b.scale_b
    for ta, tb in ((a.tune_a, b.tune_a), (a.tune_b, b.tune_b)):
        assert (ta.chi == tb.chi).all() and ta.e_star == tb.e_star and ta.dim == tb.dim and ta.edge == tb.edge


def test_async_builds_back_to_back(gpu_lib):
    """Builds enqueued without a host copy (info_host NULL) run back to back on
    the stream, reuse their outputs, and report through kvb_build_info exactly
    what a synchronous build reports."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make("sphere2_n2000", seed=4)
    Xd = torch.from_numpy(X).cuda()
    ctx = kvb.Context()
    with pytest.raises(kvb.KvbError) as e:
        kvb.build_info(w.G, ctx)      # no build yet
    assert e.value.code == kvb.E_INVALID
    ref = kvb.build(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, mode="f32",
                    margin=w.margin, ctx=ctx)
    out = None
    for _ in range(3):
        out = kvb.build(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, mode="f32",
                        margin=w.margin, ctx=ctx, out=out, sync=False)
    assert out.tune_a is None
    ta, s, tb, fb = kvb.build_info(w.G, ctx)
    for name in ("idx", "d2", "b", "rho", "rowptr", "col", "val", "P", "D"):
        assert torch.equal(getattr(ref, name), getattr(out, name)), name
    assert s == ref.scale_b and fb == kvb.knn_fallback_rows(ctx)
    for x, y in ((ta, ref.tune_a), (tb, ref.tune_b)):
        assert (x.chi == y.chi).all() and x.e_star == y.e_star and x.dim == y.dim and x.edge == y.edge
    ctx.close()
