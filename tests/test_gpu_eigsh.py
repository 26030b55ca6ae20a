"""GPU parity of the sparse eigensolver (run on an MI355X).

The paper's use of the kernel matrix is spectral (Sections 2.2, 4 and 5):
the eigenpairs of the symmetric conjugate Lhat approximate the Kolmogorov
operator's, and on the uniform 2-sphere that operator is the Laplacian with
eigenvalues -l(l+1) of multiplicity 2l + 1 (Section 5). kvb_eigsh (Lanczos
with full reorthogonalisation) is pinned to the closed-form spectrum of the
path-graph Laplacian, then compared with a dense symmetric eigensolver and
with ARPACK on the GPU-built Lhat, and with the oracle's Lhat spectrum.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

import oracle
import workloads
from oracle import spectral
from parity import say

pytestmark = pytest.mark.gpu


def csr_to_gpu(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return (torch.from_numpy(A.indptr.astype(np.int64)).cuda(), torch.from_numpy(A.indices.astype(np.int32)).cuda(),
            torch.from_numpy(A.data.astype(np.float32)).cuda())


def test_eigsh_path_laplacian_closed_form(gpu_lib):
    """-(tridiag(-1, 2, -1)) on n = 300 vertices, relabelled by a seeded
    permutation: eigenvalues -(2 - 2 cos(pi j / (n + 1))), eigenvectors
    sin(pi j (i + 1) / (n + 1)). With ncv = n the Krylov space is complete."""
    n = 300
    perm = np.random.default_rng(1).permutation(n)
    T = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    P = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    A = P @ T @ P.T
    say("[eigsh] path Laplacian n=300")
    e = gpu_lib.eigsh(*csr_to_gpu(A), nev=10, ncv=n, tol=1e-9, seed=3)
    j = np.arange(1, 11)
    exact = -(2 - 2 * np.cos(math.pi * j / (n + 1)))
    np.testing.assert_allclose(e.values, exact, rtol=0, atol=1e-10)
    assert e.converged
    Y = e.vectors.cpu().numpy()
    for q in range(4):
        u = np.sin(math.pi * (q + 1) * (np.arange(n) + 1) / (n + 1))
        u = u / np.linalg.norm(u)
        v = np.empty(n)
        v[perm] = u                     # relabelled eigenvector
        assert abs(abs(Y[q] @ v) - 1) < 1e-9, q


def build_lhat(kvb, X, k, k0=8):
    g = kvb.build(torch.from_numpy(X).cuda(), k, k0, 2.0, -0.5, -0.5, out_kind=kvb.OUT_SYMMETRIC, pattern="union")
    return g


def test_eigsh_union_conjugate_matches_dense_and_oracle(gpu_lib):
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    n = len(X)
    g = build_lhat(kvb, X, w.k, w.k0)
    say("[eigsh] Lhat of the 2-sphere, n=2000")
    e = kvb.eigsh(g.rowptr, g.col, g.val, nev=9, ncv=300, tol=1e-9, seed=1)
    A = sp.csr_matrix((g.val.cpu().numpy().astype(np.float64), g.col.cpu().numpy(), g.rowptr.cpu().numpy()),
                      shape=(n, n))
    S = (0.5 * (A + A.T)).toarray()
    wd = np.sort(np.linalg.eigvalsh(S))[::-1][:9]
    scale = np.abs(A).max()
    # the float32 matrix is symmetric to about 1e-7 of its largest entry
    np.testing.assert_allclose(e.values, wd, rtol=0, atol=1e-6 * scale)
    Y = e.vectors.cpu().numpy()
    for q in range(9):
        r = np.linalg.norm(A @ Y[q] - e.values[q] * Y[q])
        assert r <= max(10 * e.residuals[q], 1e-6 * scale), (q, r, e.residuals[q])
        assert abs(np.linalg.norm(Y[q]) - 1) < 1e-9
    wr = np.sort(np.linalg.eigvalsh(spectral.union_operator(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min,
                                                            w.e_max, w.G)[0].toarray()))[::-1][:9]
    np.testing.assert_allclose(e.values[1:], wr[1:], rtol=5e-4)
    say(f"[eigsh] n=2000: {np.round(e.values, 4).tolist()}")


def test_eigsh_sphere_spectrum_n20000(gpu_lib):
    """At n = 20,000 (beyond a dense solver's reach in a test) the leading
    spectrum of Lhat shows the Laplacian's structure on the sphere: 0, then
    three eigenvalues (l = 1), then five (l = 2), the clusters near -2 and -6
    (about 3 apart in ratio); ARPACK on the same matrix agrees."""
    kvb = gpu_lib
    X = workloads.sphere2(20000, seed=0)
    n = len(X)
    g = build_lhat(kvb, X, 32, 8)
    say("[eigsh] Lhat of the 2-sphere, n=20000")
    e = kvb.eigsh(g.rowptr, g.col, g.val, nev=9, ncv=2048, tol=1e-8, seed=2)
    A = sp.csr_matrix((g.val.cpu().numpy().astype(np.float64), g.col.cpu().numpy(), g.rowptr.cpu().numpy()),
                      shape=(n, n))
    S = 0.5 * (A + A.T)
    # ARPACK in shift-invert mode about 0.5 (above the spectrum of Lhat <= 0)
    wa = np.sort(spla.eigsh(S.tocsc(), k=9, sigma=0.5, which="LM", tol=1e-12, v0=np.ones(n))[0])[::-1]
    np.testing.assert_allclose(e.values, wa, rtol=0, atol=1e-6)
    v = e.values
    assert e.converged, e.residuals      # 2048 steps: residuals below 1e-8 of the spectrum's width
    assert abs(v[0]) < 1e-3 * abs(v[1])
    l1, l2 = v[1:4], v[4:9]
    assert (l1.max() - l1.min()) < 0.5 * (l1.min() - l2.max())     # separated clusters
    ratio = l2.mean() / l1.mean()
    assert 2.4 < ratio < 3.4, ratio
    say(f"[eigsh] n=20000: {np.round(v, 4).tolist()}, converged {e.converged}, "
        f"max residual {e.residuals.max():.3g}, l=2/l=1 ratio {ratio:.3f}")


def test_kolmogorov_solve_matches_oracle(gpu_lib):
    """Section 3.1 on the GPU (kvb_eigsh then kvb_kolmogorov_solve) against the
    oracle's dense eigenvectors and the paper's own formula: the 2-sphere,
    g = x_1, the span of the l = 1 cluster and of the l = 1 and l = 2 clusters."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    g_build = build_lhat(kvb, X, w.k, w.k0)
    A_ref, info = spectral.union_operator(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
    S_ref = info["P"] * np.sqrt(info["D"])
    g = X[:, 0].astype(np.float64)
    g = g - (S_ref ** 2 * g).sum() / (S_ref ** 2).sum()
    e = kvb.eigsh(g_build.rowptr, g_build.col, g_build.val, nev=9, ncv=300, tol=1e-9, seed=4)
    for nvec in (4, 9):
        say(f"[kolmogorov] nvec={nvec}")
        sub = kvb.Eigs(e.values[:nvec], e.residuals[:nvec], e.vectors[:nvec].contiguous(), e.converged)
        f, gl, coef = kvb.kolmogorov_solve(sub, g_build.P, g_build.D, torch.from_numpy(g).cuda(), skip=1)
        fr, glr, gtr, lam = spectral.kolmogorov_solve(A_ref, info["P"], info["D"], g, nvec, 1)
        f, gl = f.cpu().numpy(), gl.cpu().numpy()
        assert np.linalg.norm(f - fr) < 1e-3 * np.linalg.norm(fr), np.linalg.norm(f - fr) / np.linalg.norm(fr)
        assert np.linalg.norm(gl - glr) < 1e-3 * np.linalg.norm(glr)
        # the coefficients within a cluster depend on the basis chosen in it;
        # their norm over the span does not
        assert abs(np.linalg.norm(coef) / np.linalg.norm(gtr) - 1) < 1e-3


def test_carre_du_champ_matches_oracle(gpu_lib):
    """Section 3.2 on the GPU against the oracle's term-by-term triple sum: the
    2-sphere, the null pair and the l = 1 and l = 2 clusters (nvec = 9, whole
    clusters), u = x_1 and v = x_1 or x_2. The coefficients C_ljk depend on the
    basis inside a cluster; their contraction with the projections of u and v,
    and the resulting gradient product, do not. C is compared through those
    contractions and its basis-free invariants."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    gb = build_lhat(kvb, X, w.k, w.k0)
    A_ref, info = spectral.union_operator(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
    e = kvb.eigsh(gb.rowptr, gb.col, gb.val, nev=9, ncv=300, tol=1e-9, seed=5)
    u = X[:, 0].astype(np.float64)
    for s_ in (0, 1):
        v = X[:, s_].astype(np.float64)
        say(f"[cdc] u = x_1, v = x_{s_ + 1}")
        gr, C = kvb.carre_du_champ(e, gb.P, gb.D, torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(),
                                   tensor=True)
        gr_ref, C_ref, lam = spectral.carre_du_champ(A_ref, info["P"], info["D"], u, v, 9)
        gr = gr.cpu().numpy()
        assert np.linalg.norm(gr - gr_ref) < 2e-3 * np.linalg.norm(gr_ref), np.linalg.norm(gr - gr_ref) / np.linalg.norm(gr_ref)
        C = C.cpu().numpy()
        # invariants under rotations inside clusters: the Frobenius norm and C_ll0 sums
        assert abs(np.linalg.norm(C) / np.linalg.norm(C_ref) - 1) < 1e-3
        np.testing.assert_allclose(C, np.transpose(C, (1, 2, 0)), atol=1e-12 * np.abs(C).max())
        np.testing.assert_allclose(np.abs(C[:, :, 0]), np.abs(C_ref[0, 0, 0]) * np.eye(9), atol=1e-4 * abs(C_ref[0, 0, 0]))


def test_advection_step_matches_oracle(gpu_lib):
    """One step of the density-evolution example (Section 5.3) on the GPU
    (build, eigsh, Kolmogorov solve, Carre du champ per coordinate, particle
    update) against the oracle's composition, on the paper's validation case
    (N(0, I_2), g = x_1 - mean, u = 0). The eigenpair count is placed at a gap
    of the oracle's spectrum near 3 ln n, so both sides span the same space."""
    kvb = gpu_lib
    X = workloads.gaussian_iid(2000, 2, seed=3)
    n = len(X)
    A_ref, info = spectral.union_operator(X, 64, 8, 2.0, -0.5, -0.5)
    w = np.sort(np.linalg.eigvalsh(A_ref.toarray()))[::-1]
    cand = np.arange(20, 29)
    nvec = int(cand[np.argmax((w[cand - 1] - w[cand]) / np.abs(w[cand]))])
    say(f"[advect] n={n}, {nvec} eigenpairs")
    g = X[:, 0].astype(np.float64) - X[:, 0].mean()
    dt = 0.1
    Xd = torch.from_numpy(X).cuda()
    st = kvb.advection_step(Xd, torch.from_numpy(g).cuda(), dt, ell=nvec - 1, k=64, k0=8, ncv=1024, seed=6)
    Xn_ref, f_ref, grad_ref = spectral.advection_step(X, g, dt, nvec, 64, 8)
    say(f"[advect] GPU eigenvalues {np.round(st.eigs.values, 4).tolist()}, max residual {st.eigs.residuals.max():.3g}")
    say(f"[advect] oracle eigenvalues {np.round(w[:nvec], 4).tolist()}")
    f = st.f.cpu().numpy()
    grad = st.grad.cpu().numpy()
    # the Gaussian's leading modes live in its tails and sit close together,
    # so the float32 matrix moves the span slightly (3.5e-3 in f here)
    assert np.linalg.norm(f - f_ref) < 1e-2 * np.linalg.norm(f_ref), np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref)
    assert np.linalg.norm(grad - grad_ref) < 2e-2 * np.linalg.norm(grad_ref), \
        np.linalg.norm(grad - grad_ref) / np.linalg.norm(grad_ref)
    vel = (st.X.cpu().numpy().astype(np.float64) - X) / dt
    assert abs(vel[:, 0].mean() - 1) < 0.12 and abs(vel[:, 1].mean()) < 0.05
    # the diffusion term with caller-supplied draws
    noise = np.random.default_rng(9).standard_normal((n, 2))
    st2 = kvb.advection_step(Xd, torch.from_numpy(g).cuda(), dt, ell=nvec - 1, k=64, k0=8, ncv=1024, seed=6,
                             sigma=1.0, noise=torch.from_numpy(noise).cuda())
    diff = st2.X.cpu().numpy().astype(np.float64) - st.X.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(diff, np.sqrt(dt) * noise, atol=1e-5)
    say(f"[advect] mean velocity {vel.mean(axis=0).round(4).tolist()}")


def test_spectral_entry_points_reject_bad_arguments(gpu_lib):
    """Argument errors come back as KVB_E_INVALID with a message, a short
    Lanczos run reports KVB_W_NOT_CONVERGED (results still returned), and the
    context keeps working."""
    kvb = gpu_lib
    n = 300
    T = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    rp, cl, vl = csr_to_gpu(T)
    with pytest.raises(kvb.KvbError, match="ncv"):
        kvb.eigsh(rp, cl, vl, nev=10, ncv=5)
    with pytest.raises(kvb.KvbError, match="ncv"):
        kvb.eigsh(rp, cl, vl, nev=4, ncv=n + 1)
    bad = cl.clone()
    bad[7] = n                                    # a column outside [0, n)
    with pytest.raises(kvb.KvbError, match="col"):
        kvb.eigsh(rp, bad, vl, nev=2, ncv=8)
    e = kvb.eigsh(rp, cl, vl, nev=4, ncv=8, tol=1e-12)
    assert not e.converged and np.isfinite(e.values).all() and (e.residuals > 0).all()
    full = kvb.eigsh(rp, cl, vl, nev=4, ncv=n, tol=1e-9)
    assert full.converged
    P = torch.ones(n, dtype=torch.float64, device="cuda")
    D = torch.ones(n, dtype=torch.float64, device="cuda")
    g = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(kvb.KvbError, match="skip"):
        kvb.kolmogorov_solve(full, P, D, g, skip=4)
    zero = kvb.Eigs(np.array([0.0, -1.0]), full.residuals[:2], full.vectors[:2].contiguous(), True)
    with pytest.raises(kvb.KvbError, match="zero"):
        kvb.kolmogorov_solve(zero, P, D, g, skip=0)
    f, gl, coef = kvb.kolmogorov_solve(full, P, D, g, skip=0)
    assert torch.isfinite(f).all()


def test_eigsh_breakdown_on_an_invariant_subspace(gpu_lib):
    """The zero matrix (zeros stored on the diagonal) maps the start vector to
    exactly zero, so beta_0 = 0: the Krylov space is the start vector's span,
    Lanczos stops after one step, and its one Ritz pair (0, v_0) is exact
    (Golub and Van Loan, Section 10.1: a zero beta_j means the Krylov space is
    invariant). Asking for more pairs than that space holds is an error, and
    the context keeps working afterwards."""
    kvb = gpu_lib
    n = 64
    Z = sp.csr_matrix((np.zeros(n), np.arange(n), np.arange(n + 1)), shape=(n, n))
    rp, cl, vl = csr_to_gpu(Z)
    e = kvb.eigsh(rp, cl, vl, nev=1, ncv=16, tol=1e-12, seed=9)
    say("breakdown", f"value {e.values[0]!r}, residual {e.residuals[0]!r}")
    assert e.converged and e.values[0] == 0.0 and e.residuals[0] == 0.0
    v = e.vectors[0].cpu().numpy()
    assert np.isfinite(v).all() and abs(np.linalg.norm(v) - 1.0) < 1e-12
    with pytest.raises(kvb.KvbError, match="closed"):
        kvb.eigsh(rp, cl, vl, nev=2, ncv=16, seed=9)
    T = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    full = kvb.eigsh(*csr_to_gpu(T), nev=3, ncv=n, tol=1e-9, seed=9)
    exact = -2 + 2 * np.cos(np.pi * np.arange(1, 4) / (n + 1))
    assert full.converged and np.max(np.abs(full.values - exact)) < 1e-5


def test_eigsh_rejects_a_non_finite_matrix(gpu_lib):
    """A NaN or infinite stored value makes every Lanczos coefficient
    non-finite; kvb_eigsh then fails with KVB_E_INVALID instead of reading a
    NaN beta as a breakdown and returning NaN eigenvalues as converged. The
    context keeps working afterwards."""
    kvb = gpu_lib
    n = 64
    T = sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1], format="csr")
    for bad in (np.nan, np.inf):
        B = T.copy()
        B.data[5] = bad
        say(f"[eigsh] non-finite value {bad}")
        with pytest.raises(kvb.KvbError, match="non-finite") as e:
            kvb.eigsh(*csr_to_gpu(B), nev=1, ncv=8, seed=4)
        assert e.value.code == kvb.E_INVALID
    ok = kvb.eigsh(*csr_to_gpu(T), nev=2, ncv=n, tol=1e-9, seed=4)
    assert ok.converged and np.isfinite(ok.values).all()
