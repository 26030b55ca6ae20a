"""Spectral checks of the FP64 oracle (test infrastructure only).

The paper's kernel matrices are symmetric: its brute-force construction sets
K_ij and K_ji together (Section 4, Algorithm 1). A directed k-NN pattern is not
symmetric, so for spectral checks the oracle also runs every pass on the union
pattern E u E^T, where the symmetric conjugate S^{-1} Kt S^{-1} - P^{-2}
(Section 2.2, symmetric discrete Kolmogorov operator) is an exactly symmetric
matrix similar to the discrete Kolmogorov matrix L. Its eigenvalues approximate
those of the Kolmogorov operator; on the uniform unit 2-sphere the operator is
the Laplace-Beltrami operator (Section 5, spherical manifold) whose spectrum is
-l(l+1) with multiplicity 2l+1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import (Pattern, adhoc_bandwidth, chi, density, grid_scale, knn, normalize,
               SYMMETRIC, GENERATOR)


def union_pattern(idx: np.ndarray, d2: np.ndarray) -> Pattern:
    """E u E^T of the directed k-NN pattern, with each entry's squared distance.
    A pair stored in both directions carries the same exact distance (the
    oracle computes D2 symmetrically), so duplicates are merged by max."""
    n, k = idx.shape
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = idx.ravel().astype(np.int64)
    dd = d2.ravel()
    r2 = np.concatenate([rows, cols])
    c2 = np.concatenate([cols, rows])
    v2 = np.concatenate([dd, dd])
    order = np.lexsort((c2, r2))
    r2, c2, v2 = r2[order], c2[order], v2[order]
    keep = np.ones(len(r2), dtype=bool)
    keep[1:] = (r2[1:] != r2[:-1]) | (c2[1:] != c2[:-1])
    r2, c2, v2 = r2[keep], c2[keep], v2[keep]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r2 + 1, 1)
    rowptr = np.cumsum(rowptr)
    return Pattern(rowptr, c2.astype(np.int32), np.ascontiguousarray(v2, dtype=np.float64))


def union_operator(X: np.ndarray, k: int, k0: int, d: float, alpha: float, beta: float,
                   e_min: float = 1e-3, e_max: float = 1e1, G: int = 64,
                   out_kind: int = SYMMETRIC):
    """Run the full oracle pipeline on the union pattern; return the sparse
    matrix (CSR, scipy) of the requested kind, plus the diagonal factors."""
    idx, d2 = knn(X, k)
    pat = union_pattern(idx, d2)
    b = adhoc_bandwidth(d2, k0)
    ta = chi(pat, b, e_min, e_max, G)
    psi, rho = density(pat, b, ta.e_star, d, beta)
    s = grid_scale(b, rho)
    tb = chi(pat, rho, e_min * s, e_max * s, G)
    val, q, P, D = normalize(pat, rho, tb.e_star, alpha, d, out_kind)
    n = pat.n
    A = sp.csr_matrix((val, pat.col, pat.rowptr), shape=(n, n))
    return A, dict(P=P, D=D, psi=psi, rho=rho, e_a=ta.e_star, e_b=tb.e_star,
                   tune_a=ta, tune_b=tb, pattern=pat)


def leading_eigenvalues(A, count: int) -> np.ndarray:
    """The `count` eigenvalues of the symmetric matrix A nearest zero from below
    (dense symmetric eigensolver; meant for n of a few thousand)."""
    w = np.linalg.eigvalsh(A.toarray())
    return np.sort(w)[::-1][:count]


def kolmogorov_solve(A, P: np.ndarray, D: np.ndarray, g: np.ndarray, nvec: int, skip: int = 1):
    """The least-squares solution of the discrete Kolmogorov problem L f = g in
    the span of the leading eigenvectors of L (Section 3.1), from the symmetric
    conjugate A = Lhat (dense symmetric eigensolver): with S = P D^{1/2},
    the eigenvectors of L are phi_j = S^{-1} phihat_j, phihat_j the eigenvectors
    of Lhat scaled to phihat^T phihat = n, so that <phi_i, phi_j>_S =
    phi_i^T S^2 phi_j / n = delta_ij; then g~ = Q^T S^2 g / n, f = Q Lambda^{-1} g~
    and the projection of g is Q g~. The first `skip` (null) pairs are left out.
    Returns (f, g projected, g~, eigenvalues used)."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    n = len(Ad)
    w, Y = np.linalg.eigh(0.5 * (Ad + Ad.T))
    order = np.argsort(w)[::-1][:nvec]
    lam = w[order][skip:]
    S = P * np.sqrt(D)
    Q = (np.sqrt(n) * Y[:, order][:, skip:]) / S[:, None]
    gt = Q.T @ (S ** 2 * g) / n
    f = Q @ (gt / lam)
    return f, Q @ gt, gt, lam


def carre_du_champ(A, P: np.ndarray, D: np.ndarray, u: np.ndarray, v: np.ndarray, nvec: int):
    """grad u . grad v at the samples by the spectral Carre du champ formula of
    Section 3.2, written out term by term: the leading nvec eigenpairs of L
    (null pair included; phi_j = S^{-1} phihat_j with phihat^T phihat = n),
    C_ljk = <phi_l, phi_j * phi_k>_S, u~ = <u, phi>_S, v~ = <v, phi>_S and
    grad u . grad v = sum_{l,j,k} u~_j v~_k C_ljk (lambda_l - lambda_j - lambda_k) / 2 phi_l.
    Returns (the gradient product, C, eigenvalues)."""
    Ad = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    n = len(Ad)
    w, Y = np.linalg.eigh(0.5 * (Ad + Ad.T))
    order = np.argsort(w)[::-1][:nvec]
    lam = w[order]
    S = P * np.sqrt(D)
    Phi = (np.sqrt(n) * Y[:, order]) / S[:, None]
    S2 = S ** 2
    C = np.einsum("r,rl,rj,rk->ljk", S2, Phi, Phi, Phi) / n
    ut = Phi.T @ (S2 * u) / n
    vt = Phi.T @ (S2 * v) / n
    fac = lam[:, None, None] - lam[None, :, None] - lam[None, None, :]
    coef = np.einsum("j,k,ljk,ljk->l", ut, vt, C, fac) / 2
    return Phi @ coef, C, lam


def advection_step(X: np.ndarray, g: np.ndarray, dt: float, nvec: int, k: int, k0: int,
                   sigma: float = 0.0, noise: np.ndarray | None = None):
    """One explicit step of the density-evolution example (Section 5.3) with
    u = 0: the operator with c = 1 on the union pattern (alpha = -d/4,
    beta = -1/2, d = m), f solving L f = g in the span of the leading nvec - 1
    nonzero eigenvectors, grad f by the Carre du champ formula with v = x_s,
    x' = x - dt grad f + sqrt(dt) sigma w. Returns (x', f, grad f [m, n])."""
    n, m = X.shape
    A, info = union_operator(X, k, k0, float(m), -m / 4.0, -0.5)
    f, _, _, _ = kolmogorov_solve(A, info["P"], info["D"], g, nvec, 1)
    grad = np.array([carre_du_champ(A, info["P"], info["D"], f, X[:, s].astype(np.float64), nvec)[0]
                     for s in range(m)])
    Xn = X.astype(np.float64) - dt * grad.T
    if noise is not None:
        Xn = Xn + np.sqrt(dt) * sigma * noise
    return Xn, f, grad
