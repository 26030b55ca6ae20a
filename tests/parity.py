"""Comparison helpers for GPU-vs-oracle parity tests.

Tolerances (derived in the design doc, restated here):
  * k-NN index sets: bit-exact on every row whose float64 gap between the
    (k-1)-th and k-th nearest other sample exceeds 1e-12 relative; on rows
    below that gap either tied sample is correct, so those rows are checked
    by distances instead.
  * squared distances: float32 results of compensated float32 arithmetic (or
    float64 rounded once); |d2 - ref| <= 2^-21 ref (8 units in the last place).
  * kernel-matrix entries: |M - ref| <= 1e-5 ref for entries whose exponent
    x = D2/(e rho_i rho_j) is at most 25, and <= 1e-5 ref + 1e-12 max_row(ref)
    beyond; the error model is (error of x) * x with error of x a few float32
    units from d2, rho and e.
"""
from __future__ import annotations

import sys
import numpy as np

import oracle

U32 = 2.0 ** -24
D2_RTOL = 2.0 ** -21


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def knn_reference(X: np.ndarray, k: int, rows: np.ndarray | None = None):
    """Oracle k-NN with one extra neighbour (for the tie gap)."""
    n = len(X)
    kq = min(k + 1, n)
    if rows is None:
        idx, d2 = oracle.knn(X, kq)
    else:
        idx, d2 = oracle.knn_sampled(X, kq, rows)
    return idx, d2


def check_knn_rows(g_idx: np.ndarray, g_d2: np.ndarray, ref_idx: np.ndarray, ref_d2: np.ndarray, k: int,
                   row_ids: np.ndarray):
    """Compare GPU rows with oracle rows computed with k+1 neighbours."""
    n_rows = len(row_ids)
    assert g_idx.shape == (n_rows, k)
    assert (g_idx[:, 0] == row_ids).all(), "self must come first"
    assert (g_d2[:, 0] == 0).all()
    assert (np.diff(g_d2, axis=1) >= 0).all(), "distances must ascend within a row"
    kk = k - 1
    if ref_idx.shape[1] > k:
        dk = ref_d2[:, k - 1]
        dnext = ref_d2[:, k]
        gap = (dnext - dk) / np.maximum(dk, 1e-300)
        clear = gap > 1e-12
    else:
        clear = np.ones(n_rows, dtype=bool)
    gs = np.sort(g_idx[:, 1:], axis=1)
    rs = np.sort(ref_idx[:, 1:k], axis=1)
    same = (gs == rs).all(axis=1)
    bad = np.nonzero(clear & ~same)[0]
    assert len(bad) == 0, f"{len(bad)} rows with a clear gap differ, e.g. row {row_ids[bad[0]]}: " \
                          f"gpu {g_idx[bad[0]].tolist()} ref {ref_idx[bad[0], :k].tolist()}"
    # distances, position by position after sorting both rows
    gd = np.sort(g_d2[:, 1:].astype(np.float64), axis=1)
    rd = ref_d2[:, 1:k]
    err = np.abs(gd - rd)
    assert (err <= D2_RTOL * rd + 1e-30).all(), f"max d2 rel err {np.max(err / np.maximum(rd, 1e-30))}"
    if kk > 0:
        # distinct indices, none equal to the row itself
        srt = np.sort(g_idx, axis=1)
        assert (np.diff(srt, axis=1) > 0).all(), "duplicate neighbour"
    return int((~clear).sum())


def check_entries(val: np.ndarray, ref: np.ndarray, x: np.ndarray, rowmax: np.ndarray, what: str):
    """Kernel-matrix entry tolerance (see module docstring)."""
    tol = 1e-5 * np.abs(ref) + np.where(x > 25.0, 1e-12 * rowmax, 0.0)
    err = np.abs(val - ref)
    worst = np.argmax(err - tol)
    assert (err <= tol).all(), f"{what}: entry {worst} gpu {val[worst]!r} ref {ref[worst]!r} x {x[worst]:.3g}"
    big = x <= 25.0
    return float(np.max(err[big] / np.abs(ref[big]))) if big.any() else 0.0
