"""FP64 CPU oracle for the self-tuning variable-bandwidth kernel matrix.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this package; the HIP library never does. The
arithmetic lives in ``kvb_oracle.c`` (plain C, double precision, OpenMP over
rows); this module only marshals numpy arrays through ctypes and chains the
steps in the paper's order (Section 4, steps 1-2):

  k-NN -> ad-hoc bandwidth b -> tune e on the density kernel -> density psi,
  rho = 2 psi^beta -> tune e on the operator kernel -> q, Kt, D -> Markov
  matrix M (or L, or its symmetric conjugate) as CSR.

Conventions (the readings of the paper this oracle takes):
  * e denotes the paper's epsilon^2; one kernel exp(-D2/(e rho_i rho_j)) serves
    both stages, with rho = b (density) and rho = 2 psi^beta (operator).
  * Row i of the k-NN pattern is i itself followed by the k-1 nearest j != i in
    (D2, j) order; all k entries are kept unless a pattern is truncated
    explicitly (``truncate``: Algorithm 1's sparsity tolerance).
  * The tuning grid is e_g = e_min (e_max/e_min)^{g/(G-1)}; the slope is the
    forward difference of ln chi over ln e; the optimum is its first maximum.
  * The operator-stage grid is rescaled by a power of two,
    s = 2^round(log2(gm(b^2)/gm(rho^2))), which leaves M and L unchanged.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_lib = None

_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_c_i64 = ctypes.c_int64
_c_i32 = ctypes.c_int32
_c_f64 = ctypes.c_double

MARKOV, GENERATOR, SYMMETRIC = 0, 1, 2


def lib():
    """Load (building on first use if absent or stale) the oracle library."""
    global _lib
    if _lib is not None:
        return _lib
    path = _build.build(force=False)
    L = ctypes.CDLL(path)
    L.oracle_num_threads.restype = ctypes.c_int
    L.oracle_knn_rows.argtypes = [_f32p, _c_i64, _c_i32, _c_i32, _c_i64, _c_i64, _i32p, _f64p]
    L.oracle_knn_rows.restype = ctypes.c_int
    L.oracle_knn_list.argtypes = [_f32p, _c_i64, _c_i32, _c_i32, _i64p, _c_i64, _i32p, _f64p]
    L.oracle_knn_list.restype = ctypes.c_int
    L.oracle_adhoc_bandwidth.argtypes = [_f64p, _c_i64, _c_i32, _c_i32, _f64p]
    L.oracle_adhoc_bandwidth.restype = ctypes.c_int
    L.oracle_chi.argtypes = [_i64p, _i32p, _f64p, _f64p, _c_i64, _c_f64, _c_f64, _c_i32,
                             _f64p, _f64p, _f64p, ctypes.POINTER(_c_i32),
                             ctypes.POINTER(_c_f64), ctypes.POINTER(_c_f64)]
    L.oracle_chi.restype = ctypes.c_int
    L.oracle_density.argtypes = [_i64p, _i32p, _f64p, _f64p, _c_i64, _c_f64, _c_f64, _c_f64,
                                 _f64p, _f64p]
    L.oracle_density.restype = ctypes.c_int
    L.oracle_grid_scale.argtypes = [_f64p, _f64p, _c_i64]
    L.oracle_grid_scale.restype = ctypes.c_double
    L.oracle_normalize.argtypes = [_i64p, _i32p, _f64p, _f64p, _c_i64, _c_f64, _c_f64, _c_f64,
                                   _c_i32, _f64p, _f64p, _f64p, _f64p]
    L.oracle_normalize.restype = ctypes.c_int
    L.oracle_sort_rows_by_col.argtypes = [_c_i64, _c_i32, _i32p, _f64p]
    L.oracle_sort_rows_by_col.restype = ctypes.c_int
    L.oracle_truncate.argtypes = [_i64p, _i32p, _f64p, _f64p, _c_i64, _c_f64, _c_f64, _i64p, _i32p, _f64p,
                                  ctypes.POINTER(_c_i64)]
    L.oracle_truncate.restype = ctypes.c_int
    _lib = L
    return L


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")
    return rc


# ------------------------------------------------------------------ steps
def knn(X: np.ndarray, k: int, rows: np.ndarray | slice | None = None):
    """Exact k-NN (self first, then (D2, j) order). Returns idx int32 [r, k],
    d2 float64 [r, k] for all rows, or for the contiguous row range `rows`."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, m = X.shape
    if rows is None:
        b, e = 0, n
    else:
        b, e = rows.start or 0, rows.stop if rows.stop is not None else n
    idx = np.empty((e - b, k), dtype=np.int32)
    d2 = np.empty((e - b, k), dtype=np.float64)
    _check(lib().oracle_knn_rows(X, n, m, k, b, e, idx, d2), "knn")
    return idx, d2


def knn_sampled(X: np.ndarray, k: int, rows: np.ndarray):
    """Exact k-NN of the listed rows (any order) against all samples, one row
    per thread."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out_i = np.empty((len(rows), k), dtype=np.int32)
    out_d = np.empty((len(rows), k), dtype=np.float64)
    n, m = X.shape
    _check(lib().oracle_knn_list(X, n, m, k, rows, len(rows), out_i, out_d), "knn_list")
    return out_i, out_d


def adhoc_bandwidth(d2: np.ndarray, k0: int) -> np.ndarray:
    d2 = np.ascontiguousarray(d2, dtype=np.float64)
    n, k = d2.shape
    b = np.empty(n, dtype=np.float64)
    _check(lib().oracle_adhoc_bandwidth(d2, n, k, k0, b), "adhoc_bandwidth")
    return b


@dataclass
class Pattern:
    """A CSR sparsity pattern with the squared distance of every stored entry."""
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray     # int32 [nnz]
    dist2: np.ndarray   # float64 [nnz]

    @property
    def n(self) -> int:
        return len(self.rowptr) - 1

    @staticmethod
    def from_knn(idx: np.ndarray, d2: np.ndarray) -> "Pattern":
        n, k = idx.shape
        return Pattern(np.arange(n + 1, dtype=np.int64) * k,
                       np.ascontiguousarray(idx.ravel(), dtype=np.int32),
                       np.ascontiguousarray(d2.ravel(), dtype=np.float64))


@dataclass
class Tuning:
    chi: np.ndarray
    e_grid: np.ndarray
    slope: np.ndarray
    g_star: int
    e_star: float
    dim: float
    edge: bool


def chi(pat: Pattern, rho: np.ndarray, e_min: float, e_max: float, G: int) -> Tuning:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    c = np.empty(G); eg = np.empty(G); sl = np.empty(G - 1 if G > 1 else 1)
    gs, es, dm = _c_i32(), _c_f64(), _c_f64()
    rc = _check(lib().oracle_chi(pat.rowptr, pat.col, pat.dist2, rho, pat.n, e_min, e_max, G,
                                 c, eg, sl, ctypes.byref(gs), ctypes.byref(es),
                                 ctypes.byref(dm)), "chi")
    return Tuning(c, eg, sl, gs.value, es.value, dm.value, rc == 1)


def density(pat: Pattern, b: np.ndarray, e: float, d: float, beta: float):
    b = np.ascontiguousarray(b, dtype=np.float64)
    psi = np.empty(pat.n); rho = np.empty(pat.n)
    _check(lib().oracle_density(pat.rowptr, pat.col, pat.dist2, b, pat.n, e, d, beta, psi, rho),
           "density")
    return psi, rho


def grid_scale(ref: np.ndarray, rho: np.ndarray) -> float:
    ref = np.ascontiguousarray(ref, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    return float(lib().oracle_grid_scale(ref, rho, len(ref)))


def normalize(pat: Pattern, rho: np.ndarray, e: float, alpha: float, d: float,
              out_kind: int = MARKOV):
    """Values in pattern order plus q, P, D."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n = pat.n
    val = np.empty(len(pat.col)); q = np.empty(n); P = np.empty(n); D = np.empty(n)
    _check(lib().oracle_normalize(pat.rowptr, pat.col, pat.dist2, rho, n, e, alpha, d,
                                  out_kind, val, q, P, D), "normalize")
    return val, q, P, D


def truncate(pat: Pattern, rho: np.ndarray, e: float, delta: float) -> Pattern:
    """The entries of `pat` whose kernel value exp(-D2/(e rho_i rho_j)) exceeds
    delta (Section 4, Algorithm 1's sparsity tolerance), in their order."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n = pat.n
    rowptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(len(pat.col), dtype=np.int32)
    d2 = np.empty(len(pat.col), dtype=np.float64)
    nnz = _c_i64()
    _check(lib().oracle_truncate(pat.rowptr, pat.col, pat.dist2, rho, n, e, delta, rowptr, col, d2,
                                 ctypes.byref(nnz)), "truncate")
    return Pattern(rowptr, col[:nnz.value].copy(), d2[:nnz.value].copy())


def sort_rows_by_col(col: np.ndarray, val: np.ndarray, k: int):
    col = np.ascontiguousarray(col, dtype=np.int32).copy()
    val = np.ascontiguousarray(val, dtype=np.float64).copy()
    n = len(col) // k
    _check(lib().oracle_sort_rows_by_col(n, k, col, val), "sort_rows_by_col")
    return col, val


# ------------------------------------------------------------------ pipeline
@dataclass
class Result:
    idx: np.ndarray
    d2: np.ndarray
    b: np.ndarray
    tune_a: Tuning
    psi: np.ndarray
    rho: np.ndarray
    scale_b: float
    tune_b: Tuning
    q: np.ndarray
    P: np.ndarray
    D: np.ndarray
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray


def pipeline(X: np.ndarray, k: int, k0: int, d: float, alpha: float, beta: float,
             e_min: float = 1e-3, e_max: float = 1e1, G: int = 64,
             out_kind: int = MARKOV, knn_result=None) -> Result:
    """The whole kernel-matrix build in the paper's order, in FP64."""
    if knn_result is None:
        idx, d2 = knn(X, k)
    else:
        idx, d2 = knn_result
    n = idx.shape[0]
    pat = Pattern.from_knn(idx, d2)
    b = adhoc_bandwidth(d2, k0)
    ta = chi(pat, b, e_min, e_max, G)
    psi, rho = density(pat, b, ta.e_star, d, beta)
    s = grid_scale(b, rho)
    tb = chi(pat, rho, e_min * s, e_max * s, G)
    val, q, P, D = normalize(pat, rho, tb.e_star, alpha, d, out_kind)
    col, val = sort_rows_by_col(pat.col, val, k)
    return Result(idx, d2, b, ta, psi, rho, s, tb, q, P, D,
                  np.arange(n + 1, dtype=np.int64) * k, col, val)


def truncated_build(base: Pattern, d2_knn: np.ndarray, k0: int, d: float, alpha: float, beta: float,
                    delta: float, e_min: float = 1e-3, e_max: float = 1e1, G: int = 64, out_kind: int = MARKOV):
    """The build with the sparsity tolerance delta_tol of Section 4: the tuning
    sums run over the whole stored pattern `base`; the density kernel matrix
    (at e_A) and the operator kernel matrix (at e_B) keep only their entries
    above delta, and every row sum of the density, q and D runs over the kept
    entries. The ad-hoc bandwidth comes from the k-NN distances d2_knn."""
    b = adhoc_bandwidth(d2_knn, k0)
    ta = chi(base, b, e_min, e_max, G)
    pa = truncate(base, b, ta.e_star, delta)
    psi, rho = density(pa, b, ta.e_star, d, beta)
    s = grid_scale(b, rho)
    tb = chi(base, rho, e_min * s, e_max * s, G)
    pb = truncate(base, rho, tb.e_star, delta)
    val, q, P, D = normalize(pb, rho, tb.e_star, alpha, d, out_kind)
    return dict(b=b, ta=ta, pa=pa, psi=psi, rho=rho, s=s, tb=tb, pb=pb, val=val, q=q, P=P, D=D)
