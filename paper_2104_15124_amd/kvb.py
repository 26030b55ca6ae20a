"""Python binding of libkvb.so (ctypes; torch tensors for device memory).

Each function here marshals torch tensors into the C ABI declared in
``include/kvb.h`` and returns torch tensors; all arithmetic runs in the HIP
kernels of the library. A missing library or a missing GPU raises
immediately: there is no CPU path.

Names follow the C ABI without the ``kvb_`` prefix. ``build_kernel_matrix``
chains the calls in the order of the paper's pipeline (Section 4, steps 1-2).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkvb.so")

# status / enum values mirrored from include/kvb.h
OK, W_GRID_EDGE, W_FALLBACK = 0, 1, 2
E_INVALID, E_NOMEM, E_HIP, E_UNSUPPORTED, E_NOT_TRAINED, E_IO, E_NO_DEVICE = -1, -2, -3, -4, -5, -6, -7
W_NOT_CONVERGED = 3
KNN_F32, KNN_BF16, KNN_LEARNED = 0, 1, 2
BW_ADHOC, BW_DENSITY = 0, 1
OUT_MARKOV, OUT_GENERATOR, OUT_SYMMETRIC = 0, 1, 2
ROW_RECHECK, ROW_FALLBACK, ROW_UNCERTIFIED = 1, 2, 4
OPT_FORCE_FALLBACK, OPT_SCRATCH_LIMIT, OPT_BF16_SPLIT, OPT_N_PROBE, OPT_CURVE_ORDER, OPT_PATTERN = 1, 2, 3, 4, 5, 6
PATTERNS = {"knn": 0, "union": 1}
MODES = {"f32": KNN_F32, "bf16": KNN_BF16, "learned": KNN_LEARNED}

EXPORTS = ("kvb_create", "kvb_create_host", "kvb_destroy", "kvb_last_error", "kvb_set_option", "kvb_knn",
           "kvb_knn_fallback_rows", "kvb_knn_pairs", "kvb_knn_exact_rows", "kvb_bandwidth",
           "kvb_grid_scale", "kvb_tune_eps", "kvb_assemble_csr", "kvb_build", "kvb_build_info", "kvb_part_init",
           "kvb_part_teacher", "kvb_part_train", "kvb_part_route", "kvb_part_save", "kvb_part_load", "kvb_mlp_forward",
           "kvb_mlp_backward", "kvb_part_num_params", "kvb_part_get_params", "kvb_part_set_params",
           "kvb_version", "kvb_profile_enable", "kvb_profile_read", "kvb_profile_name",
           "kvb_union_pattern", "kvb_density_csr", "kvb_tune_eps_csr", "kvb_normalize_csr",
           "kvb_truncate_csr", "kvb_set_tolerance", "kvb_eigsh", "kvb_kolmogorov_solve",
           "kvb_carre_du_champ", "kvb_advect", "kvb_lanczos_prefix", "kvb_peak_probe", "kvb_tune_eps_noalloc")
PROF_SLOTS = 15
PEAK_HBM_COPY, PEAK_MFMA_BF16, PEAK_MFMA_F32, PEAK_EXP, PEAK_VALU_FMA = 0, 1, 2, 3, 4


class KvbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"kvb error {code}: {msg}")
        self.code = code


_lib = None
_vp, _i32, _i64, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double


def load_library(path: str = LIB_PATH):
    """Load libkvb.so and declare its C signatures (needs no GPU)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise KvbError(E_UNSUPPORTED, f"HIP library not built: {path} is missing "
                       "(run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    L.kvb_create.argtypes = [ctypes.POINTER(_vp), _vp]
    L.kvb_create_host.argtypes = [ctypes.POINTER(_vp)]
    L.kvb_destroy.argtypes = [_vp]
    L.kvb_destroy.restype = None
    L.kvb_last_error.argtypes = [_vp]
    L.kvb_last_error.restype = ctypes.c_char_p
    L.kvb_set_option.argtypes = [_vp, _i32, _i64]
    L.kvb_knn.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _i32, _vp, _vp, _vp]
    L.kvb_knn_fallback_rows.argtypes = [_vp, ctypes.POINTER(_i64)]
    L.kvb_knn_pairs.argtypes = [_vp, ctypes.POINTER(_f64)]
    L.kvb_knn_exact_rows.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _i64, _vp, _vp]
    L.kvb_bandwidth.argtypes = [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _vp, _f64, _f64, _f64, _vp, _vp]
    L.kvb_grid_scale.argtypes = [_vp, _vp, _vp, _i64, ctypes.POINTER(_f64)]
    L.kvb_tune_eps.argtypes = [_vp, _vp, _vp, _vp, _i64, _i32, _f64, _f64, _i32,
                               _vp, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]
    L.kvb_tune_eps_noalloc.argtypes = L.kvb_tune_eps.argtypes
    L.kvb_tune_eps_noalloc.restype = ctypes.c_int
    L.kvb_assemble_csr.argtypes = [_vp, _vp, _vp, _vp, _i64, _i32, _f64, _f64, _f64, _i32,
                                   _vp, _vp, _vp, _vp, _vp]
    L.kvb_build.argtypes = [_vp, _vp, _i64, _i32, _i32, _i32, _i32, _i32, _f64, _f64, _f64, _f64, _f64, _i32, _i32,
                            _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    L.kvb_build_info.argtypes = [_vp, _vp, _vp, _vp]
    L.kvb_union_pattern.argtypes = [_vp, _vp, _vp, _i64, _i32, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]
    L.kvb_density_csr.argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _vp, _f64, _f64, _f64, _vp, _vp]
    L.kvb_tune_eps_csr.argtypes = [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _f64, _f64, _i32, _vp,
                                   ctypes.POINTER(_f64), ctypes.POINTER(_f64)]
    L.kvb_set_tolerance.argtypes = [_vp, _f64]
    L.kvb_advect.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _f64, _f64, _vp]
    L.kvb_carre_du_champ.argtypes = [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _vp]
    L.kvb_kolmogorov_solve.argtypes = [_vp, _vp, _vp, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _vp, _vp]
    L.kvb_peak_probe.argtypes = [_vp, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]
    L.kvb_peak_probe.restype = ctypes.c_int
    L.kvb_lanczos_prefix.argtypes = [_vp, _vp, _i32, ctypes.POINTER(_i32)]
    L.kvb_lanczos_prefix.restype = ctypes.c_int
    L.kvb_eigsh.argtypes = [_vp, _vp, _vp, _vp, _i64, _i64, _i32, _i32, _f64, ctypes.c_uint64, _vp, _vp, _vp]
    L.kvb_truncate_csr.argtypes = [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _f64, _f64, _vp, _vp, _vp,
                                   ctypes.POINTER(_i64)]
    L.kvb_normalize_csr.argtypes = [_vp, _vp, _vp, _vp, _vp, _i64, _i64, _f64, _f64, _f64, _i32, _vp, _vp, _vp]
    _u64, _f32 = ctypes.c_uint64, ctypes.c_float
    L.kvb_part_init.argtypes = [_vp, _i32, _i32, _i32, _i32, _i32, _u64]
    L.kvb_part_teacher.argtypes = [_vp, _vp, _i64, _i32, _i32, _u64, _vp]
    L.kvb_part_train.argtypes = [_vp, _vp, _i64, _i32, _vp, _vp, _i32, _i32, _i32, _f32, _u64, _vp]
    L.kvb_part_route.argtypes = [_vp, _vp, _i64, _vp, _vp]
    L.kvb_part_save.argtypes = [_vp, ctypes.c_char_p]
    L.kvb_part_load.argtypes = [_vp, ctypes.c_char_p]
    L.kvb_mlp_forward.argtypes = [_vp, _vp, _i64, _vp]
    L.kvb_mlp_backward.argtypes = [_vp, _vp, _i64, _vp, _i32, _vp, _vp]
    L.kvb_part_num_params.argtypes = [_vp]
    L.kvb_part_num_params.restype = _i64
    L.kvb_part_get_params.argtypes = [_vp, _vp]
    L.kvb_part_set_params.argtypes = [_vp, _vp]
    L.kvb_version.restype = ctypes.c_char_p
    L.kvb_profile_enable.argtypes = [_vp, _i32]
    L.kvb_profile_read.argtypes = [_vp, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_i64)]
    L.kvb_profile_name.argtypes = [_i32]
    L.kvb_profile_name.restype = ctypes.c_char_p
    for name in ("kvb_create", "kvb_create_host", "kvb_set_option", "kvb_knn", "kvb_knn_fallback_rows", "kvb_knn_exact_rows",
                 "kvb_knn_pairs",
                 "kvb_bandwidth",
                 "kvb_grid_scale", "kvb_tune_eps", "kvb_assemble_csr", "kvb_profile_enable",
                 "kvb_profile_read", "kvb_build", "kvb_build_info", "kvb_part_init", "kvb_part_teacher", "kvb_part_train",
                 "kvb_part_route", "kvb_part_save", "kvb_part_load", "kvb_mlp_forward",
                 "kvb_mlp_backward", "kvb_part_get_params", "kvb_part_set_params"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


class Context:
    """A library context bound to one HIP stream of the current device."""

    def __init__(self, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise KvbError(E_UNSUPPORTED, "no GPU visible: the kvb library has no CPU path")
        self.lib = load_library()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = self.stream.device
        h = _vp()
        with torch.cuda.device(self.device):
            rc = self.lib.kvb_create(ctypes.byref(h), _vp(self.stream.cuda_stream))
        if rc != OK:
            raise KvbError(rc, "kvb_create failed (gfx950 device required)")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.kvb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc: int) -> int:
        if rc < 0:
            raise KvbError(rc, self.lib.kvb_last_error(self.h).decode())
        return rc

    def set_option(self, key: int, value: int):
        self.check(self.lib.kvb_set_option(self.h, key, int(value)))

    def profile(self, on: bool):
        """Start (or stop) per-kernel event timing; totals restart at zero."""
        self.check(self.lib.kvb_profile_enable(self.h, 1 if on else 0))

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launch sequences)} since profile(True)."""
        out = {}
        for s in range(PROF_SLOTS):
            ms, cnt = _f64(), _i64()
            self.check(self.lib.kvb_profile_read(self.h, s, ctypes.byref(ms), ctypes.byref(cnt)))
            out[self.lib.kvb_profile_name(s).decode()] = (float(ms.value), int(cnt.value))
        return out


_contexts: dict = {}


def context() -> Context:
    """The cached context of the current device and current torch stream."""
    s = torch.cuda.current_stream()
    key = (s.device.index, s.cuda_stream)
    ctx = _contexts.get(key)
    if ctx is None:
        ctx = _contexts[key] = Context(s)
    return ctx


def _ptr(t: torch.Tensor | None):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise KvbError(E_INVALID, f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise KvbError(E_INVALID, f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


# ------------------------------------------------------------------ entry points
def knn(X: torch.Tensor, k: int, mode: str = "f32", margin: int = 32, ctx: Context | None = None):
    """Exact k-NN self-join: returns idx [n,k] int32, d2 [n,k] float32, row flags [n] int32."""
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    n, m = X.shape
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, k), dtype=torch.float32, device=X.device)
    flags = torch.empty(n, dtype=torch.int32, device=X.device)
    ctx.check(ctx.lib.kvb_knn(ctx.h, _ptr(X), n, m, k, MODES[mode], margin, _ptr(idx), _ptr(d2), _ptr(flags)))
    return idx, d2, flags


def peak_probe(kind: int, ctx: Context | None = None):
    """(rate, ms) of a peak microbenchmark (kvb_peak_probe): PEAK_HBM_COPY in
    bytes/s (read + written), PEAK_MFMA_* in flop/s, PEAK_EXP in exp/s,
    PEAK_VALU_FMA in lane-op/s."""
    ctx = ctx or context()
    rate, ms = _f64(), _f64()
    ctx.check(ctx.lib.kvb_peak_probe(ctx.h, kind, ctypes.byref(rate), ctypes.byref(ms)))
    return float(rate.value), float(ms.value)


def knn_fallback_rows(ctx: Context | None = None) -> int:
    ctx = ctx or context()
    c = _i64()
    ctx.check(ctx.lib.kvb_knn_fallback_rows(ctx.h, ctypes.byref(c)))
    return int(c.value)


def knn_pairs(ctx: Context | None = None) -> float:
    """Candidate pairs scored by the last knn call on the context."""
    ctx = ctx or context()
    p = _f64()
    ctx.check(ctx.lib.kvb_knn_pairs(ctx.h, ctypes.byref(p)))
    return float(p.value)


def knn_exact_rows(X: torch.Tensor, k: int, rows: torch.Tensor, ctx: Context | None = None):
    """Exact float64 k-NN of the listed rows against all samples: idx, d2 [len(rows), k]."""
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    rows = _dev(rows, torch.int32, "rows")
    n, m = X.shape
    r = rows.numel()
    idx = torch.empty((r, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((r, k), dtype=torch.float32, device=X.device)
    ctx.check(ctx.lib.kvb_knn_exact_rows(ctx.h, _ptr(X), n, m, k, _ptr(rows), r, _ptr(idx), _ptr(d2)))
    return idx, d2


def bandwidth_adhoc(d2: torch.Tensor, k0: int, ctx: Context | None = None) -> torch.Tensor:
    ctx = ctx or context()
    d2 = _dev(d2, torch.float32, "d2")
    n, k = d2.shape
    b = torch.empty(n, dtype=torch.float32, device=d2.device)
    ctx.check(ctx.lib.kvb_bandwidth(ctx.h, _vp(0), _ptr(d2), n, k, BW_ADHOC, k0, _vp(0), 0.0, 0.0, 0.0,
                                    _ptr(b), _vp(0)))
    return b


def bandwidth_density(idx: torch.Tensor, d2: torch.Tensor, b: torch.Tensor, e: float, d: float, beta: float,
                      ctx: Context | None = None):
    """Returns (rho, psi) with psi the density estimate and rho = 2 psi^beta."""
    ctx = ctx or context()
    idx = _dev(idx, torch.int32, "idx")
    d2 = _dev(d2, torch.float32, "d2")
    b = _dev(b, torch.float32, "b")
    n, k = d2.shape
    rho = torch.empty(n, dtype=torch.float32, device=d2.device)
    psi = torch.empty(n, dtype=torch.float32, device=d2.device)
    ctx.check(ctx.lib.kvb_bandwidth(ctx.h, _ptr(idx), _ptr(d2), n, k, BW_DENSITY, 0, _ptr(b), e, d, beta,
                                    _ptr(rho), _ptr(psi)))
    return rho, psi


def grid_scale(ref: torch.Tensor, rho: torch.Tensor, ctx: Context | None = None) -> float:
    ctx = ctx or context()
    ref = _dev(ref, torch.float32, "ref")
    rho = _dev(rho, torch.float32, "rho")
    s = _f64()
    ctx.check(ctx.lib.kvb_grid_scale(ctx.h, _ptr(ref), _ptr(rho), ref.numel(), ctypes.byref(s)))
    return float(s.value)


@dataclass
class Tuning:
    chi: np.ndarray
    e_star: float
    dim: float
    edge: bool


def tune_eps(idx: torch.Tensor, d2: torch.Tensor, rho: torch.Tensor, e_min: float, e_max: float, G: int,
             ctx: Context | None = None) -> Tuning:
    ctx = ctx or context()
    idx = _dev(idx, torch.int32, "idx")
    d2 = _dev(d2, torch.float32, "d2")
    rho = _dev(rho, torch.float32, "rho")
    n, k = d2.shape
    chi = np.zeros(G, dtype=np.float64)
    es, dm = _f64(), _f64()
    rc = ctx.check(ctx.lib.kvb_tune_eps(ctx.h, _ptr(idx), _ptr(d2), _ptr(rho), n, k, e_min, e_max, G,
                                        chi.ctypes.data_as(_vp), ctypes.byref(es), ctypes.byref(dm)))
    return Tuning(chi, float(es.value), float(dm.value), rc == W_GRID_EDGE)


def assemble_csr(idx: torch.Tensor, d2: torch.Tensor, rho: torch.Tensor, e: float, alpha: float, d: float,
                 out_kind: int = OUT_MARKOV, ctx: Context | None = None):
    """Returns rowptr [n+1] int64, col [nnz] int32, val [nnz] float32, P [n] f64, D [n] f64."""
    ctx = ctx or context()
    idx = _dev(idx, torch.int32, "idx")
    d2 = _dev(d2, torch.float32, "d2")
    rho = _dev(rho, torch.float32, "rho")
    n, k = d2.shape
    dev = d2.device
    rowptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(n * k, dtype=torch.int32, device=dev)
    val = torch.empty(n * k, dtype=torch.float32, device=dev)
    P = torch.empty(n, dtype=torch.float64, device=dev)
    D = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.check(ctx.lib.kvb_assemble_csr(ctx.h, _ptr(idx), _ptr(d2), _ptr(rho), n, k, e, alpha, d, out_kind,
                                       _ptr(rowptr), _ptr(col), _ptr(val), _ptr(P), _ptr(D)))
    return rowptr, col, val, P, D


@dataclass
class KernelMatrix:
    idx: torch.Tensor
    d2: torch.Tensor
    flags: torch.Tensor
    b: torch.Tensor
    tune_a: Tuning
    rho: torch.Tensor
    psi: torch.Tensor
    scale_b: float
    tune_b: Tuning
    rowptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    P: torch.Tensor
    D: torch.Tensor
    status: int = OK      # the call's status: OK or a warning (W_GRID_EDGE, W_FALLBACK)


def build(X: torch.Tensor, k: int, k0: int, d: float, alpha: float, beta: float, e_min: float = 1e-3,
          e_max: float = 1e1, G: int = 64, mode: str = "f32", margin: int = 32, out_kind: int = OUT_MARKOV,
          ctx: Context | None = None, out: KernelMatrix | None = None, sync: bool = True,
          pattern: str = "knn", delta: float = 0.0) -> KernelMatrix:
    """The whole build in one library call (kvb_build): the same steps and results
    as build_kernel_matrix (pattern "knn") or build_union_matrix (pattern
    "union", the symmetric E u E^T), with the intermediate values kept on the
    device; delta > 0 applies the sparsity tolerance of Section 4 as
    build_truncated_matrix does (rows then in column order). `out` (a previous
    result of the same n, k and pattern) lends its device arrays. sync=False
    only enqueues the work (the tuning results of the returned matrix are then
    None; build_info(ctx) waits and returns them; with the union pattern or a
    tolerance col and val then keep their capacity and rowptr[n] is the stored
    count)."""
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    n, m = X.shape
    dev = X.device
    cap = n * k if pattern == "knn" else n * (2 * k - 1)
    ctx.check(ctx.lib.kvb_set_option(ctx.h, OPT_PATTERN, PATTERNS[pattern]))
    ctx.check(ctx.lib.kvb_set_tolerance(ctx.h, float(delta)))
    if out is not None and out.idx.shape == (n, k) and out.idx.device == dev and out.col.numel() == cap:
        idx, d2, flags, b, rho, psi = out.idx, out.d2, out.flags, out.b, out.rho, out.psi
        rowptr, col, val, P, D = out.rowptr, out.col, out.val, out.P, out.D
    else:
        idx = torch.empty((n, k), dtype=torch.int32, device=dev)
        d2 = torch.empty((n, k), dtype=torch.float32, device=dev)
        flags = torch.empty(n, dtype=torch.int32, device=dev)
        b = torch.empty(n, dtype=torch.float32, device=dev)
        rho = torch.empty(n, dtype=torch.float32, device=dev)
        psi = torch.empty(n, dtype=torch.float32, device=dev)
        rowptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
        col = torch.empty(cap, dtype=torch.int32, device=dev)
        val = torch.empty(cap, dtype=torch.float32, device=dev)
        P = torch.empty(n, dtype=torch.float64, device=dev)
        D = torch.empty(n, dtype=torch.float64, device=dev)
    chi_a = np.zeros(G, dtype=np.float64)
    chi_b = np.zeros(G, dtype=np.float64)
    info = np.zeros(8, dtype=np.float64)
    host = (chi_a.ctypes.data_as(_vp), chi_b.ctypes.data_as(_vp), info.ctypes.data_as(_vp)) if sync else \
        (None, None, None)
    rc = ctx.check(ctx.lib.kvb_build(ctx.h, _ptr(X), n, m, k, MODES[mode], margin, k0, d, alpha, beta, e_min, e_max,
                                     G, out_kind, _ptr(idx), _ptr(d2), _ptr(flags), _ptr(b), _ptr(rho), _ptr(psi),
                                     _ptr(rowptr), _ptr(col), _ptr(val), _ptr(P), _ptr(D), *host))
    if not sync:
        return KernelMatrix(idx, d2, flags, b, None, rho, psi, None, None, rowptr, col, val, P, D, rc)
    ta, s, tb = _tunings(chi_a, chi_b, info, G)
    if pattern != "knn" or delta > 0:
        nnz = int(rowptr[n].item())
        col, val = col[:nnz], val[:nnz]
    return KernelMatrix(idx, d2, flags, b, ta, rho, psi, s, tb, rowptr, col, val, P, D, rc)


def _tunings(chi_a, chi_b, info, G):
    ga, gb = int(info[5]), int(info[6])
    ta = Tuning(chi_a, float(info[0]), float(info[1]), ga in (0, G - 2))
    tb = Tuning(chi_b, float(info[3]), float(info[4]), gb in (0, G - 2))
    return ta, float(info[2]), tb


def build_info(G: int = 64, ctx: Context | None = None):
    """Wait for the last build on the context: (tuning A, grid scale, tuning B,
    rows that took the exact fallback)."""
    ctx = ctx or context()
    chi_a = np.zeros(256, dtype=np.float64)   # the library's largest grid
    chi_b = np.zeros(256, dtype=np.float64)
    info = np.zeros(8, dtype=np.float64)
    ctx.check(ctx.lib.kvb_build_info(ctx.h, chi_a.ctypes.data_as(_vp), chi_b.ctypes.data_as(_vp),
                                     info.ctypes.data_as(_vp)))
    ta, s, tb = _tunings(chi_a[:G], chi_b[:G], info, G)
    return ta, s, tb, int(info[7])


def build_kernel_matrix(X: torch.Tensor, k: int, k0: int, d: float, alpha: float, beta: float,
                        e_min: float = 1e-3, e_max: float = 1e1, G: int = 64, mode: str = "f32",
                        margin: int = 32, out_kind: int = OUT_MARKOV, ctx: Context | None = None) -> KernelMatrix:
    """The whole sparse kernel-matrix build, in the paper's order: k-NN ->
    ad-hoc bandwidth -> tune e (density kernel) -> density psi, rho = 2 psi^beta
    -> tune e (operator kernel, power-of-two shifted grid) -> q, Kt, D -> CSR."""
    ctx = ctx or context()
    idx, d2, flags = knn(X, k, mode, margin, ctx)
    b = bandwidth_adhoc(d2, k0, ctx)
    ta = tune_eps(idx, d2, b, e_min, e_max, G, ctx)
    rho, psi = bandwidth_density(idx, d2, b, ta.e_star, d, beta, ctx)
    s = grid_scale(b, rho, ctx)
    tb = tune_eps(idx, d2, rho, e_min * s, e_max * s, G, ctx)
    rowptr, col, val, P, D = assemble_csr(idx, d2, rho, tb.e_star, alpha, d, out_kind, ctx)
    return KernelMatrix(idx, d2, flags, b, ta, rho, psi, s, tb, rowptr, col, val, P, D)


# ------------------------------------------------------------------ union pattern E u E^T
@dataclass
class CsrPattern:
    """A CSR pattern with the squared distance of each stored entry (device)."""
    rowptr: torch.Tensor   # int64 [n+1]
    col: torch.Tensor      # int32 [nnz]
    d2: torch.Tensor       # float32 [nnz]

    @property
    def n(self) -> int:
        return self.rowptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.col.numel()


def union_pattern(idx: torch.Tensor, d2: torch.Tensor, ctx: Context | None = None) -> CsrPattern:
    """E u E^T of a k-NN pattern: row i holds every j with j in N(i) or i in N(j),
    columns ascending (kvb_union_pattern)."""
    ctx = ctx or context()
    idx = _dev(idx, torch.int32, "idx")
    d2 = _dev(d2, torch.float32, "d2")
    n, k = d2.shape
    cap = n * (2 * k - 1)
    rowptr = torch.empty(n + 1, dtype=torch.int64, device=d2.device)
    col = torch.empty(cap, dtype=torch.int32, device=d2.device)
    ud2 = torch.empty(cap, dtype=torch.float32, device=d2.device)
    nnz = _i64()
    ctx.check(ctx.lib.kvb_union_pattern(ctx.h, _ptr(idx), _ptr(d2), n, k, _ptr(rowptr), _ptr(col), _ptr(ud2), cap,
                                        ctypes.byref(nnz)))
    return CsrPattern(rowptr, col[:nnz.value], ud2[:nnz.value])


def knn_pattern(idx: torch.Tensor, d2: torch.Tensor) -> CsrPattern:
    """The directed k-NN pattern as CSR (views of idx and d2; rows in distance order)."""
    n, k = idx.shape
    rowptr = torch.arange(n + 1, dtype=torch.int64, device=idx.device) * k
    return CsrPattern(rowptr, _dev(idx, torch.int32, "idx").reshape(-1), _dev(d2, torch.float32, "d2").reshape(-1))


def truncate_csr(pat: CsrPattern, rho: torch.Tensor, e: float, delta: float, ctx: Context | None = None) -> CsrPattern:
    """The entries of `pat` whose kernel value exp(-d2/(e rho_i rho_j)) exceeds
    delta, in their order (kvb_truncate_csr)."""
    ctx = ctx or context()
    rho = _dev(rho, torch.float32, "rho")
    dev = rho.device
    rowptr = torch.empty(pat.n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(pat.nnz, dtype=torch.int32, device=dev)
    d2 = torch.empty(pat.nnz, dtype=torch.float32, device=dev)
    nnz = _i64()
    ctx.check(ctx.lib.kvb_truncate_csr(ctx.h, _ptr(pat.rowptr), _ptr(pat.col), _ptr(pat.d2), _ptr(rho), pat.n,
                                       pat.nnz, e, delta, _ptr(rowptr), _ptr(col), _ptr(d2), ctypes.byref(nnz)))
    return CsrPattern(rowptr, col[:nnz.value], d2[:nnz.value])


def density_csr(pat: CsrPattern, b: torch.Tensor, e: float, d: float, beta: float, ctx: Context | None = None):
    """(rho, psi) over a CSR pattern (kvb_density_csr)."""
    ctx = ctx or context()
    b = _dev(b, torch.float32, "b")
    rho = torch.empty(pat.n, dtype=torch.float32, device=b.device)
    psi = torch.empty(pat.n, dtype=torch.float32, device=b.device)
    ctx.check(ctx.lib.kvb_density_csr(ctx.h, _ptr(pat.rowptr), _ptr(pat.col), _ptr(pat.d2), pat.n, pat.nnz, _ptr(b),
                                      e, d, beta, _ptr(rho), _ptr(psi)))
    return rho, psi


def tune_eps_csr(pat: CsrPattern, rho: torch.Tensor, e_min: float, e_max: float, G: int,
                 ctx: Context | None = None) -> Tuning:
    ctx = ctx or context()
    rho = _dev(rho, torch.float32, "rho")
    chi = np.zeros(G, dtype=np.float64)
    es, dm = _f64(), _f64()
    rc = ctx.check(ctx.lib.kvb_tune_eps_csr(ctx.h, _ptr(pat.rowptr), _ptr(pat.col), _ptr(pat.d2), _ptr(rho), pat.n,
                                            pat.nnz, e_min, e_max, G, chi.ctypes.data_as(_vp), ctypes.byref(es),
                                            ctypes.byref(dm)))
    return Tuning(chi, float(es.value), float(dm.value), rc == W_GRID_EDGE)


def normalize_csr(pat: CsrPattern, rho: torch.Tensor, e: float, alpha: float, d: float, out_kind: int = OUT_MARKOV,
                  ctx: Context | None = None):
    """Values in pattern order plus P, D (kvb_normalize_csr)."""
    ctx = ctx or context()
    rho = _dev(rho, torch.float32, "rho")
    val = torch.empty(pat.nnz, dtype=torch.float32, device=rho.device)
    P = torch.empty(pat.n, dtype=torch.float64, device=rho.device)
    D = torch.empty(pat.n, dtype=torch.float64, device=rho.device)
    ctx.check(ctx.lib.kvb_normalize_csr(ctx.h, _ptr(pat.rowptr), _ptr(pat.col), _ptr(pat.d2), _ptr(rho), pat.n,
                                        pat.nnz, e, alpha, d, out_kind, _ptr(val), _ptr(P), _ptr(D)))
    return val, P, D


@dataclass
class UnionMatrix:
    idx: torch.Tensor
    d2: torch.Tensor
    pattern: CsrPattern
    b: torch.Tensor
    tune_a: Tuning
    rho: torch.Tensor
    psi: torch.Tensor
    scale_b: float
    tune_b: Tuning
    val: torch.Tensor
    P: torch.Tensor
    D: torch.Tensor


def build_union_matrix(X: torch.Tensor, k: int, k0: int, d: float, alpha: float, beta: float,
                       e_min: float = 1e-3, e_max: float = 1e1, G: int = 64, mode: str = "f32", margin: int = 32,
                       out_kind: int = OUT_MARKOV, ctx: Context | None = None, knn_result=None) -> UnionMatrix:
    """The build of build_kernel_matrix on the symmetric pattern E u E^T: the
    ad-hoc bandwidth from the k nearest neighbours, every later row sum over
    the union row. knn_result = (idx, d2) skips the search."""
    ctx = ctx or context()
    if knn_result is None:
        idx, d2, _ = knn(X, k, mode, margin, ctx)
    else:
        idx, d2 = knn_result
    b = bandwidth_adhoc(d2, k0, ctx)
    pat = union_pattern(idx, d2, ctx)
    ta = tune_eps_csr(pat, b, e_min, e_max, G, ctx)
    rho, psi = density_csr(pat, b, ta.e_star, d, beta, ctx)
    s = grid_scale(b, rho, ctx)
    tb = tune_eps_csr(pat, rho, e_min * s, e_max * s, G, ctx)
    val, P, D = normalize_csr(pat, rho, tb.e_star, alpha, d, out_kind, ctx)
    return UnionMatrix(idx, d2, pat, b, ta, rho, psi, s, tb, val, P, D)


@dataclass
class Eigs:
    values: np.ndarray          # [nev], descending
    residuals: np.ndarray       # [nev] Ritz residual norms
    vectors: torch.Tensor | None  # [nev, n] float64, unit rows
    converged: bool


def eigsh(rowptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, nev: int = 8, ncv: int = 128,
          tol: float = 1e-8, seed: int = 0, vectors: bool = True, ctx: Context | None = None) -> Eigs:
    """The nev largest eigenpairs of a symmetric CSR matrix (kvb_eigsh); for the
    symmetric conjugate Lhat these are the eigenvalues nearest zero."""
    ctx = ctx or context()
    rowptr = _dev(rowptr, torch.int64, "rowptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float32, "val")
    n = rowptr.numel() - 1
    ev = np.zeros(nev, dtype=np.float64)
    rs = np.zeros(nev, dtype=np.float64)
    vec = torch.empty((nev, n), dtype=torch.float64, device=val.device) if vectors else None
    rc = ctx.check(ctx.lib.kvb_eigsh(ctx.h, _ptr(rowptr), _ptr(col), _ptr(val), n, col.numel(), nev, ncv, tol,
                                     seed, ev.ctypes.data_as(_vp), rs.ctypes.data_as(_vp), _ptr(vec)))
    return Eigs(ev, rs, vec, rc != W_NOT_CONVERGED)


def kolmogorov_solve(eigs: Eigs, P: torch.Tensor, D: torch.Tensor, g: torch.Tensor, skip: int = 1,
                     ctx: Context | None = None):
    """Least-squares solution of L f = g in the span of the leading eigenvectors
    (kvb_kolmogorov_solve): returns (f, g projected on the span, coefficients)."""
    ctx = ctx or context()
    g = _dev(g, torch.float64, "g")
    n = g.numel()
    f = torch.empty(n, dtype=torch.float64, device=g.device)
    gl = torch.empty(n, dtype=torch.float64, device=g.device)
    nvec = len(eigs.values)
    coef = np.zeros(nvec - skip, dtype=np.float64)
    ev = np.ascontiguousarray(eigs.values, dtype=np.float64)
    ctx.check(ctx.lib.kvb_kolmogorov_solve(ctx.h, _ptr(eigs.vectors), ev.ctypes.data_as(_vp), nvec, skip,
                                           _ptr(_dev(P, torch.float64, "P")), _ptr(_dev(D, torch.float64, "D")),
                                           _ptr(g), n, _ptr(f), _ptr(gl), coef.ctypes.data_as(_vp)))
    return f, gl, coef


def carre_du_champ(eigs: Eigs, P: torch.Tensor, D: torch.Tensor, u: torch.Tensor, v: torch.Tensor,
                   tensor: bool = False, ctx: Context | None = None):
    """grad u . grad v at the samples from the eigenbasis (kvb_carre_du_champ);
    with tensor=True also the coefficients C_ljk as a [nvec, nvec, nvec] tensor."""
    ctx = ctx or context()
    u = _dev(u, torch.float64, "u")
    v = _dev(v, torch.float64, "v")
    n = u.numel()
    nvec = len(eigs.values)
    grad = torch.empty(n, dtype=torch.float64, device=u.device)
    C = torch.empty((nvec, nvec, nvec), dtype=torch.float64, device=u.device) if tensor else None
    ev = np.ascontiguousarray(eigs.values, dtype=np.float64)
    ctx.check(ctx.lib.kvb_carre_du_champ(ctx.h, _ptr(eigs.vectors), ev.ctypes.data_as(_vp), nvec,
                                         _ptr(_dev(P, torch.float64, "P")), _ptr(_dev(D, torch.float64, "D")),
                                         _ptr(u), _ptr(v), n, _ptr(grad), _ptr(C)))
    return grad, C


@dataclass
class AdvectionStep:
    X: torch.Tensor          # [n, m] float32, the moved samples
    f: torch.Tensor          # [n] float64, the Kolmogorov solution
    grad: torch.Tensor       # [m, n] float64, grad f at the samples
    eigs: Eigs


def advection_step(X: torch.Tensor, g: torch.Tensor, dt: float, ell: int | None = None, k: int = 64, k0: int = 8,
                   sigma: float = 0.0, velocity: torch.Tensor | None = None, noise: torch.Tensor | None = None,
                   ncv: int = 400, seed: int = 0, ctx: Context | None = None) -> AdvectionStep:
    """One time step of the density-evolution example (Section 5.3): the
    kernel matrix of the samples (symmetric conjugate on the union pattern,
    c = 1: alpha = -d/4, beta = -1/2 with d = m), its leading ell nonzero
    eigenpairs (default 3 ln n), the Kolmogorov solution of L f = g, grad f
    through the Carre du champ identity, then the particle update
    x + dt (u - grad f) + sqrt(dt) sigma w."""
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    n, m = X.shape
    ell = ell or int(round(3 * np.log(n)))
    km = build(X, k, k0, float(m), -m / 4.0, -0.5, out_kind=OUT_SYMMETRIC, pattern="union", ctx=ctx)
    eg = eigsh(km.rowptr, km.col, km.val, nev=ell + 1, ncv=max(ncv, ell + 1), seed=seed, ctx=ctx)
    f, _, _ = kolmogorov_solve(eg, km.P, km.D, g, skip=1, ctx=ctx)
    grad = torch.empty((m, n), dtype=torch.float64, device=X.device)
    for s in range(m):
        gs, _ = carre_du_champ(eg, km.P, km.D, f, X[:, s].to(torch.float64), ctx=ctx)
        grad[s] = gs
    Xo = torch.empty_like(X)
    u = None if velocity is None else _dev(velocity, torch.float64, "velocity")
    w = None if noise is None else _dev(noise, torch.float64, "noise")
    ctx.check(ctx.lib.kvb_advect(ctx.h, _ptr(X), n, m, _ptr(u), _ptr(grad), _ptr(w), dt, sigma, _ptr(Xo)))
    return AdvectionStep(Xo, f, grad, eg)


@dataclass
class TruncatedMatrix:
    idx: torch.Tensor
    d2: torch.Tensor
    base: CsrPattern
    b: torch.Tensor
    tune_a: Tuning
    density_pattern: CsrPattern
    rho: torch.Tensor
    psi: torch.Tensor
    scale_b: float
    tune_b: Tuning
    pattern: CsrPattern
    val: torch.Tensor
    P: torch.Tensor
    D: torch.Tensor


def build_truncated_matrix(X: torch.Tensor, k: int, k0: int, d: float, alpha: float, beta: float, delta: float,
                           e_min: float = 1e-3, e_max: float = 1e1, G: int = 64, mode: str = "f32",
                           margin: int = 32, out_kind: int = OUT_MARKOV, pattern: str = "knn",
                           ctx: Context | None = None, knn_result=None) -> TruncatedMatrix:
    """The build with the sparsity tolerance delta_tol of Section 4 on the k-NN
    pattern (rows in distance order) or its union E u E^T (columns ascending):
    the tuning sums run over the whole pattern; the density kernel matrix (at
    e_A) and the operator kernel matrix (at e_B) keep only entries above delta,
    and the density, q and D row sums run over the kept entries."""
    ctx = ctx or context()
    if knn_result is None:
        idx, d2, _ = knn(X, k, mode, margin, ctx)
    else:
        idx, d2 = knn_result
    b = bandwidth_adhoc(d2, k0, ctx)
    base = knn_pattern(idx, d2) if pattern == "knn" else union_pattern(idx, d2, ctx)
    ta = tune_eps_csr(base, b, e_min, e_max, G, ctx)
    pa = truncate_csr(base, b, ta.e_star, delta, ctx)
    rho, psi = density_csr(pa, b, ta.e_star, d, beta, ctx)
    s = grid_scale(b, rho, ctx)
    tb = tune_eps_csr(base, rho, e_min * s, e_max * s, G, ctx)
    pb = truncate_csr(base, rho, tb.e_star, delta, ctx)
    val, P, D = normalize_csr(pb, rho, tb.e_star, alpha, d, out_kind, ctx)
    return TruncatedMatrix(idx, d2, base, b, ta, pa, rho, psi, s, tb, pb, val, P, D)


# ------------------------------------------------------------------ learned partitioner
def part_init(m: int, h1: int = 256, h2: int = 256, n_buckets: int = 1024, n_probe: int = 4, seed: int = 0,
              ctx: Context | None = None):
    """Fresh partitioner parameters in the context (He-normal weights, zero biases)."""
    ctx = ctx or context()
    ctx.check(ctx.lib.kvb_part_init(ctx.h, m, h1, h2, n_buckets, n_probe, int(seed)))


def part_teacher(Xs: torch.Tensor, levels: int = 10, seed: int = 0, ctx: Context | None = None) -> torch.Tensor:
    """Balanced teacher partition of Xs: labels [ns] int32 in [0, 2^levels)."""
    ctx = ctx or context()
    Xs = _dev(Xs, torch.float32, "Xs")
    ns, m = Xs.shape
    labels = torch.empty(ns, dtype=torch.int32, device=Xs.device)
    ctx.check(ctx.lib.kvb_part_teacher(ctx.h, _ptr(Xs), ns, m, levels, int(seed), _ptr(labels)))
    return labels


def part_train(Xs: torch.Tensor, labels: torch.Tensor, idx_s: torch.Tensor, epochs: int = 10, batch: int = 512,
               lr: float = 1e-3, seed: int = 0, ctx: Context | None = None) -> np.ndarray:
    """Adam training on neighbour-histogram targets; returns the per-epoch mean losses."""
    ctx = ctx or context()
    Xs = _dev(Xs, torch.float32, "Xs")
    labels = _dev(labels, torch.int32, "labels")
    idx_s = _dev(idx_s, torch.int32, "idx_s")
    ns, m = Xs.shape
    ks = idx_s.shape[1]
    loss = np.zeros(epochs, dtype=np.float32)
    ctx.check(ctx.lib.kvb_part_train(ctx.h, _ptr(Xs), ns, m, _ptr(labels), _ptr(idx_s), ks, epochs, batch,
                                     float(lr), int(seed), loss.ctypes.data_as(_vp)))
    return loss


def part_route(X: torch.Tensor, n_probe: int, ctx: Context | None = None):
    """Returns (home [n] int32, probe [n, n_probe] int32)."""
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    n = X.shape[0]
    home = torch.empty(n, dtype=torch.int32, device=X.device)
    probe = torch.empty((n, n_probe), dtype=torch.int32, device=X.device)
    ctx.check(ctx.lib.kvb_part_route(ctx.h, _ptr(X), n, _ptr(home), _ptr(probe)))
    return home, probe


def part_save(path: str, ctx: Context | None = None):
    ctx = ctx or context()
    ctx.check(ctx.lib.kvb_part_save(ctx.h, os.fsencode(path)))


def part_load(path: str, ctx: Context | None = None):
    ctx = ctx or context()
    ctx.check(ctx.lib.kvb_part_load(ctx.h, os.fsencode(path)))


def part_num_params(ctx: Context | None = None) -> int:
    ctx = ctx or context()
    return int(ctx.check(int(ctx.lib.kvb_part_num_params(ctx.h))))


def part_get_params(ctx: Context | None = None) -> torch.Tensor:
    ctx = ctx or context()
    p = torch.empty(part_num_params(ctx), dtype=torch.float32, device=torch.device("cuda", ctx.device.index))
    ctx.check(ctx.lib.kvb_part_get_params(ctx.h, _ptr(p)))
    return p


def part_set_params(params: torch.Tensor, ctx: Context | None = None):
    ctx = ctx or context()
    params = _dev(params, torch.float32, "params")
    if params.numel() != part_num_params(ctx):
        raise KvbError(E_INVALID, "params has the wrong number of elements")
    ctx.check(ctx.lib.kvb_part_set_params(ctx.h, _ptr(params)))


def mlp_forward(X: torch.Tensor, n_buckets: int, ctx: Context | None = None) -> torch.Tensor:
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    B = X.shape[0]
    logits = torch.empty((B, n_buckets), dtype=torch.float32, device=X.device)
    ctx.check(ctx.lib.kvb_mlp_forward(ctx.h, _ptr(X), B, _ptr(logits)))
    return logits


def mlp_backward(X: torch.Tensor, nbr_labels: torch.Tensor, ctx: Context | None = None):
    """Returns (mean loss, flat gradient [num_params] float32) without updating."""
    ctx = ctx or context()
    X = _dev(X, torch.float32, "X")
    nbr_labels = _dev(nbr_labels, torch.int32, "nbr_labels")
    B = X.shape[0]
    grads = torch.empty(part_num_params(ctx), dtype=torch.float32, device=X.device)
    loss = ctypes.c_float()
    ctx.check(ctx.lib.kvb_mlp_backward(ctx.h, _ptr(X), B, _ptr(nbr_labels), nbr_labels.shape[1],
                                       ctypes.byref(loss), _ptr(grads)))
    return float(loss.value), grads


def train_partitioner(X: torch.Tensor, k: int, n_train: int = 200_000, levels: int = 10, h1: int = 256,
                      h2: int = 256, n_probe: int = 4, epochs: int = 10, batch: int = 512, lr: float = 1e-3,
                      seed: int = 0, exact_mode: str = "bf16", ctx: Context | None = None) -> np.ndarray:
    """Neural-LSH style training on a seeded subsample of X: exact k-NN of the
    subsample (k neighbours, self included), teacher partition into
    2^levels buckets, then Adam on the neighbour-histogram targets. Returns the
    per-epoch losses; the trained partitioner stays in the context."""
    ctx = ctx or context()
    n, m = X.shape
    ns = min(n, n_train)
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    sel = torch.randperm(n, generator=g)[:ns].to(X.device)
    Xs = X.index_select(0, sel).contiguous()
    mode = exact_mode if m > 8 else "f32"
    idx_s, _, _ = knn(Xs, k, mode, 32, ctx)
    labels = part_teacher(Xs, levels, seed, ctx)
    part_init(m, h1, h2, 1 << levels, n_probe, seed, ctx)
    return part_train(Xs, labels, idx_s, epochs, batch, lr, seed, ctx)
