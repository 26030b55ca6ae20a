"""The C-ABI library loads without a GPU, exports every declared symbol, and
checks every entry point's arguments on a host-only context.

No compute call is made here: this container has no GPU, and the library has
no CPU path by design. A host-only context (kvb_create_host) runs each entry
point's argument checks and stops with KVB_E_NO_DEVICE where device work would
start; the pointers passed are aligned placeholder addresses that nothing reads.
"""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kvb.h")
LIB = os.path.join(ROOT, "paper_2104_15124_amd", "libkvb.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kvb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("kvb_knn", "kvb_bandwidth", "kvb_tune_eps", "kvb_assemble_csr", "kvb_create",
                     "kvb_destroy", "kvb_last_error", "kvb_grid_scale"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkvb.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s+(kvb_[a-z0-9_]+)", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkvb.so not built")
def test_library_loads_and_binding_matches_header():
    from paper_2104_15124_amd import kvb
    L = kvb.load_library()
    assert L.kvb_version().startswith(b"kvb")
    assert sorted(kvb.EXPORTS) == declared_functions()
    for name in kvb.EXPORTS:
        assert hasattr(L, name)


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2104_15124_amd import kvb
    with pytest.raises(kvb.KvbError):
        kvb.Context()


def test_header_constants_match_binding():
    from paper_2104_15124_amd import kvb
    text = open(HEADER).read()
    consts = dict((k, int(v)) for k, v in re.findall(r"#define (KVB_[A-Z0-9_]+) \(?(-?\d+)\)?", text))
    pairs = {"KVB_OK": kvb.OK, "KVB_W_GRID_EDGE": kvb.W_GRID_EDGE, "KVB_W_FALLBACK": kvb.W_FALLBACK,
             "KVB_E_INVALID": kvb.E_INVALID, "KVB_E_NOMEM": kvb.E_NOMEM, "KVB_E_HIP": kvb.E_HIP,
             "KVB_E_UNSUPPORTED": kvb.E_UNSUPPORTED, "KVB_KNN_F32": kvb.KNN_F32, "KVB_KNN_BF16": kvb.KNN_BF16,
             "KVB_KNN_LEARNED": kvb.KNN_LEARNED, "KVB_BW_ADHOC": kvb.BW_ADHOC, "KVB_BW_DENSITY": kvb.BW_DENSITY,
             "KVB_OUT_MARKOV": kvb.OUT_MARKOV, "KVB_OUT_GENERATOR": kvb.OUT_GENERATOR,
             "KVB_OUT_SYMMETRIC": kvb.OUT_SYMMETRIC, "KVB_ROW_RECHECK": kvb.ROW_RECHECK,
             "KVB_ROW_FALLBACK": kvb.ROW_FALLBACK, "KVB_OPT_FORCE_FALLBACK": kvb.OPT_FORCE_FALLBACK,
             "KVB_OPT_SCRATCH_LIMIT": kvb.OPT_SCRATCH_LIMIT, "KVB_OPT_BF16_SPLIT": kvb.OPT_BF16_SPLIT,
             "KVB_OPT_N_PROBE": kvb.OPT_N_PROBE, "KVB_OPT_CURVE_ORDER": kvb.OPT_CURVE_ORDER,
             "KVB_OPT_PATTERN": kvb.OPT_PATTERN, "KVB_PATTERN_KNN": kvb.PATTERNS["knn"],
             "KVB_PATTERN_UNION": kvb.PATTERNS["union"], "KVB_ROW_UNCERTIFIED": kvb.ROW_UNCERTIFIED,
             "KVB_E_NOT_TRAINED": kvb.E_NOT_TRAINED, "KVB_E_IO": kvb.E_IO, "KVB_E_NO_DEVICE": kvb.E_NO_DEVICE,
             "KVB_W_NOT_CONVERGED": kvb.W_NOT_CONVERGED,
             "KVB_PROF_SLOTS": kvb.PROF_SLOTS}
    for k, v in pairs.items():
        assert consts[k] == v, k


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 exits with a message, before any
    GPU or library work."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.skipif(not os.path.exists(LIB), reason="libkvb.so not built")
def test_lanczos_prefix_rejects_non_finite_coefficients():
    """The host-side decision of kvb_eigsh on its tridiagonal (no device
    needed): it keeps the steps up to the first breakdown (beta = 0, an
    invariant subspace, whose Ritz pairs are exact) or all of them, and
    refuses a NaN or infinite coefficient instead of reading a NaN beta as a
    breakdown (a non-finite matrix would otherwise return NaN eigenvalues
    reported as converged)."""
    import ctypes
    import numpy as np
    from paper_2104_15124_amd import kvb
    L = kvb.load_library()

    def prefix(a, b):
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        m = ctypes.c_int32(-7)
        rc = L.kvb_lanczos_prefix(a.ctypes.data_as(ctypes.c_void_p), b.ctypes.data_as(ctypes.c_void_p),
                                  len(a), ctypes.byref(m))
        return rc, m.value

    assert prefix([1.0, 2.0, 3.0], [0.5, 0.25, 0.1]) == (kvb.OK, 3)
    assert prefix([1.0, 2.0, 3.0], [0.5, 0.0, np.nan]) == (kvb.OK, 2)      # breakdown at step 1
    assert prefix([1.0, 2.0, 3.0], [0.5, 1e-310, 0.3]) == (kvb.OK, 2)      # underflowed norm
    assert prefix([np.nan], [np.nan]) == (kvb.E_INVALID, 0)                 # NaN matrix: not a breakdown
    assert prefix([1.0, 2.0], [np.nan, 0.3]) == (kvb.E_INVALID, 0)
    assert prefix([1.0, np.inf, 3.0], [0.5, 0.5, 0.5]) == (kvb.E_INVALID, 1)
    assert prefix([1.0, 2.0, 3.0], [0.5, 0.5, np.inf]) == (kvb.E_INVALID, 2)
    assert prefix([1.0, 2.0], [-0.5, 0.5]) == (kvb.E_INVALID, 0)
    assert prefix([], []) [0] == kvb.E_INVALID


# ---------------------------------------------------------------- argument checks on a host-only context
@pytest.fixture
def host_ctx():
    if not os.path.exists(LIB):
        pytest.skip("libkvb.so not built")
    import ctypes
    from paper_2104_15124_amd import kvb
    L = kvb.load_library()
    h = ctypes.c_void_p()
    assert L.kvb_create_host(ctypes.byref(h)) == kvb.OK
    yield L, h, kvb
    L.kvb_destroy(h)


P = 4096   # an aligned placeholder device address (never read: the host-only context stops first)


def _err(L, h):
    return L.kvb_last_error(h).decode()


def test_host_context_knn_checks(host_ctx):
    L, h, kvb = host_ctx
    ok = dict(X=P, n=100000, m=16, k=64, mode=kvb.KNN_F32, margin=32, idx=P, d2=P, flags=0)

    def call(**kw):
        a = dict(ok, **kw)
        return L.kvb_knn(h, a["X"], a["n"], a["m"], a["k"], a["mode"], a["margin"], a["idx"], a["d2"], a["flags"])

    assert call() == kvb.E_NO_DEVICE
    assert call(m=3) == kvb.E_NO_DEVICE              # the direct path stops at its first device call too
    assert call(mode=kvb.KNN_BF16, m=64) == kvb.E_NO_DEVICE
    assert call(n=0) == kvb.E_INVALID and "n must be" in _err(L, h)
    assert call(k=0) == kvb.E_INVALID and "k must be" in _err(L, h)
    assert call(n=10, k=11) == kvb.E_INVALID
    assert call(m=0) == kvb.E_INVALID
    assert call(margin=-1) == kvb.E_INVALID and "margin" in _err(L, h)
    assert call(mode=7) == kvb.E_INVALID and "mode" in _err(L, h)
    assert call(X=0) == kvb.E_INVALID and "X must be" in _err(L, h)
    assert call(idx=P + 2) == kvb.E_INVALID and "idx" in _err(L, h)   # misaligned int32 pointer
    assert call(d2=0) == kvb.E_INVALID
    assert call(k=200, margin=100) == kvb.E_UNSUPPORTED and "256" in _err(L, h)
    assert call(m=2000) == kvb.E_UNSUPPORTED
    assert call(mode=kvb.KNN_LEARNED) == kvb.E_NOT_TRAINED


def test_host_context_pass_checks(host_ctx):
    L, h, kvb = host_ctx
    n, k = 100000, 64
    # bandwidth: ad-hoc needs 1 <= k0 < k; density needs finite positive e and d
    assert L.kvb_bandwidth(h, P, P, n, k, kvb.BW_ADHOC, 8, 0, 0.0, 0.0, 0.0, P, 0) == kvb.E_NO_DEVICE
    assert L.kvb_bandwidth(h, P, P, n, k, kvb.BW_ADHOC, k, 0, 0.0, 0.0, 0.0, P, 0) == kvb.E_INVALID
    assert L.kvb_bandwidth(h, P, P, n, k, kvb.BW_DENSITY, 8, P, 0.1, 2.0, -0.5, P, 0) == kvb.E_NO_DEVICE
    assert L.kvb_bandwidth(h, P, P, n, k, kvb.BW_DENSITY, 8, P, -0.1, 2.0, -0.5, P, 0) == kvb.E_INVALID
    assert L.kvb_bandwidth(h, P, P, n, k, kvb.BW_DENSITY, 8, P, 0.1, 0.0, -0.5, P, 0) == kvb.E_INVALID
    assert L.kvb_bandwidth(h, P, P, n, k, kvb.BW_DENSITY, 8, 0, 0.1, 2.0, -0.5, P, 0) == kvb.E_INVALID
    # tuning: 3 <= G <= 256, 0 < e_min < e_max
    import ctypes
    e = ctypes.c_double()
    dim = ctypes.c_double()
    for fn in (L.kvb_tune_eps, L.kvb_tune_eps_noalloc):
        assert fn(h, P, P, P, n, k, 1e-3, 10.0, 64, 0, ctypes.byref(e), ctypes.byref(dim)) == kvb.E_NO_DEVICE
        assert fn(h, P, P, P, n, k, 1e-3, 10.0, 2, 0, ctypes.byref(e), ctypes.byref(dim)) == kvb.E_INVALID
        assert fn(h, P, P, P, n, k, 10.0, 1e-3, 64, 0, ctypes.byref(e), ctypes.byref(dim)) == kvb.E_INVALID
        assert fn(h, P, P, P, n, 300, 1e-3, 10.0, 64, 0, ctypes.byref(e), ctypes.byref(dim)) == kvb.E_INVALID
        assert fn(h, P, P, P, n, k, 1e-3, 10.0, 64, 0, None, ctypes.byref(dim)) == kvb.E_INVALID
    # assembly: out_kind in {Markov, generator, symmetric}, e > 0, d > 0
    assert L.kvb_assemble_csr(h, P, P, P, n, k, 0.01, -1.0, 2.0, kvb.OUT_MARKOV, P, P, P, 0, 0) == kvb.E_NO_DEVICE
    assert L.kvb_assemble_csr(h, P, P, P, n, k, 0.01, -1.0, 2.0, 9, P, P, P, 0, 0) == kvb.E_INVALID
    assert L.kvb_assemble_csr(h, P, P, P, n, k, 0.0, -1.0, 2.0, kvb.OUT_MARKOV, P, P, P, 0, 0) == kvb.E_INVALID
    assert L.kvb_assemble_csr(h, P, P, P, n, k, 0.01, -1.0, 2.0, kvb.OUT_MARKOV, 0, P, P, 0, 0) == kvb.E_INVALID


def test_host_context_build_and_partitioner_checks(host_ctx):
    L, h, kvb = host_ctx

    def build(**kw):
        a = dict(n=100000, m=16, k=64, mode=kvb.KNN_F32, margin=32, k0=8, G=64, out_kind=kvb.OUT_MARKOV,
                 e_min=1e-3, e_max=10.0, d=4.0)
        a.update(kw)
        return L.kvb_build(h, P, a["n"], a["m"], a["k"], a["mode"], a["margin"], a["k0"], a["d"], -1.0, -0.5,
                           a["e_min"], a["e_max"], a["G"], a["out_kind"], P, P, 0, P, P, 0, P, P, P, 0, 0, 0, 0, 0)

    assert build() == kvb.E_NO_DEVICE
    assert build(k0=64) == kvb.E_INVALID and "k0" in _err(L, h)
    assert build(G=1) == kvb.E_INVALID
    assert build(out_kind=5) == kvb.E_INVALID
    assert build(n=0) == kvb.E_INVALID
    assert build(d=0.0) == kvb.E_INVALID
    assert build(k=200, margin=100) == kvb.E_UNSUPPORTED
    # options are host state: they work on a host-only context
    assert L.kvb_set_option(h, kvb.OPT_SCRATCH_LIMIT, 1 << 20) == kvb.OK
    assert L.kvb_set_option(h, kvb.OPT_SCRATCH_LIMIT, -1) == kvb.E_INVALID
    assert L.kvb_set_option(h, 999, 0) == kvb.E_INVALID
    # the partitioner: shape checks, then no device
    assert L.kvb_part_init(h, 16, 256, 256, 1024, 4, 1) == kvb.E_NO_DEVICE
    assert L.kvb_part_init(h, 16, 250, 256, 1024, 4, 1) == kvb.E_INVALID
    assert L.kvb_part_init(h, 16, 256, 256, 1024, 64, 1) == kvb.E_INVALID
    assert L.kvb_part_route(h, P, 1000, P, P) == kvb.E_NOT_TRAINED
    assert L.kvb_profile_enable(h, 1) == kvb.E_NO_DEVICE
