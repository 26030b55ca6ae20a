"""The C-ABI library loads without a GPU and exports every declared symbol.

No compute call is made here: this container has no GPU, and the library has
no CPU path by design.
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
             "KVB_E_NOT_TRAINED": kvb.E_NOT_TRAINED, "KVB_E_IO": kvb.E_IO,
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
