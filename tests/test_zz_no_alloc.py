"""The allocation-free entry point kvb_tune_eps_noalloc against kvb_tune_eps
(run on an MI355X): the same tuning sums, optimum and dimension estimate, bit
for bit, on two calls in a row, the second on a smaller input; and it runs in
a context whose scratch limit forbids the allocating entry point's scratch."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
from parity import say

pytestmark = pytest.mark.gpu


def noalloc_tune(kvb, ctx, idx, d2, rho, e_min, e_max, G):
    n, k = d2.shape
    chi = np.zeros(G, dtype=np.float64)
    es, dm = ctypes.c_double(), ctypes.c_double()
    rc = ctx.check(ctx.lib.kvb_tune_eps_noalloc(ctx.h, kvb._ptr(idx), kvb._ptr(d2), kvb._ptr(rho), n, k, e_min,
                                                 e_max, G, chi.ctypes.data_as(ctypes.c_void_p), ctypes.byref(es),
                                                 ctypes.byref(dm)))
    return rc, chi, es.value, dm.value


def test_tune_eps_noalloc_matches_tune_eps(gpu_lib):
    kvb = gpu_lib
    ctx = kvb.Context()
    for n, k, G, seed in ((300_000, 64, 64, 1), (2_500, 16, 40, 2)):
        say(f"[noalloc] n={n} k={k} G={G}")
        X = workloads.torus(n, seed=seed)
        Xd = torch.from_numpy(X).cuda()
        idx, d2, _ = kvb.knn(Xd, k, "f32", 8, ctx)
        b = kvb.bandwidth_adhoc(d2, 8, ctx)
        ref = kvb.tune_eps(idx, d2, b, 1e-3, 10.0, G, ctx)
        rc, chi, e_star, dim = noalloc_tune(kvb, ctx, idx, d2, b, 1e-3, 10.0, G)
        assert (rc == kvb.W_GRID_EDGE) == ref.edge
        np.testing.assert_array_equal(chi, ref.chi)
        assert e_star == ref.e_star and dim == ref.dim
    # a fresh context whose scratch limit forbids any scratch: the allocating
    # entry point fails, the allocation-free one still answers
    c2 = kvb.Context()
    c2.set_option(kvb.OPT_SCRATCH_LIMIT, 1)
    with pytest.raises(kvb.KvbError) as e:
        kvb.tune_eps(idx, d2, b, 1e-3, 10.0, G, c2)
    assert e.value.code == kvb.E_NOMEM
    rc, chi2, e2, d2_ = noalloc_tune(kvb, c2, idx, d2, b, 1e-3, 10.0, G)
    np.testing.assert_array_equal(chi2, ref.chi)
    assert e2 == ref.e_star and d2_ == ref.dim
    with pytest.raises(kvb.KvbError) as e:
        noalloc_tune(kvb, c2, idx, d2, b, 1e-3, 10.0, 257)
    assert e.value.code == kvb.E_INVALID
    c2.close()
    ctx.close()
