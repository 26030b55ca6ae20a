"""Failure modes the host can force (run on an MI355X): a scratch limit below
what a call needs, and a tuning grid that excludes the optimum. Every kernel
still runs to its normal end; the conditions come from the host."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from parity import check_knn_rows, knn_reference, say

pytestmark = pytest.mark.gpu


def test_scratch_limit_returns_nomem_and_context_recovers(gpu_lib):
    """KVB_OPT_SCRATCH_LIMIT below a call's scratch need: the call fails with
    KVB_E_NOMEM before any work is enqueued, names the limit, and the same
    context then runs the call normally once the limit is lifted."""
    kvb = gpu_lib
    X = workloads.gaussian_iid(4000, 16, seed=2)
    Xd = torch.from_numpy(X).cuda()
    ctx = kvb.Context()
    say("[failure] scratch limit 4096 bytes")
    ctx.set_option(kvb.OPT_SCRATCH_LIMIT, 4096)
    for mode in ("f32", "bf16"):
        with pytest.raises(kvb.KvbError) as e:
            kvb.knn(Xd, 32, mode, 32, ctx)
        assert e.value.code == kvb.E_NOMEM
        assert "limit" in str(e.value)
    with pytest.raises(kvb.KvbError) as e:
        kvb.build(Xd, 32, 8, 4.0, -1.0, -0.5, ctx=ctx)
    assert e.value.code == kvb.E_NOMEM
    with pytest.raises(kvb.KvbError):
        ctx.set_option(kvb.OPT_SCRATCH_LIMIT, -1)
    ctx.set_option(kvb.OPT_SCRATCH_LIMIT, 0)          # unlimited
    idx, d2, _ = kvb.knn(Xd, 32, "f32", 32, ctx)
    torch.cuda.synchronize()
    ri, rd = knn_reference(X, 32)
    check_knn_rows(idx.cpu().numpy(), d2.cpu().numpy(), ri, rd, 32, np.arange(len(X)))
    # a limit above what is already held is no obstacle
    ctx.set_option(kvb.OPT_SCRATCH_LIMIT, 1 << 40)
    r = kvb.build(Xd, 32, 8, 4.0, -1.0, -0.5, ctx=ctx)
    assert torch.equal(r.idx, idx)
    ctx.close()
    say("[failure] scratch limit: ok")


def test_grid_excluding_the_optimum_warns_grid_edge(gpu_lib):
    """Section 2.3 tuning on a grid that lies entirely below (or above) the
    bandwidth where the log-slope of chi peaks: the slope rises (falls) across
    the grid, so its last (first) value is the largest, the call returns
    KVB_W_GRID_EDGE and e* is that end of the grid, exactly as the oracle
    decides on the same inputs."""
    kvb = gpu_lib
    w = workloads.WORKLOADS["sphere2_n2000"]
    X = workloads.make(w.name, seed=0)
    Xd = torch.from_numpy(X).cuda()
    idx, d2, _ = kvb.knn(Xd, w.k, "f32", w.margin)
    b = kvb.bandwidth_adhoc(d2, w.k0)
    pat = oracle.Pattern.from_knn(idx.cpu().numpy(), d2.cpu().numpy().astype(np.float64))
    bh = b.cpu().numpy().astype(np.float64)
    # the optimum of the density stage is near e = 0.17 on this workload
    for lo, hi, g_end in ((1e-3, 5e-2, w.G - 2), (1.0, 1e2, 0)):
        say(f"[failure] grid [{lo:g}, {hi:g}]")
        t = kvb.tune_eps(idx, d2, b, lo, hi, w.G)
        ref = oracle.chi(pat, bh, lo, hi, w.G)
        assert ref.edge and ref.g_star == g_end
        assert t.edge
        assert t.e_star == pytest.approx(ref.e_star, rel=1e-13)
        r = kvb.build(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, lo, hi, w.G, mode="f32", margin=w.margin)
        assert r.status == kvb.W_GRID_EDGE and r.tune_a.edge
        assert r.tune_a.e_star == pytest.approx(ref.e_star, rel=1e-13)
    # the configured grid holds both optima inside: no warning
    r = kvb.build(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, mode="f32", margin=w.margin)
    assert r.status == kvb.OK and not r.tune_a.edge and not r.tune_b.edge
