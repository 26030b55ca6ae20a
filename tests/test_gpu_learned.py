"""GPU tests of the learned partitioner and the routed k-NN search (MI355X).

* MLP forward logits and backward gradients against the float64 oracle with
  the same bfloat16 cast points (parameters and inputs drawn on the host).
* One Adam step against the oracle's update.
* Teacher labels bit-exact against the oracle.
* Routing decisions equal wherever the oracle's logit gaps exceed the
  forward tolerance.
* Routed search probing every bucket equals the exact oracle k-NN.
* Training gain: the trained partitioner keeps recall against the exact
  search high while its probed buckets hold a small share of the samples,
  with at least twice the recall per scanned candidate of an untrained one.
* Save / load round trip and argument errors.
"""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import learned as OL
from parity import check_knn_rows, knn_reference, say

pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-4   # norm-wise, logits and gradients


def _ctx(kvb):
    return kvb.Context()


def _setup(kvb, m, h1, h2, nb, P, seed):
    ctx = _ctx(kvb)
    kvb.part_init(m, h1, h2, nb, P, seed, ctx)
    params = OL.init_params(m, h1, h2, nb, seed=seed + 100)
    kvb.part_set_params(torch.from_numpy(OL.flatten(params).astype(np.float32)).cuda(), ctx)
    return ctx, params


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


MLP_CASES = [
    # (name, m, h1, h2, nb, B, ks)
    ("c4_shape", 128, 256, 256, 1024, 256, 128),
    ("c5_shape", 16, 256, 256, 1024, 128, 64),
    ("ragged_m", 37, 64, 96, 64, 96, 9),
]


@pytest.mark.parametrize("name,m,h1,h2,nb,B,ks", MLP_CASES, ids=[c[0] for c in MLP_CASES])
def test_mlp_forward_backward_parity(gpu_lib, name, m, h1, h2, nb, B, ks):
    say(f"[mlp] {name}: m={m} h1={h1} h2={h2} nb={nb} B={B} ks={ks}")
    kvb = gpu_lib
    ctx, params = _setup(kvb, m, h1, h2, nb, 4, seed=len(name))
    rng = np.random.default_rng(7)
    X = rng.standard_normal((B, m)).astype(np.float32)
    lab = rng.integers(0, nb, size=(B, ks)).astype(np.int32)
    # labels concentrated on a few buckets per row, like neighbour histograms
    lab[:, : ks // 2] = lab[:, :1]
    Xd = torch.from_numpy(X).cuda()
    Z = kvb.mlp_forward(Xd, nb, ctx).cpu().numpy()
    ref = OL.forward(params, X, cast=True)["Z"]
    assert _rel(Z, ref) <= FWD_RTOL, _rel(Z, ref)
    loss, g = kvb.mlp_backward(Xd, torch.from_numpy(lab).cuda(), ctx)
    rloss, rg = OL.backward(params, X, lab, cast=True)
    assert abs(loss - rloss) <= 1e-5 * abs(rloss)
    g = g.cpu().numpy()
    o = 0
    for t, r in zip(("dW1", "db1", "dW2", "db2", "dW3", "db3"), rg):
        part = g[o:o + r.size].reshape(r.shape)
        o += r.size
        assert _rel(part, r) <= FWD_RTOL, (t, _rel(part, r))
    assert o == g.size
    # the parameters are not changed by the hooks
    got = kvb.part_get_params(ctx).cpu().numpy()
    assert np.array_equal(got, OL.flatten(params).astype(np.float32))
    ctx.close()


def test_adam_one_step(gpu_lib):
    kvb = gpu_lib
    m, h1, h2, nb, B, ks, lr = 24, 64, 64, 64, 64, 8, 1e-3
    ctx, params = _setup(kvb, m, h1, h2, nb, 2, seed=3)
    rng = np.random.default_rng(8)
    X = rng.standard_normal((B, m)).astype(np.float32)
    labels = rng.integers(0, nb, size=B).astype(np.int32)
    idx_s = np.stack([rng.permutation(B)[:ks] for _ in range(B)]).astype(np.int32)
    loss = kvb.part_train(torch.from_numpy(X).cuda(), torch.from_numpy(labels).cuda(),
                          torch.from_numpy(idx_s).cuda(), epochs=1, batch=B, lr=lr, seed=1, ctx=ctx)
    p1 = kvb.part_get_params(ctx).cpu().numpy().astype(np.float64)
    nbr = labels[idx_s]
    rloss, rg = OL.backward(params, X, nbr, cast=True)
    assert abs(loss[0] - rloss) <= 1e-5 * abs(rloss)
    p0 = OL.flatten(params)
    g = OL.flatten(rg)
    want, _, _ = OL.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    # the first Adam step moves each parameter by about lr * sign(g); where |g| is
    # at the level of rounding noise the sign is not determined
    clear = np.abs(g) > 1e-4 * np.sqrt(np.mean(g * g)) + 1e-6
    assert clear.mean() > 0.5
    assert np.max(np.abs((p1 - want)[clear])) <= 2e-3 * lr + 1e-7
    assert np.all(np.abs(p1 - p0) <= lr * 1.001 + 1e-7)
    ctx.close()


TEACHER_CASES = [("n5000_m16_l6", 5000, 16, 6, 1), ("n777_m3_l5", 777, 3, 5, 2), ("n40000_m128_l10", 40000, 128, 10, 3)]


@pytest.mark.parametrize("name,ns,m,levels,seed", TEACHER_CASES, ids=[c[0] for c in TEACHER_CASES])
def test_teacher_bit_exact(gpu_lib, name, ns, m, levels, seed):
    say(f"[teacher] {name}")
    kvb = gpu_lib
    X = workloads.gaussian_iid(ns, m, seed=seed)
    lab = kvb.part_teacher(torch.from_numpy(X).cuda(), levels, seed).cpu().numpy()
    ref = OL.teacher_labels(X, levels, seed)
    assert np.array_equal(lab, ref)


def test_routing_decisions(gpu_lib):
    kvb = gpu_lib
    m, h1, h2, nb, P, n = 32, 128, 128, 256, 4, 3000
    ctx, params = _setup(kvb, m, h1, h2, nb, P, seed=5)
    X = workloads.gaussian_iid(n, m, seed=9)
    home, probe = kvb.part_route(torch.from_numpy(X).cuda(), P, ctx)
    home, probe = home.cpu().numpy(), probe.cpu().numpy()
    assert np.array_equal(home, probe[:, 0])
    assert all(len(set(r)) == P for r in probe)
    Z = OL.forward(params, X, cast=True)["Z"]
    tol = 2 * FWD_RTOL * np.sqrt(np.mean(Z * Z)) * 10
    s = -np.sort(-Z, axis=1)
    gaps = -np.diff(s[:, : P + 1], axis=1)
    clear = (gaps > tol).all(axis=1)
    assert clear.mean() > 0.9
    want = OL.top_buckets(Z, P)
    assert np.array_equal(probe[clear], want[clear])
    ctx.close()


ALLPROBE_CASES = [
    # (name, n, m, k, margin, nb, split)
    ("n3000_m64_k32", 3000, 64, 32, 32, 32, 3),
    ("n1037_m20_k17", 1037, 20, 17, 16, 32, 3),
    ("n2500_m16_k64_split6", 2500, 16, 64, 32, 32, 6),
]


@pytest.mark.parametrize("name,n,m,k,margin,nb,split", ALLPROBE_CASES, ids=[c[0] for c in ALLPROBE_CASES])
def test_routed_search_probing_every_bucket_is_exact(gpu_lib, name, n, m, k, margin, nb, split):
    say(f"[routed-all] {name}")
    kvb = gpu_lib
    ctx = _ctx(kvb)
    ctx.set_option(kvb.OPT_BF16_SPLIT, split)
    kvb.part_init(m, 64, 64, nb, nb, 11, ctx)
    X = workloads.gaussian_iid(n, m, seed=n)
    idx, d2, flags = kvb.knn(torch.from_numpy(X).cuda(), k, mode="learned", margin=margin, ctx=ctx)
    idx, d2, flags = idx.cpu().numpy(), d2.cpu().numpy(), flags.cpu().numpy()
    assert (flags & kvb.ROW_UNCERTIFIED).all()
    ri, rd = knn_reference(X, k)
    check_knn_rows(idx, d2, ri, rd, k, np.arange(n))
    ctx.close()


def _recall_on(kvb, X, k, idx_exact, ctx):
    idx, _, flags = kvb.knn(X, k, mode="learned", margin=32, ctx=ctx)
    torch.cuda.synchronize()
    return OL.recall(idx.cpu().numpy()[:, 1:], idx_exact[:, 1:]), flags.cpu().numpy()


def _candidate_fraction(kvb, X, nb, P, ctx):
    """Mean over queries of the share of all samples held by its probed buckets."""
    home, probe = kvb.part_route(X, P, ctx)
    sizes = torch.bincount(home.long(), minlength=nb).double()
    return float(sizes[probe.long()].sum()) / float(X.shape[0]) ** 2


def test_training_gain_and_recall(gpu_lib, tmp_path):
    kvb = gpu_lib
    wl = workloads.WORKLOADS["sphere3_n4m"]
    n, k, nb, P = 60_000, 32, 64, 4
    X = torch.from_numpy(workloads.make("sphere3_n4m", seed=0, n=n)).cuda()
    ctx = _ctx(kvb)
    exact, _, _ = kvb.knn(X, k, mode="bf16", margin=32, ctx=ctx)
    exact = exact.cpu().numpy()
    # untrained partitioner with the same shape
    kvb.part_init(wl.m, 256, 256, nb, P, 1, ctx)
    r0, _ = _recall_on(kvb, X, k, exact, ctx)
    c0 = _candidate_fraction(kvb, X, nb, P, ctx)
    losses = kvb.train_partitioner(X, k, n_train=n, levels=6, n_probe=P, epochs=8, batch=512, lr=2e-3,
                                   seed=1, ctx=ctx)
    say(f"[train] losses {np.round(losses, 4).tolist()}")
    assert losses[-1] < losses[0]
    r1, flags = _recall_on(kvb, X, k, exact, ctx)
    c1 = _candidate_fraction(kvb, X, nb, P, ctx)
    say(f"[train] untrained recall {r0:.4f} candidates {c0:.4f}; trained recall {r1:.4f} candidates {c1:.4f}")
    assert (flags & kvb.ROW_UNCERTIFIED).all()
    # the gain: high recall while scanning a small share of the samples, and at
    # least twice the recall per scanned candidate of the untrained partition
    assert r1 >= 0.97
    assert c1 <= 3.0 * P / nb
    assert r1 / c1 >= 2.0 * r0 / c0
    # save / load round trip: a second context routes identically
    path = os.path.join(tmp_path, "part.bin")
    kvb.part_save(path, ctx)
    ctx2 = _ctx(kvb)
    kvb.part_load(path, ctx2)
    h1, p1 = kvb.part_route(X, 4, ctx)
    h2, p2 = kvb.part_route(X, 4, ctx2)
    assert torch.equal(p1, p2) and torch.equal(h1, h2)
    assert torch.equal(kvb.part_get_params(ctx), kvb.part_get_params(ctx2))
    ctx.close()
    ctx2.close()


def test_learned_argument_errors(gpu_lib):
    kvb = gpu_lib
    ctx = _ctx(kvb)
    X = torch.zeros((64, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(kvb.KvbError) as e:
        kvb.knn(X, 4, mode="learned", ctx=ctx)
    assert e.value.code == kvb.E_NOT_TRAINED
    with pytest.raises(kvb.KvbError) as e:
        kvb.part_init(8, 48, 64, 64, 4, 0, ctx)        # h1 not a multiple of 32
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.part_init(8, 64, 64, 64, 65, 0, ctx)       # n_probe > n_buckets
    assert e.value.code == kvb.E_INVALID
    kvb.part_init(8, 64, 64, 64, 4, 0, ctx)
    with pytest.raises(kvb.KvbError) as e:
        kvb.knn(torch.zeros((64, 9), dtype=torch.float32, device="cuda"), 4, mode="learned", ctx=ctx)
    assert e.value.code == kvb.E_INVALID
    with pytest.raises(kvb.KvbError) as e:
        kvb.part_load("/nonexistent/part.bin", ctx)
    assert e.value.code == kvb.E_IO
    ctx.close()


RECALL_CASES = [
    # (workload recipe, n, buckets (2^levels), k): about 3000-6000 samples per
    # bucket, as at the full configurations (4M / 1024, 8M / 1024)
    ("sphere3_n4m", 400_000, 128, 128),
    ("gmm_n8m", 800_000, 128, 64),
]


@pytest.mark.parametrize("name,n,nb,k", RECALL_CASES, ids=[c[0] for c in RECALL_CASES])
def test_learned_recall_judged_by_oracle(gpu_lib, name, n, nb, k):
    """The learned search at its configured top-4 probe (and at top-8) on a
    reduced-n draw of the recipe, trained as configured (200k-sample
    subsample, neighbour-histogram targets). Recall is judged by the FP64
    oracle's exact k-NN of 1024 random rows; the search is also compared with
    the exact curve-ordered scan on the same samples (time and scored pairs).
    The top-4 probe stays below the 0.999 recall bar on these recipes (about
    0.99-0.997); top-8 reaches it."""
    import time
    kvb = gpu_lib
    w = workloads.WORKLOADS[name]
    X = workloads.make(name, seed=3, n=n)
    Xd = torch.from_numpy(X).cuda()
    rows = np.sort(np.random.default_rng(5).choice(n, 1024, replace=False))
    say(f"[learned-recall] {name}: n={n} m={w.m} k={k} buckets={nb}; oracle rows {len(rows)}")
    rfull, dfull = knn_reference(X, k, rows)
    ri = rfull[:, :k]
    ctx = _ctx(kvb)
    # the exact scan on the same samples
    kvb.knn(Xd, k, mode="bf16", margin=32, ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ex, exd, _ = kvb.knn(Xd, k, mode="bf16", margin=32, ctx=ctx)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t0
    pairs_exact = kvb.knn_pairs(ctx)
    check_knn_rows(ex.cpu().numpy()[rows], exd.cpu().numpy()[rows], rfull, dfull, k, rows)
    levels = int(np.log2(nb))
    kvb.train_partitioner(Xd, k, n_train=min(n, 200_000), levels=levels, h1=256, h2=256, n_probe=4, epochs=10,
                          batch=512, lr=2e-3, seed=3, ctx=ctx)
    out = {}
    for P in (4, 8):
        ctx.set_option(kvb.OPT_N_PROBE, P)
        kvb.knn(Xd, k, mode="learned", margin=32, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx, _, flags = kvb.knn(Xd, k, mode="learned", margin=32, ctx=ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        got = idx.cpu().numpy()[rows]
        rec = OL.recall(got[:, 1:], ri[:, 1:])
        out[P] = (rec, dt, kvb.knn_pairs(ctx))
        say(f"[learned-recall] {name}: top-{P} recall {rec:.5f}, {dt * 1e3:.1f} ms, pairs {out[P][2]:.4g}; "
            f"exact scan {t_exact * 1e3:.1f} ms, pairs {pairs_exact:.4g}")
        assert (flags.cpu().numpy() & kvb.ROW_UNCERTIFIED).all()
    assert out[4][0] >= 0.985
    assert out[8][0] >= 0.999
    assert out[8][0] >= out[4][0]
    ctx.close()
