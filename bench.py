"""Throughput of the sparse kernel-matrix build on one MI355X.

One step = the whole hot path on one batch of samples already resident in HBM:
k-NN -> ad-hoc bandwidth -> e tuning (density kernel) -> density / rho ->
grid scale -> e tuning (operator kernel) -> q, Kt, D, Markov CSR.

The default workload is the largest one that fits one GPU: 8M samples of a
3-component Gaussian mixture on a 4-D subspace of R^16, k = 64. Its primary
form (the line's `value`) is the plain FP32 form (FP32 distance tiles, exact
k-NN sets); the BF16-tile form (exact, certified, margin 32) and the learned
partitioner form (recall reported) run on the same samples and are reported in
the same line under "forms".

Prints ONE JSON line on stdout; per-kernel details go to stderr.
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published figures: 256 CUs x 64 lanes x 2.4 GHz for unpacked FP32
# lane operations (the vendor's 157.3 TFLOP/s FP32 vector figure counts packed
# FMAs, two lanes' worth of flops each), HBM3E 8 TB/s, dense MFMA 2.5 PFLOP/s
# BF16 and 157.3 TFLOP/s FP32
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}

DEFAULT_FORMS = {"gmm_n8m": ("f32", ("bf16", "learned"))}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(workload: str, kernel: str, mode: str):
    """HBM bytes per launch from the committed counter runs (profiles/traffic.txt),
    or None when there are none for this kernel or its sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#") or f[0] != f"{workload}:{mode}" or f[1] != kernel:
            continue
        h = hashlib.sha256()
        for src in f[2].split("+"):
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest()[:16] != f[3]:
            log(f"  traffic: the counters in profiles/{f[6]} predate changes to {f[2]}; not reported")
            return None
        return int(f[4]) + int(f[5])
    return None


def measure_peaks(kvb, ctx):
    """The build's own microbenchmarks of the resources it is bound by."""
    out = {}
    for key, kind, scale in (("hbm_GB/s", kvb.PEAK_HBM_COPY, 1e9), ("mfma_bf16_TFLOP/s", kvb.PEAK_MFMA_BF16, 1e12),
                             ("mfma_f32_TFLOP/s", kvb.PEAK_MFMA_F32, 1e12), ("exp_per_s", kvb.PEAK_EXP, 1.0),
                             ("valu_Tlane-op/s", kvb.PEAK_VALU_FMA, 1e12)):
        rate, _ = kvb.peak_probe(kind, ctx)
        out[key] = float(f"{rate / scale:.5g}")
    log("  measured peaks: " + ", ".join(f"{k} {v}" for k, v in out.items()))
    return out


def select_roofline(w, mode, pairs, sel_avg_s, peaks, learned, traffic):
    """Roofline of the distance tiles + selection: algorithmic work = the
    candidate pairs the tiles scored (after the spatial pruning or the learned
    routing) times the work per pair."""
    if mode == "f32" and w.m <= 8:
        ops = 2 * w.m + 1      # m subtractions, m multiply(-add)s, 1 threshold compare
        ach = pairs * ops / sel_avg_s / 1e12
        meas = peaks.get("valu_Tlane-op/s") if peaks else None
        return {"kernel": "knn_select", "bound": "alu", "achieved": round(ach, 3), "peak": round(ALU_PEAK_TOPS, 3),
                "unit": "TOP/s", "frac": round(ach / ALU_PEAK_TOPS, 4),
                "measured_peak": meas, "frac_measured": round(ach / meas, 4) if meas else None,
                "traffic": traffic, "avg_ms": round(sel_avg_s * 1e3, 4),
                "work": f"{ops} VALU lane-ops per scored candidate pair, {pairs:.4g} pairs per launch "
                        f"(the pairs the bounding-box scan did not skip)"}
    prec = "f32" if mode == "f32" else "bf16"
    flops = 2 * w.m          # the algorithmic contraction y_i . y_j
    ach = pairs * flops / sel_avg_s / 1e12
    peak = MFMA_PEAK_TFLOPS[prec]
    meas = peaks.get(f"mfma_{prec}_TFLOP/s") if peaks else None
    # the epilogue: one threshold compare per scored pair on the vector ALUs
    valu = pairs / sel_avg_s / 1e12
    vmeas = peaks.get("valu_Tlane-op/s") if peaks else None
    what = ("routed query-candidate pairs, all probe passes" if learned
            else "the pairs the curve-ordered scan did not skip")
    return {"kernel": "knn_select", "bound": "mfma", "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ach / peak, 5), "measured_peak": meas, "frac_measured": round(ach / meas, 5) if meas else None,
            "traffic": traffic, "avg_ms": round(sel_avg_s * 1e3, 4),
            "epilogue_frac": round(valu / (vmeas or ALU_PEAK_TOPS), 5),
            "work": f"{flops} algorithmic flops per scored candidate pair (2m, {prec} MFMA), {pairs:.4g} pairs per "
                    f"launch ({what}); epilogue_frac: one compare per pair against the VALU lane rate"}


def pass_rooflines(w, prof, r, nnz, base_nnz, csr, union, delta, peaks):
    """The O(nk) passes against the HBM roofline: algorithmic bytes per launch
    (each stored entry: d2 4 B + idx 4 B + the gathered rho_j / q_j 4 B)."""
    nk = float(w.n) * w.k
    kp = min(w.k + w.margin, w.n)
    rows8 = float(w.n) * 8 if csr else 0.0                         # rowptr reads of the CSR passes
    # after a curve-ordered k-NN the passes run on curve-ordered rows, and the
    # assemble pass reads the sample ids of its output row as well
    curve_rows = prof.get("curve_rows", (0.0, 0))[1] > 0
    pass_bytes = {
        "knn_refine": float(w.n) * kp * (w.m * 4 + 8) + nk * 8,    # candidate rows + keys, idx/d2 out
        "adhoc_bandwidth": float(w.n) * (w.k0 * 4 + 4),
        "chi_tuning": base_nnz * 12 + float(w.n) * 4 + rows8 + (base_nnz * 4 if csr else 0.0),   # + row ids
        "density": nnz * 12 + float(w.n) * 12 + rows8,
        "q_pass": nnz * 12 + float(w.n) * 12 + rows8,
        # entries in / CSR out (the union pattern's columns are already written), P and D
        "assemble": nnz * (16 + (4 if csr else 8) + (4 if curve_rows else 0)) + float(w.n) * (16 + 4 * curve_rows) + rows8,
        # idx/d2 rows in, the neighbours' curve positions gathered, idx/d2 out; the bandwidths and the row map
        "curve_rows": nk * 20 + float(w.n) * 8,
    }
    if union:
        pass_bytes["union_pattern"] = nk * 8 + nnz * 8 + float(w.n + 1) * 8
    if delta > 0:
        pass_bytes["truncate"] = 2 * base_nnz * 12 + 2 * nnz * 8 + float(w.n) * 32
    hbm_meas = peaks.get("hbm_GB/s") if peaks else None
    passes = {}
    for name, byt in pass_bytes.items():
        ms, cnt = prof.get(name, (0.0, 0))
        if not cnt:
            continue
        sec = ms / cnt / 1e3
        gbs = byt / sec / 1e9
        passes[name] = {"avg_ms": round(sec * 1e3, 4), "bytes": int(byt), "GB/s": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "frac_measured": round(gbs / hbm_meas, 4) if hbm_meas else None}
    if "chi_tuning" in passes:
        # G exponentials per stored entry
        exps = base_nnz * w.G / (passes["chi_tuning"]["avg_ms"] / 1e3)
        passes["chi_tuning"]["exp_per_s"] = float(f"{exps:.4g}")
        if peaks and peaks.get("exp_per_s"):
            passes["chi_tuning"]["exp_frac_measured"] = round(exps / peaks["exp_per_s"], 4)
    return passes


def run_form(kvb, ctx, Xd, w, mode, steps, warmup, args, peaks, learned=None, passes=False):
    """Warm-up, then `steps` timed builds enqueued back to back (bracketed by
    device synchronisation), with per-kernel event timing."""
    import numpy as np
    import torch

    prev = [None]
    delta = args.delta
    pattern = args.pattern

    def step():
        # outputs preallocated: each step reuses the previous step's device
        # arrays; the build is only enqueued and its tuning results are read
        # once, after the timed region
        prev[0] = kvb.build(Xd, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G,
                            mode=mode, margin=w.margin, ctx=ctx, out=prev[0], sync=False, pattern=pattern,
                            delta=delta, out_kind=kvb.OUT_SYMMETRIC if args.eigs else kvb.OUT_MARKOV)
        return prev[0]

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    tune_a, _, tune_b, fb = kvb.build_info(w.G, ctx)
    ms_per_step = (t1 - t0) * 1e3 / steps
    log(f"bench: form {mode}: {ms_per_step:.3f} ms/step over {steps} steps ({w.n / (ms_per_step / 1e3):.4g} rows/s)")
    for name, (ms, cnt) in sorted(prof.items(), key=lambda kv: -kv[1][0]):
        if cnt:
            log(f"  {name:16s} {ms / cnt:9.4f} ms/launch  x{cnt // steps}/step  "
                f"{100 * ms / ((t1 - t0) * 1e3):5.1f}% of wall")
    log(f"  fallback rows {fb}, e_A={tune_a.e_star:.5g}, e_B={tune_b.e_star:.5g}, "
        f"dim_A={tune_a.dim:.3f}, dim_B={tune_b.dim:.3f}")
    sel_ms, sel_cnt = prof["knn_select"]
    pairs = kvb.knn_pairs(ctx)
    log(f"  knn pairs scored {pairs:.4g} ({pairs / (float(w.n) ** 2):.4%} of n^2)")
    traffic = measured_traffic(w.name, "knn_select", mode) if not args.n else None
    roof = select_roofline(w, mode, pairs, sel_ms / sel_cnt / 1e3, peaks, learned, traffic)
    out = {"mode": mode, "value": round(w.n / (ms_per_step / 1e3), 1), "unit": "rows/s",
           "ms_per_step": round(ms_per_step, 4), "steps": steps, "warmup": warmup, "fallback_rows": fb,
           "pairs_scored": float(f"{pairs:.4g}"), "roofline": roof,
           "e_A": tune_a.e_star, "e_B": tune_b.e_star}
    if passes:
        union = pattern == "union"
        csr = union or delta > 0
        nk = float(w.n) * w.k
        nnz = float(r.rowptr[-1].item()) if csr else nk
        base_nnz = nk if not union else (nnz if delta <= 0 else float(kvb.union_pattern(r.idx, r.d2, ctx).nnz))
        out["passes"] = pass_rooflines(w, prof, r, nnz, base_nnz, csr, union, delta, peaks)
        out["nnz"] = int(nnz)
        log("  passes: " + ", ".join(f"{k} {v['GB/s']} GB/s ({100 * v['frac']:.1f}% HBM)"
                                     for k, v in out["passes"].items()))
    if learned is not None:
        # recall judged on sampled rows by the exact float64 row search
        home, probe = kvb.part_route(Xd, learned["n_probe"], ctx)
        sizes = torch.bincount(home.long(), minlength=1024).double()
        learned["candidate_share"] = round(float(sizes[probe.long()].sum()) / float(w.n) ** 2, 5)
        learned["largest_bucket"] = int(sizes.max())
        g = torch.Generator().manual_seed(args.seed + 1)
        rows = torch.randperm(w.n, generator=g)[: args.recall_rows].to(torch.int32).cuda()
        ex_idx, _ = kvb.knn_exact_rows(Xd, w.k, rows, ctx)
        got = r.idx.index_select(0, rows.long())
        ex, gt = ex_idx[:, 1:].cpu().numpy(), got[:, 1:].cpu().numpy()
        hits = sum(len(np.intersect1d(a, b)) for a, b in zip(gt, ex))
        learned["recall"] = round(hits / float(ex.size), 5)
        learned["recall_rows"] = int(rows.numel())
        log(f"  learned: recall {learned['recall']} on {rows.numel()} rows, candidate share "
            f"{learned['candidate_share']}, largest bucket {learned['largest_bucket']}")
        out["learned"] = learned
    out["result"] = r
    return out


def train(kvb, ctx, Xd, w, args):
    """Partitioner training (timed separately, not part of a step)."""
    import torch
    n_train = min(w.n, 200_000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = kvb.train_partitioner(Xd, w.k, n_train=n_train, levels=10, h1=256, h2=256, n_probe=args.n_probe,
                                   epochs=args.train_epochs, batch=512, lr=2e-3, seed=args.seed, ctx=ctx)
    torch.cuda.synchronize()
    learned = {"train_s": round(time.perf_counter() - t0, 3), "train_rows": n_train, "epochs": args.train_epochs,
               "loss_first": round(float(losses[0]), 4), "loss_last": round(float(losses[-1]), 4),
               "mlp": [w.m, 256, 256, 1024], "n_probe": args.n_probe}
    log(f"bench: partitioner trained on {n_train} rows in {learned['train_s']} s, "
        f"loss {losses[0]:.4f} -> {losses[-1]:.4g}")
    return learned


def cpu_baseline(w, X, args):
    """The FP64 oracle on the host cores, on a bounded sample of the workload.
    Small workloads: the whole pipeline once. Large ones: the k-NN of random
    rows against all n samples (each row costs exactly n distance evaluations
    and one selection, so rows/s carries over), plus the O(nk) passes of the
    oracle's whole pipeline on a smaller draw of the same recipe (a row's passes
    cost O(k) whatever n is); rows/s = 1 / (k-NN s/row + passes s/row)."""
    import numpy as np
    import oracle
    import workloads
    union = args.pattern == "union"
    if w.n <= 200_000:
        log("bench: timing the FP64 oracle on the host cores (whole workload, one run)")
        c0 = time.perf_counter()
        if args.delta > 0:
            from oracle import spectral
            idx_o, d2_o = oracle.knn(X, w.k)
            base_o = spectral.union_pattern(idx_o, d2_o) if union else oracle.Pattern.from_knn(idx_o, d2_o)
            oracle.truncated_build(base_o, d2_o, w.k0, float(w.d), w.alpha, w.beta, args.delta, w.e_min,
                                   w.e_max, w.G)
        elif union:
            from oracle import spectral
            spectral.union_operator(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G,
                                    out_kind=oracle.MARKOV)
        else:
            oracle.pipeline(X, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G)
        c1 = time.perf_counter()
        return {"value": round(w.n / (c1 - c0), 2), "unit": "rows/s", "cores": oracle.num_threads(),
                "kind": "oracle", "sample": f"whole workload ({w.n} rows), one run, {c1 - c0:.2f} s"}
    rng = np.random.default_rng(args.seed + 7)
    # calibrate the k-NN sample to about 12 s of CPU work
    probe = rng.choice(w.n, 16, replace=False)
    c0 = time.perf_counter()
    oracle.knn_sampled(X, w.k, probe)
    per_row = (time.perf_counter() - c0) / 16
    rows = int(min(16384, max(64, 12.0 / per_row)))
    sel = rng.choice(w.n, rows, replace=False)
    log(f"bench: timing the FP64 oracle k-NN on {rows} random rows against all {w.n} samples")
    c0 = time.perf_counter()
    oracle.knn_sampled(X, w.k, sel)
    t_knn = time.perf_counter() - c0
    n_p = 50_000 if w.m <= 32 else 20_000
    Xp = workloads.make(w.name, seed=args.seed + 1, n=n_p)
    knn_p = oracle.knn(Xp, w.k)
    log(f"bench: timing the FP64 oracle's O(nk) passes on a {n_p}-sample draw of the same recipe")
    c0 = time.perf_counter()
    oracle.pipeline(Xp, w.k, w.k0, float(w.d), w.alpha, w.beta, w.e_min, w.e_max, w.G, knn_result=knn_p)
    t_pass = time.perf_counter() - c0
    per = t_knn / rows + t_pass / n_p
    return {"value": round(1.0 / per, 2), "unit": "rows/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"k-NN of {rows} random rows against all {w.n} samples ({t_knn:.2f} s) + the O(nk) passes "
                      f"(bandwidth, both tunings, density, q, normalisation, CSR order) on a {n_p}-sample draw of "
                      f"the same recipe ({t_pass:.2f} s); rows/s = 1 / (k-NN s/row + passes s/row)"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="gmm_n8m")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--mode", default="", choices=["", "f32", "bf16", "learned"],
                    help="k-NN mode of the timed form (the other forms are then not run)")
    ap.add_argument("--forms", default=None,
                    help="comma list of further k-NN forms timed on the same samples (default: bf16,learned on "
                         "the mixture workload, none elsewhere; '' for none)")
    ap.add_argument("--form-steps", type=int, default=5, help="timed steps of each further form")
    ap.add_argument("--n", type=int, default=0,
                    help="sample count override (same recipe, for profiling runs; not a bench line)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-peaks", action="store_true", help="skip the peak microbenchmarks")
    ap.add_argument("--curve-order", type=int, default=2, choices=[0, 1, 2],
                    help="exact matrix-core modes: 1 scans candidates in Morton curve order with projected-box "
                         "pruning, 2 also halves each 4096-tile group of the curve at its medians down to single "
                         "tiles, 0 scans every tile")
    ap.add_argument("--pattern", default="knn", choices=["knn", "union"],
                    help="matrix pattern: the directed k-NN rows, or their union with the transpose (symmetric)")
    ap.add_argument("--delta", type=float, default=0.0,
                    help="sparsity tolerance: keep only kernel entries above it (0 keeps every entry)")
    ap.add_argument("--eigs", type=int, default=0,
                    help="after the timed builds, the NEV leading eigenpairs of the symmetric conjugate on the union "
                         "pattern (sets --pattern union and the symmetric output), timed once")
    ap.add_argument("--ncv", type=int, default=1024, help="Lanczos steps of --eigs")
    ap.add_argument("--train-epochs", type=int, default=10, help="learned mode: partitioner training epochs")
    ap.add_argument("--n-probe", type=int, default=4,
                    help="learned mode: buckets each query searches (the configured top-4 by default)")
    ap.add_argument("--recall-rows", type=int, default=1024,
                    help="learned mode: rows whose recall is judged by the exact float64 row search")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.eigs:
        args.pattern = "union"
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the row-sharded design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per dispatch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("copy calibration: 3 dispatches of 1 GiB read + 1 GiB write")
        return 0

    import workloads
    from paper_2104_15124_amd import kvb

    w = workloads.WORKLOADS[args.workload]
    primary, extra = DEFAULT_FORMS.get(w.name, (w.mode, ()))
    if args.mode:
        primary, extra = args.mode, ()
    if args.forms is not None:
        extra = tuple(f for f in args.forms.split(",") if f)
    if args.n:
        w = dataclasses.replace(w, n=args.n)
    w = dataclasses.replace(w, mode=primary)
    log(f"bench: workload {w.name} n={w.n} m={w.m} k={w.k} primary form {primary}, further forms {list(extra)}, "
        f"margin={w.margin}")
    X = workloads.make(w.name, seed=args.seed, n=w.n)
    torch.cuda.set_device(0)
    Xd = torch.from_numpy(X).cuda()
    ctx = kvb.context()
    ctx.set_option(kvb.OPT_CURVE_ORDER, args.curve_order)
    peaks = None if args.no_peaks else measure_peaks(kvb, ctx)

    learned = train(kvb, ctx, Xd, w, args) if primary == "learned" else None
    main_form = run_form(kvb, ctx, Xd, w, primary, args.steps, args.warmup, args, peaks, learned, passes=True)
    r = main_form.pop("result")

    forms = {}
    for mode in extra:
        if mode == primary:
            continue
        lf = train(kvb, ctx, Xd, w, args) if mode == "learned" else None
        f = run_form(kvb, ctx, Xd, w, mode, args.form_steps, 1, args, peaks, lf)
        f.pop("result")
        f["vs_primary"] = round(f["value"] / main_form["value"], 4)
        if mode != "learned":
            f["exact"] = "certified k-NN sets (uncertified rows rescanned exactly)"
        forms[mode] = f

    eigs = None
    if args.eigs:
        eigs = run_eigs(kvb, ctx, Xd, w, r, args)

    cpu = None if args.no_cpu_baseline else cpu_baseline(w, X, args)

    union = args.pattern == "union"
    recall_txt = "learned-routed kNN (recall reported)" if primary == "learned" else "exact kNN sets"
    out = {
        "metric": "kernel-matrix rows/s (kNN+VB kernel->CSR) at " + recall_txt
                  + (", union pattern E u E^T" if union else "")
                  + (f", entries above {args.delta:g}" if args.delta > 0 else ""),
        "value": main_form["value"],
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if primary == "f32" else "bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "m": w.m, "k": w.k, "k0": w.k0, "d": w.d,
                   "mode": primary, "margin": w.margin, "grid": [w.e_min, w.e_max, w.G],
                   "curve_order": (args.curve_order if primary != "learned" and not (primary == "f32" and w.m <= 8)
                                   else 0),
                   "alpha": w.alpha, "beta": w.beta, "fallback_rows": main_form["fallback_rows"],
                   "learned": main_form.get("learned"), "pattern": args.pattern, "delta": args.delta,
                   "nnz": main_form["nnz"]},
        "roofline": main_form["roofline"],
        "passes": main_form["passes"],
        "forms": forms,
        "peaks_measured": peaks,
        "cpu_baseline": cpu,
    }
    if eigs is not None:
        out["eigsh"] = eigs
    print(json.dumps(out), flush=True)
    return 0


def run_eigs(kvb, ctx, Xd, w, r, args):
    """Leading eigenpairs of the symmetric conjugate on the union pattern, then
    the downstream steps of Sections 3 and 5.3 on that eigenbasis, timed once."""
    import torch
    nnz_i = int(r.rowptr[-1].item())
    col, val = r.col[:nnz_i], r.val[:nnz_i]
    kvb.eigsh(r.rowptr, col, val, nev=args.eigs, ncv=max(args.eigs, 16), ctx=ctx)    # warm-up
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    ev = kvb.eigsh(r.rowptr, col, val, nev=args.eigs, ncv=args.ncv, tol=1e-8, seed=args.seed, ctx=ctx)
    e1 = time.perf_counter()
    # per Lanczos step: one sparse product (12 B per entry + the vectors),
    # two projections and two subtractions over the basis (j n 8 B each, j
    # the step), one norm: the basis sweeps dominate
    basis_bytes = 4.0 * 8 * w.n * args.ncv * (args.ncv + 1) / 2
    eigs = {"nev": args.eigs, "ncv": args.ncv, "ms": round((e1 - e0) * 1e3, 2),
            "values": [round(float(x), 6) for x in ev.values],
            "max_residual": float(f"{ev.residuals.max():.4g}"), "converged": ev.converged,
            "basis_GB/s": round(basis_bytes / (e1 - e0) / 1e9, 1)}
    log(f"  eigsh: {args.eigs} pairs, {args.ncv} Lanczos steps in {eigs['ms']} ms, values {eigs['values']}, "
        f"max residual {eigs['max_residual']}")
    # Kolmogorov solve for g = x_1 - mean, grad f per coordinate, particle update
    g = (Xd[:, 0].double() - Xd[:, 0].double().mean()).contiguous()
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    f, _, _ = kvb.kolmogorov_solve(ev, r.P, r.D, g, skip=1, ctx=ctx)
    s1 = time.perf_counter()
    grad = torch.empty((w.m, w.n), dtype=torch.float64, device="cuda")
    for c in range(w.m):
        grad[c], _ = kvb.carre_du_champ(ev, r.P, r.D, f, Xd[:, c].double().contiguous(), ctx=ctx)
    s2 = time.perf_counter()
    Xo = torch.empty_like(Xd)
    ctx.check(ctx.lib.kvb_advect(ctx.h, kvb._ptr(Xd), w.n, w.m, None, kvb._ptr(grad), None, 0.01, 0.0,
                                 kvb._ptr(Xo)))
    torch.cuda.synchronize()
    s3 = time.perf_counter()
    eigs.update({"solve_ms": round((s1 - s0) * 1e3, 3), "grad_ms": round((s2 - s1) * 1e3, 3),
                 "advect_ms": round((s3 - s2) * 1e3, 3)})
    log(f"  Kolmogorov solve {eigs['solve_ms']} ms, grad f ({w.m} coordinates) {eigs['grad_ms']} ms, "
        f"particle update {eigs['advect_ms']} ms")
    return eigs


if __name__ == "__main__":
    sys.exit(main())
