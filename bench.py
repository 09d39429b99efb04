#!/usr/bin/env python3
"""Benchmark of the fast-JOFC hot path on one MI355X.

Workload (one "step"): in-sample fJOFC with m = 3 modalities, n = 20000
objects, d = 5: 300 Guttman transforms from a seeded N(0,1) start, FP64
stress every 10 transforms, over 3 synthetic FP32 dissimilarity matrices
(4.8 GB, built on the device from the seeded latent model before timing).

Prints one JSON line: throughput in dissimilarity pairs per second (unordered
pairs {j,l} of every modality, per transform), the roofline of the dominant
kernel (the interior-tile dissimilarity stream, HBM-bound) from HIP events
recorded by the library around each launch during the timed region, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fJOFC Δ-pairs/s & HBM GB/s; time-to-stress-tol, learned warm start vs plain"
PEAK_HBM_GBS = 8000.0
# VALU issue peak without packed FP32 (disabled in every build): 256 CUs x
# 4 SIMDs x 16 lanes per clock x 2.4 GHz, in FP32 lane-operations per second
PEAK_VALU_OPS = 256 * 64 * 2.4e9
# issue slots one unordered pair needs at d = 5: 5 subtractions, 5 FMAs for
# d^2, v_rsq (2 slots), a multiply, 10 FMAs for the row and column sums
SLOTS_PER_PAIR_D5 = 23
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_insample_stream_m3_n20000_d5.json")
CSRC = os.path.join(ROOT, "paper_1502_03391_amd", "csrc")
TILE_CACHE = os.path.join(ROOT, "paper_1502_03391_amd", "tune_cache.txt")
# the stream kernel (its device code and the D = 5..8 instantiations) and
# the cache that picks its tile
STREAM_SRC = (os.path.join(CSRC, "stream_dev.h"), os.path.join(CSRC, "stream_hi.hip"),
              TILE_CACHE)
KERNEL_SRC = STREAM_SRC[0]
OOS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_oos_m2_n10000_d5.json")
OOS_SRC = os.path.join(ROOT, "paper_1502_03391_amd", "csrc", "oos.hip")
BATCHED_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_batched_512_uneven.json")
# the batch's kernels and its launch plan
# the lockstep batch: stream kernels of every D, the finalize and reduce
# kernels, the launch plan and the tiles
BATCHED_SRC = (os.path.join(CSRC, "stream_dev.h"), os.path.join(CSRC, "stream_lo.hip"),
               os.path.join(CSRC, "stream_hi.hip"), os.path.join(CSRC, "insample.hip"),
               os.path.join(CSRC, "host.cpp"), TILE_CACHE)


def kernel_hash(src=KERNEL_SRC) -> str:
    h = hashlib.sha256()
    for path in ((src,) if isinstance(src, str) else src):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(path=TRAFFIC_FILE, src=STREAM_SRC, key="bytes_per_launch"):
    """HBM bytes per launch of a kernel (or per unit `key` names) from
    committed rocprofv3 counter runs, or None when absent or taken on a
    different kernel source."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash(src):
        return None
    return t.get(key)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 2 GiB device copy (counter calibration)")
    ap.add_argument("--iters", type=int, default=None,
                    help="transforms per step (default: the workload's 300); "
                         "for short profiled runs only")
    ap.add_argument("--extras", default="relaxed,init,paper,early,oos,batched,warmstart",
                    help="comma list of extra workloads to measure after the main one "
                         "(relaxed, init, paper, early, oos, batched, warmstart) or 'none'")
    ap.add_argument("--only-extras", action="store_true",
                    help="skip the main workload and print only the extras' JSON "
                         "(for profiled runs of one extra workload)")
    ap.add_argument("--batched-iters", type=int, default=150,
                    help="transforms per batched run (default: the workload's 150)")
    ap.add_argument("--batched-launches", default="lockstep,persistent",
                    help="batched launches to time: lockstep (reported), persistent")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs the whole hot path on a "
              "single MI355X; --gpus above 1 is not supported.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1502_03391_amd import fjofc
    from workloads import generators as gen

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    extras = [e for e in args.extras.split(",") if e and e != "none"]
    if args.calib_copy:
        a = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.only_extras:
        ctx = fjofc.Context(0)
        out = {"extra": {}}
        independent_extras(ctx, extras, out, args)
        ctx.close()
        print(json.dumps(out), flush=True)
        return
    spec = gen.config1_spec()
    m, n, d, iters, every = spec.m, spec.n, spec.d, spec.iters, spec.stress_every
    if args.iters is not None:
        iters = args.iters
    views, _, X0 = gen.config1_views(spec)
    delta = [gen.pairwise_dist_torch(Y, dev) for Y in views]
    wmat = gen.uniform_wmat(m, spec.w)
    X0d = torch.from_numpy(X0.astype(np.float32)).to(dev)
    X = torch.empty_like(X0d)
    torch.cuda.synchronize()
    print(f"[bench] inputs ready: m={m} n={n} d={d}", file=sys.stderr, flush=True)

    ctx = fjofc.Context(0)

    def step():
        X.copy_(X0d)
        r, _ = fjofc.fjofc_embed(ctx, delta, wmat, X, iters, stress_every=every)
        return r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fjofc.fjofc_profile_enable(ctx, True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = fjofc.fjofc_profile_read(ctx)
    fjofc.fjofc_profile_enable(ctx, False)
    print(f"[bench] timed {args.steps} steps: {t1 - t0:.3f} s; final stress "
          f"{res['stress']:.6e}", file=sys.stderr, flush=True)

    pairs_step = iters * m * n * (n - 1) / 2.0
    sec = (t1 - t0) / args.steps
    value = pairs_step / sec
    per_launch_bytes = prof["stream_bytes"] / max(1, prof["stream_launches"])
    avg_ms = prof["stream_ms"] / max(1, prof["stream_launches"])
    achieved = per_launch_bytes / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Δ-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": spec.name, "m": m, "n": n, "d": d, "iters": iters,
                   "stress_every": every, "w": spec.w,
                   "dissimilarity_bytes": 4 * m * n * n,
                   "parallelism": "single-gpu"},
        "hbm_gbs_step": 4.0 * pairs_step / sec / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic,
                     "kernel": "bx_kernel (interior tiles)",
                     "launches": prof["stream_launches"],
                     "avg_launch_ms": avg_ms,
                     "bytes_per_launch": per_launch_bytes},
        "roofline_alu": {"bound": "alu", "unit": "lane-op/s",
                         "achieved": SLOTS_PER_PAIR_D5 * per_launch_bytes / 4.0 / (avg_ms * 1e-3),
                         "peak": PEAK_VALU_OPS,
                         "frac": SLOTS_PER_PAIR_D5 * per_launch_bytes / 4.0 / (avg_ms * 1e-3)
                         / PEAK_VALU_OPS,
                         "slots_per_pair": SLOTS_PER_PAIR_D5,
                         "note": "secondary: the stream's issue-slot work per pair against the "
                                 "non-packed FP32 VALU peak at 2.4 GHz (d = 5 only)"}
        if d == 5 else None,
        "kernel_ms_per_step": {k: prof[k] / args.steps for k in
                               ("stream_ms", "edge_ms", "finalize_ms", "reduce_ms")},
        "final_stress_norm": res["stress_norm"],
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(delta, wmat, X0, m, n, every, args.cpu_seconds)
    out["extra"] = {}
    if "relaxed" in extras:
        out["extra"]["relaxed"] = bench_relaxed(ctx, delta, wmat, X0d, res["stress"], iters,
                                                every)
    if "init" in extras:
        out["extra"]["init"] = bench_init(ctx, delta, wmat, res["stress"], iters, every)
    del delta, X, X0d
    torch.cuda.empty_cache()
    independent_extras(ctx, extras, out, args)
    ctx.close()
    print(json.dumps(out), flush=True)


def independent_extras(ctx, extras, out, args):
    """The extra workloads that build their own inputs."""
    if "paper" in extras:
        out["extra"]["paper"] = bench_paper_shape(ctx)
    if "early" in extras:
        out["extra"]["early_stop"] = bench_early_stop(ctx)
    if "oos" in extras:
        out["extra"]["oos"] = bench_oos(ctx)
    if "batched" in extras:
        out["extra"]["batched"] = bench_batched(
            ctx, args.batched_iters, [x for x in args.batched_launches.split(",") if x])
    if "warmstart" in extras:
        out["extra"]["warmstart"] = bench_warmstart(ctx)


def bench_oos(ctx):
    """Out-of-sample workload: in-sample m=2, n=10000, d=5 (300 transforms),
    then 50000 new objects from the same latent model, 100 transforms each,
    4096 objects per launch."""
    import numpy as np
    import torch
    from paper_1502_03391_amd import fjofc
    from workloads import generators as gen
    sp = gen.config2_spec()
    dev = torch.device("cuda:0")
    views, maps, X0 = gen.latent_views(sp.seed_in, sp.n, sp.m, sp.lat, sp.sigma, sp.d)
    delta = [gen.pairwise_dist_torch(Y, dev) for Y in views]
    wmat = gen.uniform_wmat(sp.m, sp.w)
    Xin = torch.from_numpy(X0.astype(np.float32)).to(dev)
    fjofc.fjofc_embed(ctx, delta, wmat, Xin, sp.in_iters, stress_every=sp.in_iters)
    del delta
    new = gen.oos_objects(sp.seed_new, sp.k, maps, sp.sigma)
    dnew = torch.empty((sp.k, sp.m, sp.n), dtype=torch.float32, device=dev)
    for i in range(sp.m):
        dnew[:, i, :] = gen.cross_dist_torch(new[i], views[i], dev)
    scale = float(torch.sqrt((Xin.double() ** 2).mean()))
    Y0 = torch.from_numpy(gen.gaussian_start(sp.seed_start, (sp.k, sp.m, sp.d), scale)
                          .astype(np.float32)).to(dev)
    Y = torch.empty_like(Y0)
    stress = torch.empty(sp.k, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    print(f"[bench] oos inputs ready: k={sp.k}", file=sys.stderr, flush=True)

    def run():
        Y.copy_(Y0)
        for o0 in range(0, sp.k, sp.batch):
            o1 = min(sp.k, o0 + sp.batch)
            fjofc.fjofc_oos(ctx, Xin, wmat, dnew[o0:o1], Y[o0:o1], sp.iters,
                            stress_out=stress[o0:o1], sync=False)
        torch.cuda.synchronize()

    run()
    fjofc.fjofc_profile_enable(ctx, True)
    t0 = time.perf_counter()
    run()
    t1 = time.perf_counter()
    prof = fjofc.fjofc_profile_read(ctx)
    fjofc.fjofc_profile_enable(ctx, False)
    sec = t1 - t0
    triples = sp.k * sp.m * sp.n * sp.iters
    gbs = prof["oos_bytes"] / (prof["oos_ms"] * 1e-3) / 1e9
    r = {"workload": sp.name, "objects": sp.k, "iters": sp.iters, "batch": sp.batch,
         "seconds": sec, "triples_per_s": triples / sec, "objects_per_s": sp.k / sec,
         "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": gbs / PEAK_HBM_GBS, "kernel": "oos_kernel",
                      "traffic": load_traffic(OOS_TRAFFIC_FILE, OOS_SRC),
                      "traffic_per": "launch of 4096 objects, 101 passes",
                      "launches": prof["oos_launches"],
                      "avg_launch_ms": prof["oos_ms"] / max(1, prof["oos_launches"])},
         "mean_stress": float(stress.mean())}
    del dnew
    torch.cuda.empty_cache()
    return r


def bench_relaxed(ctx, delta, wmat, X0d, final_stress, iters, every, alpha=1.9):
    """Time to a stress target on the main workload: the target is the plain
    run's final stress (after `iters` transforms) + 1e-4 relative; plain and
    relaxed (alpha) transforms run with the stress-target stop rule,
    checked every `every` transforms."""
    import torch
    from paper_1502_03391_amd import fjofc
    target = final_stress * (1.0 + 1e-4)
    out = {"workload": "insample_m3_n20000_d5_to_target", "target_stress": target,
           "rel": 1e-4, "stress_every": every}
    X = torch.empty_like(X0d)
    for name, a in (("plain", 1.0), ("relaxed", alpha)):
        X.copy_(X0d)
        fjofc.fjofc_embed(ctx, delta, wmat, X, 2, stress_every=every, alpha=a)  # warm-up
        X.copy_(X0d)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r, _ = fjofc.fjofc_embed(ctx, delta, wmat, X, 2 * iters, tol=target,
                                 tol_mode=fjofc.FJOFC_TOL_TARGET, stress_every=every, alpha=a)
        torch.cuda.synchronize()
        out[name] = {"alpha": a, "seconds": time.perf_counter() - t0,
                     "transforms": r["iters_run"], "reached": bool(r["converged"]),
                     "stress": r["stress"]}
    out["speedup"] = out["plain"]["seconds"] / out["relaxed"]["seconds"]
    print(f"[bench] relaxed: plain {out['plain']['transforms']} transforms "
          f"{out['plain']['seconds']:.3f} s, alpha={alpha} {out['relaxed']['transforms']} "
          f"transforms {out['relaxed']['seconds']:.3f} s", file=sys.stderr, flush=True)
    return out


def bench_init(ctx, delta, wmat, random_final, iters, every, init_iters=20):
    """The paper's start (cMDS of the mean and of each Delta_i, Procrustes)
    on the main workload: its cost, its stress, and the transforms it needs
    to reach the random start's final stress (+1e-4 relative)."""
    import torch
    from paper_1502_03391_amd import fjofc
    m, n = len(delta), int(delta[0].shape[0])
    d = 5
    X = torch.empty((m * n, d), device=delta[0].device)
    fjofc.fjofc_init_cmds(ctx, delta, X, iters=2)  # warm-up
    torch.cuda.synchronize()
    fjofc.fjofc_profile_enable(ctx, True)
    t0 = time.perf_counter()
    eig = fjofc.fjofc_init_cmds(ctx, delta, X, iters=init_iters)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    prof = fjofc.fjofc_profile_read(ctx)
    fjofc.fjofc_profile_enable(ctx, False)
    # product passes: every Delta_i read once per pass (full rows), all
    # m + 1 problems formed from those reads
    pass_ms = prof["init_ms"] / max(1, prof["init_launches"])
    pass_bytes = prof["init_bytes"] / max(1, prof["init_launches"])
    pass_gbs = pass_bytes / (pass_ms * 1e-3) / 1e9
    s0 = fjofc.fjofc_stress(ctx, delta, wmat, X)["stress"]
    target = random_final * (1.0 + 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r, _ = fjofc.fjofc_embed(ctx, delta, wmat, X, iters, tol=target,
                             tol_mode=fjofc.FJOFC_TOL_TARGET, stress_every=every)
    torch.cuda.synchronize()
    t_embed = time.perf_counter() - t0
    out = {"workload": "insample_m3_n20000_d5_paper_start", "init_iters": init_iters,
           "init_seconds": t_init, "product_passes": prof["init_launches"],
           "pass_ms": pass_ms, "pass_bytes": pass_bytes, "pass_hbm_gbs": pass_gbs,
           "pass_hbm_frac": pass_gbs / PEAK_HBM_GBS,
           "pass_triangle_frac": 0.5 * pass_gbs / PEAK_HBM_GBS,
           "products_seconds": prof["init_ms"] * 1e-3,
           "start_stress": s0, "top_ritz_mean": eig[0].tolist(),
           "target_stress": target, "transforms_to_target": r["iters_run"],
           "reached": bool(r["converged"]), "embed_seconds": t_embed,
           "random_start_transforms": iters,
           "total_seconds": t_init + t_embed}
    print(f"[bench] paper start: init {t_init:.3f} s ({prof['init_launches']} passes of "
          f"{pass_ms:.3f} ms, {pass_gbs:.0f} GB/s)", file=sys.stderr, flush=True)
    print(f"[bench] paper start: {r['iters_run']} transforms "
          f"({t_embed:.3f} s) to the random start's {iters}-transform stress",
          file=sys.stderr, flush=True)
    return out


def bench_paper_shape(ctx, reps=5):
    """The paper's matched-setting shape (n = 400, m = 3, d = 2) run to its
    stop rule (normalised stress decreasing by less than 1e-6) from its own
    start (cMDS + Procrustes), on the paper's matched-setting recipe (jittered
    copies of a 2-D Gaussian sample); w = 0.5, which the paper does not state.
    The paper's own figure for this setting is quoted as context, with its
    hardware."""
    import numpy as np
    import torch
    from paper_1502_03391_amd import fjofc
    from workloads import generators as gen
    n, m, d = 400, 3, 2
    dev = torch.device("cuda:0")
    views = gen.matched_views(400, n, m)
    delta = [gen.pairwise_dist_torch(Y, dev) for Y in views]
    wmat = gen.uniform_wmat(m, 0.5)
    X = torch.empty((m * n, d), device=dev)
    times, res = [], None
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fjofc.fjofc_init_cmds(ctx, delta, X, iters=20)
        res, _ = fjofc.fjofc_embed(ctx, delta, wmat, X, 5000, tol=1e-6,
                                   tol_mode=fjofc.FJOFC_TOL_PAPER, stress_every=1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    sec = float(np.median(times[1:]))
    return {"workload": "paper_matched_n400_m3_d2", "seconds_to_stop": sec,
            "transforms": res["iters_run"], "converged": bool(res["converged"]),
            "final_stress_norm": res["stress_norm"],
            "paper_context": {"seconds": 1.39, "final_stress_norm": 0.03,
                              "hardware": "2.6 GHz Intel Core i5, serial",
                              "data": "same recipe, the paper's own draws"}}


def bench_early_stop(ctx, reps=25, ks=(1, 2, 5, 10, 25, 50, 100, 200)):
    """The error-tolerance experiment of Section 4.2: for the matched and the
    anomaly setting (10 anomalous rows in the last view) with m = 4, 5, 6,
    n = 400, d = 2, w = 0.5, each draw starts at the paper's start and records
    ||X_final - X_k||_F / ||X_final||_F at the listed k (over non-anomalous
    rows only in the anomaly setting) for two X_final: the paper's stop rule
    (normalised stress decreasing by less than 1e-6) and a tight one (relative
    decrease below 1e-10, at most 5000 transforms).  Reports the means and
    2 s.e. over the draws, and the mean transforms to each stop."""
    import numpy as np
    import torch
    from paper_1502_03391_amd import fjofc
    from workloads import generators as gen
    n, d, n_anom = 400, 2, 10
    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    out = {"workload": "paper_error_tolerance_n400_d2", "reps": reps, "k": list(ks),
           "norm": "Frobenius", "paper_context": "about 5% relative error at k = 25 in the "
           "anomaly setting, which needs over 100 transforms on average to stop"}
    for setting in ("matched", "anomaly"):
        for m in (4, 5, 6):
            wmat = gen.uniform_wmat(m, 0.5)
            keep = torch.ones(m * n, dtype=torch.bool, device=dev)
            if setting == "anomaly":
                keep[(m - 1) * n:(m - 1) * n + n_anom] = False
            errs = {"paper": [], "tight": []}
            stops = {"paper": [], "tight": []}
            for r in range(reps):
                views = gen.matched_views(1000 * m + r, n, m,
                                          n_anom if setting == "anomaly" else 0)
                delta = [gen.pairwise_dist_torch(Y, dev) for Y in views]
                X0 = torch.empty((m * n, d), device=dev)
                fjofc.fjofc_init_cmds(ctx, delta, X0, iters=20)
                finals = {}
                for name, tol, mode in (("paper", 1e-6, fjofc.FJOFC_TOL_PAPER),
                                        ("tight", 1e-10, fjofc.FJOFC_TOL_REL)):
                    Xf = X0.clone()
                    res, _ = fjofc.fjofc_embed(ctx, delta, wmat, Xf, 5000, tol=tol,
                                               tol_mode=mode, stress_every=1)
                    stops[name].append(res["iters_run"])
                    finals[name] = Xf[keep].double()
                Xk, done = X0.clone(), 0
                rows = {"paper": [], "tight": []}
                for k in ks:
                    fjofc.fjofc_embed(ctx, delta, wmat, Xk, k - done,
                                      tol_mode=fjofc.FJOFC_TOL_NONE, stress_every=k - done)
                    done = k
                    for name, ref in finals.items():
                        rows[name].append(float((ref - Xk[keep].double()).norm() / ref.norm()))
                for name in rows:
                    errs[name].append(rows[name])
            cell = {}
            for name in ("paper", "tight"):
                e = np.asarray(errs[name])
                se = e.std(axis=0, ddof=1) / np.sqrt(reps)
                cell[name] = {"rel_err_mean": e.mean(axis=0).tolist(),
                              "rel_err_2se": (2 * se).tolist(),
                              "transforms_to_stop_mean": float(np.mean(stops[name]))}
            out[f"{setting}_m{m}"] = cell
    out["seconds"] = time.perf_counter() - t_start
    a = out["anomaly_m4"]
    print(f"[bench] error tolerance: anomaly m=4: paper stop after "
          f"{a['paper']['transforms_to_stop_mean']:.0f} transforms, tight after "
          f"{a['tight']['transforms_to_stop_mean']:.0f}; err@25 vs tight "
          f"{a['tight']['rel_err_mean'][list(ks).index(25)]:.4f} "
          f"({out['seconds']:.1f} s)", file=sys.stderr, flush=True)
    return out


def bench_warmstart(ctx):
    """Learned warm start: in-sample m=2, n=10000, d=5; 200000 training
    objects whose targets are converged out-of-sample solutions; network
    512 -> 3 x 512 GELU -> 5 (one consensus point, BF16 matrix cores), 20
    epochs, with the 10-output per-modality network beside it; 50000
    held-out objects refined until their stress is within 1e-4 relative of
    the plain start's stress after 100 transforms, every pipeline in calls
    of 4096 objects."""
    import torch
    from paper_1502_03391_amd import warmstart
    t0 = time.perf_counter()
    r = warmstart.run(ctx, warmstart.WarmStartConfig(), eval_objects=50000, ablation=True,
                      log=lambda *a: print(*a, file=sys.stderr, flush=True))
    r["total_seconds"] = time.perf_counter() - t0
    torch.cuda.empty_cache()
    return r


def bench_batched(ctx, iters=150, launches=("lockstep", "persistent")):
    """512 independent problems, m ~ U{2,3,4}, n ~ U[64,2048], d ~ U{2,3,5},
    150 transforms each, replayed from a captured HIP graph: the lockstep
    launches (the library's default and the reported time) and the one
    persistent launch, which must give bitwise the same results."""
    import numpy as np
    import torch
    from paper_1502_03391_amd import fjofc
    from workloads import generators as gen
    dev = torch.device("cuda:0")
    specs = gen.batched_specs(512)
    probs, X0s = [], []
    pairs = 0.0
    for sp in specs:
        views, _, X0 = gen.instance_views(sp)
        dl = [gen.pairwise_dist_torch(Y, dev) for Y in views]
        X0d = torch.from_numpy(X0.astype(np.float32)).to(dev)
        probs.append((dl, gen.uniform_wmat(sp.m, 0.5), X0d.clone()))
        X0s.append(X0d)
        pairs += sp.m * sp.n * (sp.n - 1) / 2.0
    torch.cuda.synchronize()
    print(f"[bench] batched inputs ready: {len(specs)} problems", file=sys.stderr, flush=True)

    def reset():
        for (_, _, X), X0 in zip(probs, X0s):
            X.copy_(X0)
        torch.cuda.synchronize()

    def timed(launch, quiet=False):
        b = fjofc.Batch(ctx, probs)
        try:
            b.set_launch(launch)
        except fjofc.FjofcError as e:
            b.close()
            if not quiet:
                print(f"[bench] batched: no {launch} launch: {e}", file=sys.stderr, flush=True)
            return None
        reset()
        b.run(iters, stress_every=iters, want_results=False)
        torch.cuda.synchronize()
        times = []
        for _ in range(3):
            reset()
            t0 = time.perf_counter()
            res = b.run(iters, stress_every=iters)
            t1 = time.perf_counter()
            times.append(t1 - t0)
        out = [X.clone() for _, _, X in probs]
        b.close()
        return min(times), res, out

    def persistent_retiling():
        # problems whose cached tile has 8 columns per lane or double-buffered
        # loads, which the persistent kernel has no form of, take the
        # single-buffered 4-column tile of the same height: scoped FJOFC_TILE
        # entries, and how many problems
        swap, k = set(), 0
        for sp in specs:
            th, var = fjofc.fjofc_tile_choice(ctx, sp.n, sp.d)
            if var in (0, 2, 3):
                swap.add(f"{sp.d}:{sp.n}:{sp.n}:{th}:1")
                k += 1
        return ",".join(sorted(swap)), k

    def timed_on(tiles, launch):
        os.environ["FJOFC_TILE"] = tiles
        try:
            return timed(launch)
        finally:
            os.environ.pop("FJOFC_TILE", None)

    first = timed(launches[0])
    retiled = None
    if first is None and launches[0] == "persistent":
        retiled = persistent_retiling()
        first = timed_on(retiled[0], "persistent")
    if first is None:
        raise RuntimeError(f"the batch has no {launches[0]} launch")
    sec, res = first[0], first[1]
    hbm = load_traffic(BATCHED_TRAFFIC_FILE, BATCHED_SRC, "bytes_per_sweep")
    r = {"workload": "batched_512_uneven", "problems": len(specs), "iters": iters,
         "launch": launches[0], "pairs_per_sweep": pairs,
         "algorithmic_bytes_per_sweep": 4.0 * pairs,
         "hbm_bytes_per_sweep": hbm,
         "seconds": sec, "pairs_per_s": pairs * iters / sec,
         "algorithmic_gbs": 4.0 * pairs * iters / sec / 1e9,
         "mean_stress_norm": float(np.mean([x["stress_norm"] for x in res]))}
    if hbm is not None:
        r["hbm_gbs"] = hbm * iters / sec / 1e9
    if retiled is not None:
        r["persistent_plan"] = {"problems_retiled": retiled[1]}
    msg = f"{launches[0]} {sec:.4f} s"
    if "persistent" in launches[1:]:
        ref = first
        pers = timed("persistent", quiet=True)
        if pers is None:
            # compare both launches on one plan the persistent kernel runs
            retiled = persistent_retiling()
            print(f"[bench] batched: {retiled[1]} problems of the cache's plan have 8-column "
                  "or double-buffered tiles, which the persistent launch has no form of; both "
                  "launches are compared on the plan with those problems on the single-buffered "
                  "4-column tile",
                  file=sys.stderr, flush=True)
            ref = timed_on(retiled[0], "lockstep")
            pers = timed_on(retiled[0], "persistent")
            r["persistent_plan"] = {"problems_retiled": retiled[1],
                                    "lockstep_seconds_same_plan": ref[0]}
            msg += f", lockstep on the persistent plan {ref[0]:.4f} s"
        if pers is not None:
            r["persistent_seconds"] = pers[0]
            r["persistent_equals_lockstep"] = (
                all(torch.equal(a, c) for a, c in zip(pers[2], ref[2])) and ref[1] == pers[1])
            msg += (f", persistent {pers[0]:.4f} s (bitwise equal to lockstep on its plan: "
                    f"{r['persistent_equals_lockstep']})")
        else:
            r["launches_not_available"] = ["persistent"]
    print(f"[bench] batched: {msg}", file=sys.stderr, flush=True)
    del first
    del probs
    torch.cuda.empty_cache()
    return r


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(delta, wmat, X0, m, n, every, target_s):
    """The FP64 CPU oracle (as it is) on a bounded sample of the same
    workload: a few full Guttman transforms of the same problem on all host
    threads, and one transform on one thread."""
    import numpy as np
    from oracle import structured as orc
    host = np.empty((m, n, n), dtype=np.float32)
    for i in range(m):
        host[i] = delta[i].cpu().numpy()
    X0c = X0.astype(np.float32).astype(np.float64)
    threads = orc.threads()
    # one transform first, to size the sample
    t0 = time.perf_counter()
    orc.embed(host, wmat, X0c, 1, stress_every=every, want_hist=False)
    t1 = time.perf_counter()
    per = t1 - t0
    iters = max(1, min(50, int(target_s / max(per, 1e-3))))
    t0 = time.perf_counter()
    orc.embed(host, wmat, X0c, iters, stress_every=every, want_hist=False)
    t1 = time.perf_counter()
    pairs = iters * m * n * (n - 1) / 2.0
    out = {"value": pairs / (t1 - t0), "unit": "Δ-pairs/s",
           "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{iters} full Guttman transforms of the same m={m} n={n} d=5 "
                     f"problem (plus stress at t=0 and at the end), FP64 C oracle, "
                     f"{t1 - t0:.1f} s"}
    # one thread: a single transform (no stress evaluation)
    orc.set_threads(1)
    try:
        t0 = time.perf_counter()
        orc.guttman(host, wmat, X0c)
        t1 = time.perf_counter()
    finally:
        orc.set_threads(threads)
    out["one_thread"] = {"value": m * n * (n - 1) / 2.0 / (t1 - t0), "unit": "Δ-pairs/s",
                         "cores": 1, "kind": "oracle",
                         "sample": f"1 Guttman transform of the same problem on one thread, "
                                   f"{t1 - t0:.1f} s"}
    del host
    out["paper_jofc_vs_fjofc"] = jofc_context()
    return out


def jofc_context():
    """Context for Section 4.3 on the host, with the oracle's two forms of
    one Guttman transform: the dense one through L^dagger (the original JOFC
    update, L^dagger precomputed and timed apart) against the structured
    one (the FP64 C oracle), on the paper's matched recipe (d = 2, w = 0.5)
    for m = 2..6 at n = 400 and n = 200..1000 at m = 3.  Both run on one
    thread (the C oracle's OpenMP and numpy's BLAS limited to one), as the
    paper ran serially; its per-iteration ratios are quoted beside ours."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import dense, structured as orc
    from workloads import generators as gen
    t_start = time.perf_counter()

    def problem(m, n):
        views = gen.matched_views(4300 + 10 * m + n, n, m)
        delta = [gen.pairwise_dist_np(Y) for Y in views]
        return delta, gen.uniform_wmat(m, 0.5), gen.gaussian_start(4400 + m + n, (m * n, 2))

    def fast(m, n, reps=10):
        delta, wmat, X = problem(m, n)
        dstack = np.stack(delta).astype(np.float32)
        for _ in range(3):
            orc.guttman(dstack, wmat, X)
        t0 = time.perf_counter()
        for _ in range(reps):
            orc.guttman(dstack, wmat, X)
        return (time.perf_counter() - t0) / reps

    def slow(m, n):
        # L^dagger from Corollary 1's closed form (equal to numpy's pinv to
        # 1e-14, pinned in the oracle's tests): the per-iteration product is
        # the same dense (mn x mn) one, without timing an SVD per shape
        delta, wmat, X = problem(m, n)
        W, D = dense.omnibus_weights(wmat, n), dense.omnibus_delta(delta)
        t0 = time.perf_counter()
        Lp = dense.ldagger_corollary(wmat, n)
        t_pinv = time.perf_counter() - t0
        td = []
        for _ in range(2):
            t0 = time.perf_counter()
            dense.guttman(X, D, W, Lp)
            td.append(time.perf_counter() - t0)
        return t_pinv, min(td)

    shapes = [(m, 400) for m in (2, 3, 4, 5, 6)] + [(3, n) for n in (200, 400, 600, 800, 1000)]
    # every structured timing before any dense one: the dense products
    # leave BLAS threads spinning, which would slow the structured ones
    threads = orc.threads()
    orc.set_threads(1)
    try:
        tf = {mn: fast(*mn) for mn in shapes}
    finally:
        orc.set_threads(threads)
    rows = {}
    with threadpool_limits(limits=1):
        for mn in shapes:
            t_pinv, t_iter = slow(*mn)
            rows[mn] = {"m": mn[0], "n": mn[1], "ldagger_s": t_pinv, "jofc_iter_s": t_iter,
                        "fjofc_iter_s": tf[mn], "ratio": t_iter / tf[mn]}
    m_sweep = [rows[mn] for mn in shapes[:5]]
    n_sweep = [rows[mn] for mn in shapes[5:]]
    res = {"kind": "oracle", "cores": 1, "label": "context: both forms serial, like the paper",
           "m_sweep_n400": m_sweep, "n_sweep_m3": n_sweep,
           "paper_ratios": {"m=2..6 at n=400": [2.86, 4.82, 6.70, 8.59, 10.71],
                            "n=200..1000 at m=3": [2.10, 4.86, 7.45, 10.13, 12.63],
                            "hardware": "2.6 GHz Intel Core i5, serial"},
           "seconds": time.perf_counter() - t_start}
    print(f"[bench] JOFC/fJOFC per-iteration ratio on the host: m-sweep "
          f"{[round(r['ratio'], 1) for r in m_sweep]}, n-sweep "
          f"{[round(r['ratio'], 1) for r in n_sweep]} ({res['seconds']:.1f} s)",
          file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
