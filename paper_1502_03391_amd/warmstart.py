"""Learned warm start for out-of-sample fJOFC (all GPU work through libfjofc).

Pipeline (every numerical step runs in the library's kernels; torch holds
device memory and does index plumbing):

1. In-sample embedding X of n objects in m modalities (fjofc_embed).
2. Training pairs: new objects from the same latent model and their
   dissimilarities to all in-sample objects; out-of-sample transforms from
   the nearest-in-sample start run until the stress stops decreasing
   (fjofc_oos_nearest_start, fjofc_oos with a tolerance).  The target is the
   converged point of every modality (m d outputs, `per_modality`), or the
   consensus point, their mean over the modalities (fjofc_oos_consensus; d
   outputs, every modality then starts from it).
3. Features: the dissimilarities to L fixed landmark objects in every
   modality, standardised with training statistics (fjofc_mlp_feature_stats,
   fjofc_mlp_features).
4. Training: MSE, Adam, cosine learning rate (fjofc_mlp_backward / _adam);
   validation loss by fjofc_mlp_loss.
5. Evaluation on held-out objects: the plain random start runs `oos_iters`
   transforms and defines each object's reference stress.  Then, each until
   its stress is within `rel` of the reference (fjofc_oos target, the same
   iteration cap): the same plain start again, the learned start (features +
   network, fjofc_mlp_predict_start) and the nearest-in-sample start.  Every
   pipeline runs in calls of `oos_batch` objects.  Iterations per object and
   the wall time of each whole start-plus-refine pipeline are reported.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import fjofc


@dataclass
class WarmStartConfig:
    landmarks: int = 256
    hidden: int = 512
    depth: int = 3            # hidden layers
    train_objects: int = 200000
    val_frac: float = 0.05
    epochs: int = 20
    batch: int = 1024
    lr: float = 1e-3
    oos_iters: int = 100
    oos_batch: int = 4096     # objects per fjofc_oos call (and network call), every pipeline
    chunk: int = 20000        # training objects generated per chunk
    rel: float = 1e-4
    per_modality: bool = True  # False: one consensus point (d outputs)
    target_iters: int = 300   # cap of the transforms that make training targets
    target_tol: float = 1e-7  # ... stopped when the stress decreases by less
    seed_landmarks: int = 22
    seed_train: int = 21
    seed_eval: int = 20
    seed_start: int = 23
    seed_init: int = 24


class Problem:
    """In-sample side: views, maps, weights and the embedded X (device)."""

    def __init__(self, ctx, spec, device):
        import torch
        from workloads import generators as gen
        self.spec = spec
        self.device = device
        self.views, self.maps, X0 = gen.latent_views(spec.seed_in, spec.n, spec.m, spec.lat,
                                                     spec.sigma, spec.d)
        delta = [gen.pairwise_dist_torch(Y, device) for Y in self.views]
        self.wmat = gen.uniform_wmat(spec.m, spec.w)
        self.X = torch.from_numpy(X0.astype(np.float32)).to(device)
        self.in_result, _ = fjofc.fjofc_embed(ctx, delta, self.wmat, self.X, spec.in_iters,
                                              stress_every=spec.in_iters)
        del delta
        self.scale = float(torch.sqrt((self.X.double() ** 2).mean()))

    def new_delta(self, new_views, o0, o1, out=None):
        """k x m x n FP32 dissimilarities of new objects o0..o1-1."""
        import torch
        from workloads import generators as gen
        sp = self.spec
        k = o1 - o0
        if out is None:
            out = torch.empty((k, sp.m, sp.n), dtype=torch.float32, device=self.device)
        for i in range(sp.m):
            out[:, i, :] = gen.cross_dist_torch(new_views[i][o0:o1], self.views[i], self.device)
        return out

    def plain_start(self, seed, k):
        import torch
        from workloads import generators as gen
        sp = self.spec
        return torch.from_numpy(gen.gaussian_start(seed, (k, sp.m, sp.d), self.scale)
                                .astype(np.float32)).to(self.device)


def _run_oos(ctx, prob, dnew, Y, iters, batch, target=None, stress=None, its=None):
    k = dnew.shape[0]
    for o0 in range(0, k, batch):
        o1 = min(k, o0 + batch)
        fjofc.fjofc_oos(ctx, prob.X, prob.wmat, dnew[o0:o1], Y[o0:o1], iters,
                        target=None if target is None else target[o0:o1],
                        stress_out=None if stress is None else stress[o0:o1],
                        iters_out=None if its is None else its[o0:o1], sync=False)


def training_data(ctx, prob, cfg: WarmStartConfig, landmarks, log=print):
    """Raw landmark features (FP32, for the statistics) and the converged
    out-of-sample points (N x m x d) of the training objects, generated
    chunk by chunk."""
    import torch
    from workloads import generators as gen
    sp = prob.spec
    new = gen.oos_objects(cfg.seed_train, cfg.train_objects, prob.maps, sp.sigma)
    raw = torch.empty((cfg.train_objects, sp.m * cfg.landmarks), dtype=torch.float32,
                      device=prob.device)
    Yt = torch.empty((cfg.train_objects, sp.m, sp.d), dtype=torch.float32, device=prob.device)
    buf = None
    lm = landmarks.long()
    its_all = []
    for o0 in range(0, cfg.train_objects, cfg.chunk):
        o1 = min(cfg.train_objects, o0 + cfg.chunk)
        buf = prob.new_delta(new, o0, o1, None if buf is None or buf.shape[0] != o1 - o0 else buf)
        Y = Yt[o0:o1]
        fjofc.fjofc_oos_nearest_start(ctx, prob.X, buf, Y)
        its = torch.empty(o1 - o0, dtype=torch.int32, device=prob.device)
        fjofc.fjofc_oos(ctx, prob.X, prob.wmat, buf, Y, cfg.target_iters, tol=cfg.target_tol,
                        iters_out=its, sync=False)
        raw[o0:o1] = buf[:, :, lm].reshape(o1 - o0, -1)
        its_all.append(its)
        log(f"[warmstart] training data {o1}/{cfg.train_objects}")
    torch.cuda.synchronize()
    its = torch.cat(its_all).float()
    log(f"[warmstart] target transforms: mean {float(its.mean()):.1f}, "
        f"capped {float((its >= cfg.target_iters).float().mean()):.3f}")
    return raw, Yt


def targets(ctx, Yt, per_modality: bool):
    """Network targets from the converged points: every modality's point
    (N x m d) or the consensus point (N x d)."""
    import torch
    N, m, d = Yt.shape
    if per_modality:
        return Yt.reshape(N, m * d)
    out = torch.empty((N, d), dtype=torch.float32, device=Yt.device)
    return fjofc.fjofc_oos_consensus(ctx, Yt, out)


def train_network(ctx, raw, tgt, cfg: WarmStartConfig, log=print):
    """Standardise, split off a validation set, train with Adam and a cosine
    learning rate.  Returns (net, mu, inv_sd, history)."""
    import torch
    N = raw.shape[0]
    mu = torch.empty(raw.shape[1], dtype=torch.float32, device=raw.device)
    inv_sd = torch.empty_like(mu)
    fjofc.fjofc_mlp_feature_stats(ctx, raw, mu, inv_sd, min_sd=1e-6)
    dims = [raw.shape[1]] + [cfg.hidden] * cfg.depth + [tgt.shape[1]]
    rng = np.random.default_rng(cfg.seed_init)
    W = [torch.from_numpy((rng.standard_normal((a, b)) * math.sqrt(2.0 / a)).astype(np.float32))
         .to(raw.device) for a, b in zip(dims[:-1], dims[1:])]
    b = [torch.zeros(c, dtype=torch.float32, device=raw.device) for c in dims[1:]]
    net = fjofc.Mlp(ctx, dims, cfg.batch)
    net.set_params(W, b)
    # standardise with the feature kernel: raw is N x m x L, landmarks 0..L-1
    m = raw.shape[1] // cfg.landmarks
    xs = torch.empty(raw.shape, dtype=torch.bfloat16, device=raw.device)
    ident = torch.arange(cfg.landmarks, dtype=torch.int32, device=raw.device)
    fjofc.fjofc_mlp_features(ctx, raw.view(N, m, cfg.landmarks), ident, mu, inv_sd, xs)
    perm0 = torch.from_numpy(rng.permutation(N)).to(raw.device)
    nval = int(N * cfg.val_frac)
    val_idx, tr_idx = perm0[:nval], perm0[nval:]
    ntr = tr_idx.shape[0]
    steps_per_epoch = ntr // cfg.batch
    total = steps_per_epoch * cfg.epochs
    hist = []
    step = 0
    for ep in range(cfg.epochs):
        order = tr_idx[torch.from_numpy(rng.permutation(ntr)).to(raw.device)]
        xe, ye = xs[order], tgt[order]
        acc = torch.zeros(1, dtype=torch.float64, device=raw.device)
        # one library call per epoch: consecutive batches of the shuffled
        # rows, each with its cosine learning rate
        lrs = [cfg.lr * 0.5 * (1.0 + math.cos(math.pi * (step + s) / max(1, total)))
               for s in range(steps_per_epoch)]
        net.train_steps(xe, ye, cfg.batch, lrs, acc)
        step += steps_per_epoch
        vl = evaluate_loss(net, xs[val_idx], tgt[val_idx], cfg.batch)
        hist.append({"epoch": ep, "train_mse": float(acc.item() / steps_per_epoch), "val_mse": vl})
        log(f"[warmstart] epoch {ep}: train {hist[-1]['train_mse']:.4e} val {vl:.4e}")
    return net, mu, inv_sd, hist


def evaluate_loss(net, x, y, batch):
    """Mean squared error over x (library forward and MSE kernels)."""
    import torch
    tot = 0.0
    loss = torch.zeros(1, dtype=torch.float64, device=x.device)
    for o0 in range(0, x.shape[0], batch):
        o1 = min(x.shape[0], o0 + batch)
        net.loss(x[o0:o1], y[o0:o1], loss)
        tot += float(loss.item()) * (o1 - o0)
    return tot / x.shape[0]


def evaluate(ctx, prob, nets, landmarks, cfg: WarmStartConfig, k: int = 50000, log=print):
    """On k held-out objects: the plain start's reference run, then the time
    and transforms each start needs to reach that reference stress within
    `rel` (the same start, every learned start in `nets`, the
    nearest-in-sample start).  `nets` maps a name to (net, mu, inv_sd).
    Every pipeline runs in calls of cfg.oos_batch objects."""
    import torch
    from workloads import generators as gen
    sp = prob.spec
    dev = prob.device
    nb = cfg.oos_batch
    new = gen.oos_objects(cfg.seed_eval, k, prob.maps, sp.sigma)
    dnew = prob.new_delta(new, 0, k)
    Y0 = prob.plain_start(cfg.seed_start, k)
    torch.cuda.synchronize()

    # plain start: the reference run (oos_iters transforms, no stop rule)
    Yp = Y0.clone()
    sp_stress = torch.empty(k, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _run_oos(ctx, prob, dnew, Yp, cfg.oos_iters, nb, stress=sp_stress)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    target = sp_stress * (1.0 + cfg.rel)

    def refine(Ystart, o0, o1, st, it):
        fjofc.fjofc_oos(ctx, prob.X, prob.wmat, dnew[o0:o1], Ystart[o0:o1], cfg.oos_iters,
                        target=target[o0:o1], stress_out=st[o0:o1], iters_out=it[o0:o1],
                        sync=False)

    def timed(start_fn):
        """start_fn(o0, o1, Y) writes the start of objects o0..o1-1 into Y;
        the pipeline (start + refine) runs call by call and is timed whole."""
        Y = torch.empty((k, sp.m, sp.d), dtype=torch.float32, device=dev)
        st = torch.empty(k, dtype=torch.float64, device=dev)
        it = torch.empty(k, dtype=torch.int32, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for o0 in range(0, k, nb):
            o1 = min(k, o0 + nb)
            start_fn(o0, o1, Y)
            refine(Y, o0, o1, st, it)
        torch.cuda.synchronize()
        return st, it, time.perf_counter() - t0

    def summ(st, it, t):
        itn = it.cpu().numpy()
        ok = (st <= target).cpu().numpy()
        return {"seconds": t, "iters_mean": float(itn.mean()),
                "iters_p50": float(np.percentile(itn, 50)),
                "iters_p99": float(np.percentile(itn, 99)),
                "reached_frac": float(ok.mean())}

    res = {"objects": k, "rel": cfg.rel, "oos_iters_cap": cfg.oos_iters, "call_objects": nb,
           "plain": {"seconds": t_plain, "iters": cfg.oos_iters,
                     "mean_stress": float(sp_stress.mean())}}

    # the plain start again, stopped by the same target rule
    def plain_copy(o0, o1, Y):
        Y[o0:o1].copy_(Y0[o0:o1])
    res["plain_target"] = summ(*timed(plain_copy))

    # learned starts: features + network + refinement, timed together
    x = torch.empty((k, sp.m * cfg.landmarks), dtype=torch.bfloat16, device=dev)
    for name, (net, mu, inv_sd) in nets.items():
        ninf = fjofc.Mlp(ctx, net.dims, nb)
        ninf.set_params(*net.get_params())

        def learned(o0, o1, Y, ninf=ninf, mu=mu, inv_sd=inv_sd):
            fjofc.fjofc_mlp_features(ctx, dnew[o0:o1], landmarks, mu, inv_sd, x[o0:o1])
            ninf.predict_start(x[o0:o1], Y[o0:o1])
        res[name] = summ(*timed(learned))
        res[name]["outputs"] = net.dims[-1]
        ninf.close()

    # nearest-in-sample start (comparison)
    def nearest(o0, o1, Y):
        fjofc.fjofc_oos_nearest_start(ctx, prob.X, dnew[o0:o1], Y[o0:o1])
    res["nearest"] = summ(*timed(nearest))

    w = res["warm"]
    res["speedup_vs_plain"] = t_plain / w["seconds"]
    res["speedup_vs_plain_target"] = res["plain_target"]["seconds"] / w["seconds"]
    res["speedup_vs_nearest"] = res["nearest"]["seconds"] / w["seconds"]
    for name in ["plain_target", *nets.keys(), "nearest"]:
        r = res[name]
        log(f"[warmstart] {name}: {r['seconds']:.4f}s, mean {r['iters_mean']:.1f} transforms, "
            f"reached {r['reached_frac']:.4f}")
    log(f"[warmstart] plain reference {t_plain:.4f}s")
    return res


def run(ctx, cfg: Optional[WarmStartConfig] = None, eval_objects: int = 50000, log=print,
        spec=None, ablation: bool = False):
    """The whole learned warm-start workload; returns a summary dict.  `spec`
    defaults to the out-of-sample workload (m=2, n=10000, d=5).  The network
    of cfg is reported as "warm"; with `ablation` a second network with the
    other output layout (per-modality points vs one consensus point) is
    trained on the same objects and reported beside it."""
    import dataclasses
    import torch
    from workloads import generators as gen
    cfg = cfg or WarmStartConfig()
    spec = spec or gen.config2_spec()
    dev = torch.device("cuda:0")
    prob = Problem(ctx, spec, dev)
    rng = np.random.default_rng(cfg.seed_landmarks)
    landmarks = torch.from_numpy(rng.choice(spec.n, cfg.landmarks, replace=False)
                                 .astype(np.int32)).to(dev)
    cfgs = {"warm": cfg}
    if ablation:
        alt = "warm_per_modality" if not cfg.per_modality else "warm_consensus"
        cfgs[alt] = dataclasses.replace(cfg, per_modality=not cfg.per_modality)
    nets, info = {}, {}
    t1 = time.perf_counter()
    raw, Yt = training_data(ctx, prob, cfg, landmarks, log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t1
    for name, c in cfgs.items():
        t2 = time.perf_counter()
        net, mu, inv_sd, hist = train_network(ctx, raw, targets(ctx, Yt, c.per_modality), c, log)
        torch.cuda.synchronize()
        nets[name] = (net, mu, inv_sd)
        info[name] = {"outputs": net.dims[-1], "per_modality": c.per_modality,
                      "train_seconds": time.perf_counter() - t2,
                      "final_val_mse": hist[-1]["val_mse"]}
    del raw, Yt
    ev = evaluate(ctx, prob, nets, landmarks, cfg, eval_objects, log)
    for net, _, _ in nets.values():
        net.close()
    return {"workload": f"warm_start_m{spec.m}_n{spec.n}_d{spec.d}",
            "train_objects": cfg.train_objects, "epochs": cfg.epochs,
            "networks": info, "data_seconds": t_data,
            "train_seconds": info["warm"]["train_seconds"],
            "final_val_mse": info["warm"]["final_val_mse"], "eval": ev}
