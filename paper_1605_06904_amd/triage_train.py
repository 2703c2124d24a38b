"""Training of the bucket-triage network on pairs the method itself produces.

    python -m paper_1605_06904_amd.triage_train [--out PATH] [--pairs 200000]

1. Run the full path (every enriched bucket refined) on generated workloads:
   one (18,6) instance of the plain-at-scale shape and an uneven batch of
   the batching shape (t, n, l drawn per instance, d = floor(l/4) + 1,
   k = clamp(l - d - 4, 6, 9), s = 3), each shape class as one batch.
2. Each refined bucket gives one pair: its features (the library's
   triage_features) and its post-EM score LLR(theta^iters) / t.
3. Standardise features and scores with the training statistics, train the
   network with the library's FP32 forward/backward and Adam kernels on
   mini-batches, then fold the score standardisation into the last layer.
4. Fallback threshold per motif length l: the 1st percentile of the winner's
   J(theta^iters) / t over training instances whose winner is the planted
   motif (the pooled value for lengths with no such instance).

Every step of the arithmetic runs in the library's kernels; this module only
moves arrays, draws the mini-batches and keeps the bookkeeping.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def _run_full(pm, torch, insts, l, k, s, iters, bg):
    """Full path over one shape class: raw features, scores, per-instance
    winners."""
    B = pm.Batch(4, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])
    nb_, nm_ = pm.size_batch(B, s)
    if nb_ == 0:
        return None
    P = pm.BatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_)
    P.run()
    feat = torch.zeros((nb_, pm.PM_TRIAGE_INPUTS), dtype=torch.float32, device="cuda")
    pm.triage_features(l, P.b.profile, nb_, P.b.n_out, P.bg, None, None, feat)
    torch.cuda.synchronize()
    bk = P.b.buckets[:nb_].cpu().numpy().view(np.uint32)
    inst_of = B.item_inst.cpu().numpy()[bk[:, 0]]
    t = np.array(B.t)[inst_of]
    score = P.b.llr[:nb_, -1].cpu().numpy() / t
    res = P.results()
    winners = []
    for p, (inst, _) in enumerate(insts):
        r = res[p]
        if r["best"] >= 0:
            winners.append((l, r["J"] / B.t[p], r["consensus"] == inst.motif))
    return feat.cpu().numpy(), score, winners


def collect(pm, torch, seed: int, batch_count: int, batch_m: int, log=print):
    from synth import batch_config, make_config
    bg = np.full(4, 0.25)
    X, y, win = [], [], []
    inst, masks = make_config("c2", seed=seed)
    cfg = inst.meta
    out = _run_full(pm, torch, [(inst, masks)], cfg["l"], cfg["k"], cfg["s"], cfg["iters"], bg)
    X.append(out[0])
    y.append(out[1])
    win += out[2]
    log(f"(18,6) instance: {len(out[1])} pairs")
    insts = batch_config(seed, count=batch_count, m=batch_m)
    classes = {}
    for inst, masks in insts:
        classes.setdefault(inst.meta["l"], []).append((inst, masks))
    for l in sorted(classes):
        group = classes[l]
        meta = group[0][0].meta
        out = _run_full(pm, torch, group, l, meta["k"], meta["s"], meta["iters"], bg)
        if out is None:
            continue
        X.append(out[0])
        y.append(out[1])
        win += out[2]
        log(f"batch class l={l}: {len(group)} instances, {len(out[1])} pairs")
    return X, y, win


def train(pm, torch, X, y, epochs: int, batch: int, lr: float, seed: int, log=print):
    """Adam on mini-batches with the library's FP32 training kernels.
    X, y already standardised.  Returns the FP32 parameter vector."""
    rng = np.random.default_rng(seed)
    sizes = (pm.PM_TRIAGE_INPUTS, 256, 256, 1)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / a), size=a * b))
        parts.append(np.zeros(b))
    params = torch.from_numpy(np.concatenate(parts).astype(np.float32)).cuda()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    dX = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    dy = torch.from_numpy(np.ascontiguousarray(y, dtype=np.float32)).cuda()
    N = len(y)
    wsb = pm.pm_triage_workspace(batch)
    ws = torch.zeros((wsb + 3) // 4, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    step = 0
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).cuda()
        Xp, yp = dX[perm].contiguous(), dy[perm].contiguous()  # shuffled copies (data movement)
        tot = 0.0
        nb = N // batch
        for i in range(nb):
            step += 1
            pm.triage_train_step(params, m, v, step, Xp[i * batch:(i + 1) * batch],
                                 yp[i * batch:(i + 1) * batch], batch, lr, loss, None, ws, wsb)
            if i % 50 == 0 or i == nb - 1:
                tot = float(loss.item())
        log(f"epoch {ep + 1}/{epochs}: last mini-batch loss {tot:.4f}")
    torch.cuda.synchronize()
    return params.cpu().numpy()


def thresholds(winners, pct=1.0):
    solved = [(l, j) for l, j, ok in winners if ok]
    pooled = float(np.percentile([j for _, j in solved], pct)) if solved else -math.inf
    per_l = {}
    for l in sorted({l for l, _ in solved}):
        per_l[int(l)] = float(np.percentile([j for ll, j in solved if ll == l], pct))
    return pooled, per_l


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "triage_weights.npz"))
    ap.add_argument("--pairs", type=int, default=200000)
    ap.add_argument("--seed", type=int, default=101)
    ap.add_argument("--batch-count", type=int, default=48)
    ap.add_argument("--batch-m", type=int, default=60)
    ap.add_argument("--epochs", type=int, default=12)
    ap.add_argument("--mb", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    args = ap.parse_args(argv)
    import torch

    import paper_1605_06904_amd as pm
    t0 = time.time()
    log = lambda *a: print("[triage-train]", *a, flush=True)
    Xs, ys, win = collect(pm, torch, args.seed, args.batch_count, args.batch_m, log)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    rng = np.random.default_rng(args.seed)
    if len(y) > args.pairs:
        keep = rng.choice(len(y), size=args.pairs, replace=False)
        X, y = X[keep], y[keep]
    log(f"{len(y)} pairs collected in {time.time() - t0:.1f} s")
    mu, sd = X.mean(axis=0), X.std(axis=0)
    sd[sd < 1e-6] = 1.0
    ymu, ysd = float(y.mean()), float(y.std() or 1.0)
    Xs_ = (X - mu) / sd
    ys_ = (y - ymu) / ysd
    params = train(pm, torch, Xs_, ys_, args.epochs, args.mb, args.lr, args.seed, log)
    # fold the score standardisation into the output layer: y = ysd * y' + ymu
    n_w3 = 256
    o_w3 = pm.PM_TRIAGE_PARAMS - 1 - n_w3
    params[o_w3:o_w3 + n_w3] *= ysd
    params[-1] = params[-1] * ysd + ymu
    pooled, per_l = thresholds(win)
    meta = dict(pairs=int(len(y)), seed=args.seed, epochs=args.epochs, minibatch=args.mb, lr=args.lr,
                label="LLR(theta^iters)/t", thresholds_by_l=per_l, threshold_pooled=pooled,
                winners=len(win), solved_winners=int(sum(ok for _, _, ok in win)),
                seconds=round(time.time() - t0, 1))
    tri = pm.Triage(params, mu, sd, pooled, meta=meta)
    tri.save(args.out)
    log(f"saved {args.out}: {json.dumps(meta)}")


if __name__ == "__main__":
    main()
