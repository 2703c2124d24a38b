"""Training of the bucket-triage network on pairs the method itself produces.

    python -m paper_1605_06904_amd.triage_train [--out PATH] [--pairs 200000]

1. Run the full path (every enriched bucket refined) on generated workloads:
   one (18,6) instance of the plain-at-scale shape and an uneven batch of
   the batching shape (t, n, l drawn per instance, d = floor(l/4) + 1,
   k = clamp(l - d - 4, 6, 9), s = 3), each shape class as one batch.
2. Each refined bucket gives one pair: its features (the library's
   triage_features) and its post-EM outcome: 1 when its refinement ends at the
   motif of its instance's winner (same consensus), else 0 -- what triage must
   rank.  Winning buckets are rare and are kept up to a third of the pairs.
   (--label planted: 1 when the refinement ends at the motif planted in the
   instance, which the generator knows; --label llr: the post-EM
   LLR(theta^iters) / t standardised within the instance.)
3. Standardise features and scores with the training statistics, train the
   network with the library's FP32 forward/backward and Adam kernels on
   mini-batches, then fold the score standardisation into the last layer.
4. Fallback threshold per motif length l: run the triaged pipeline (no
   fallback) over the training instances with the trained network and take
   the 1st percentile of the triaged winner's z-score (its J among the J of
   the instance's refined buckets) over the instances whose triaged winner
   is the planted motif (the pooled value for lengths with no such instance).
   A z-score carries no scale of t or n, so it transfers across shapes.

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


def _run_full(pm, torch, insts, l, k, s, iters, bg, label="winner"):
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
    res = P.results()
    if label == "winner":
        # 1 where the bucket's refinement ends at the instance winner's motif
        # (same consensus), else 0: the post-EM outcome triage has to rank
        cons = P.b.theta[:nb_].argmax(dim=1)            # [nb, l] letter codes (label bookkeeping)
        best = torch.tensor([max(r["best"], 0) for r in res], device="cuda")
        inst_d = torch.from_numpy(inst_of.astype(np.int64)).cuda()
        win_cons = cons[best[inst_d]]
        has = torch.tensor([r["best"] >= 0 for r in res], device="cuda")[inst_d]
        score = ((cons == win_cons).all(dim=1) & has).float().cpu().numpy()
    elif label == "planted":
        # 1 where the bucket's refinement ends at the motif planted in its
        # instance (the generator knows it; serving never needs it), else 0
        order = pm.code_order(4)
        planted = torch.tensor([[order.index(ch) for ch in inst.motif] for inst, _ in insts], device="cuda")
        cons = P.b.theta[:nb_].argmax(dim=1)
        inst_d = torch.from_numpy(inst_of.astype(np.int64)).cuda()
        score = (cons == planted[inst_d]).all(dim=1).float().cpu().numpy()
    else:
        t = np.array(B.t)[inst_of]
        score = P.b.llr[:nb_, -1].cpu().numpy() / t
        # the network sees a bucket, not its instance (no t, n): keep only the
        # within-instance part of the score, standardised per instance
        for p in np.unique(inst_of):
            sel = inst_of == p
            mu, sd = score[sel].mean(), score[sel].std()
            score[sel] = (score[sel] - mu) / (sd if sd > 0 else 1.0)
    winners = []
    for p, (inst, _) in enumerate(insts):
        r = res[p]
        if r["best"] >= 0:
            winners.append((l, r["J"] / B.t[p], r["consensus"] == inst.motif))
    return feat.cpu().numpy(), score, winners


def collect(pm, torch, seed: int, batch_count: int, batch_m: int, label: str = "winner", extra_c1: int = 0,
            log=print):
    from synth import batch_config, make_config
    bg = np.full(4, 0.25)
    X, y, win, groups = [], [], [], []
    inst, masks = make_config("c2", seed=seed)
    cfg = inst.meta
    out = _run_full(pm, torch, [(inst, masks)], cfg["l"], cfg["k"], cfg["s"], cfg["iters"], bg, label)
    X.append(out[0])
    y.append(out[1])
    win += out[2]
    groups.append(([(inst, masks)], cfg["l"], cfg["k"], cfg["s"], cfg["iters"]))
    log(f"(18,6) instance: {len(out[1])} pairs")
    if extra_c1:
        # instances of the (15,4) plain shape the network serves (seeds apart
        # from every evaluation seed)
        c1 = [make_config("c1", seed=30000 + seed + i) for i in range(extra_c1)]
        cfg1 = c1[0][0].meta
        out = _run_full(pm, torch, c1, cfg1["l"], cfg1["k"], cfg1["s"], cfg1["iters"], bg, label)
        X.append(out[0])
        y.append(out[1])
        win += out[2]
        groups.append((c1, cfg1["l"], cfg1["k"], cfg1["s"], cfg1["iters"]))
        log(f"(15,4) instances: {extra_c1}, {len(out[1])} pairs")
    insts = batch_config(seed, count=batch_count, m=batch_m)
    classes = {}
    for inst, masks in insts:
        classes.setdefault(inst.meta["l"], []).append((inst, masks))
    for l in sorted(classes):
        group = classes[l]
        meta = group[0][0].meta
        out = _run_full(pm, torch, group, l, meta["k"], meta["s"], meta["iters"], bg, label)
        if out is None:
            continue
        X.append(out[0])
        y.append(out[1])
        win += out[2]
        groups.append((group, l, meta["k"], meta["s"], meta["iters"]))
        log(f"batch class l={l}: {len(group)} instances, {len(out[1])} pairs")
    return X, y, win, groups


def triaged_z(pm, torch, tri, groups, frac: float):
    """(l, z of the triaged winner, triaged winner is the planted motif) for
    every training instance, from the library's triaged pipeline without
    fallback."""
    bg = np.full(4, 0.25)
    rows = []
    for insts, l, k, s, iters in groups:
        B = pm.Batch(4, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])
        nb_, nm_ = pm.size_batch(B, s)
        if nb_ == 0:
            continue
        TP = pm.TriagedBatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_, tri, frac=frac)
        TP.threshold = -math.inf
        TP.run()
        for r, (inst, _) in zip(TP.results(), insts):
            if r["best"] >= 0:
                rows.append((l, r["z"], r.get("consensus") == inst.motif))
        del TP, B
        torch.cuda.empty_cache()
    return rows


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
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-m", type=int, default=20)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--mb", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--frac", type=float, default=0.05)
    ap.add_argument("--label", choices=["winner", "planted", "llr"], default="winner")
    ap.add_argument("--extra-c1", type=int, default=0, help="(15,4) instances added to the training runs")
    args = ap.parse_args(argv)
    import torch

    import paper_1605_06904_amd as pm
    t0 = time.time()
    log = lambda *a: print("[triage-train]", *a, flush=True)
    Xs, ys, win, groups = collect(pm, torch, args.seed, args.batch_count, args.batch_m, args.label, args.extra_c1,
                                  log)
    X, y = np.concatenate(Xs), np.concatenate(ys)
    rng = np.random.default_rng(args.seed)
    if args.label in ("winner", "planted"):
        # positive buckets are rare: keep them up to a third of the pairs
        pos, neg = np.nonzero(y > 0.5)[0], np.nonzero(y <= 0.5)[0]
        npos = min(len(pos), args.pairs // 3)
        keep = np.concatenate([rng.choice(pos, size=npos, replace=False),
                               rng.choice(neg, size=min(len(neg), args.pairs - npos), replace=False)])
        log(f"winning buckets: {len(pos)} of {len(y)}; kept {npos}")
        X, y = X[keep], y[keep]
    elif len(y) > args.pairs:
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
    zrows = triaged_z(pm, torch, pm.Triage(params, mu, sd, -math.inf), groups, args.frac)
    pooled, per_l = thresholds(zrows)
    log(f"triaged winners: {len(zrows)}, planted {sum(ok for _, _, ok in zrows)}; full EM winners planted: "
        f"{sum(ok for _, _, ok in win)} of {len(win)}")
    meta = dict(pairs=int(len(y)), seed=args.seed, extra_c1=args.extra_c1, epochs=args.epochs, minibatch=args.mb, lr=args.lr,
                fallback="z-score of the triaged winner's J among the instance's refined buckets",
                frac=args.frac, triaged_solved=int(sum(ok for _, _, ok in zrows)),
                label={"winner": "1 if the bucket's refinement ends at the instance winner's consensus",
                       "planted": "1 if the bucket's refinement ends at the planted motif's consensus",
                       "llr": "LLR(theta^iters)/t, standardised within the instance"}[args.label],
                thresholds_by_l=per_l, threshold_pooled=pooled,
                winners=len(win), solved_winners=int(sum(ok for _, _, ok in win)),
                seconds=round(time.time() - t0, 1))
    tri = pm.Triage(params, mu, sd, pooled, meta=meta)
    tri.save(args.out)
    tri.save_bin(os.path.splitext(args.out)[0] + ".bin")
    log(f"saved {args.out}: {json.dumps(meta)}")


if __name__ == "__main__":
    main()
