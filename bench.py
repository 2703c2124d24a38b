#!/usr/bin/env python3
"""Benchmark of the PROJECTION hot path on one MI355X.

One step = one whole pass of the path over the (18,6) DNA workload (t = 20
sequences of n = 1000, planted (18,6) motif, k = 8, s = 4, m = 5000 trials,
10 EM iterations in FP32-class arithmetic): projection + keys + bucket histogram for all trials,
enriched-bucket selection, profiles and theta^0, EM of every enriched bucket,
and the pick of the best model.  Inputs are seeded, synthetic and resident in
HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP16_MFMA_PEAK = 2500.0      # TFLOP/s, MI355X dense FP16 matrix cores

# HBM bytes per launch from the FETCH_SIZE/WRITE_SIZE counter runs recorded in
# profiles/hbm_traffic_dna_18-6_m5000.md (copy-calibrated), valid only while
# the kernel source is the one they were taken on (sha256 prefix).
MEASURED_TRAFFIC = {
    "hash.hip": ("8544af7b0b679691", {"k_hash<4,8>": 1.705e9, "k_hash<4,9>": 14.492e9, "k_hash<20,4>": 1.517e9}),
    "em_mfma.hip": ("ff6a29f1b25ea3d3", {
        "k_em_mfma<5,2,true,1,1>": 0.740e9 + 0.694e9,
        "k_em_mfma<5,2,true,2,1>": 0.699e9 + 0.705e9,
        "k_em_mfma<5,2,true,4,1>": 0.732e9 + 0.693e9,
        "k_em_mfma<5,2,true,1,2>": 0.745e9 + 0.723e9,
        "k_em_mfma<5,2,true,2,2>": 0.733e9 + 0.731e9,
        "k_em_mfma<5,2,true,4,2>": 0.763e9 + 0.742e9,
    }),
}


def traffic(src, kernel):
    """HBM bytes per launch of `kernel` measured with the counters, or None when
    the kernel's source has changed since they were taken."""
    import hashlib
    sha, per_kernel = MEASURED_TRAFFIC[src]
    path = os.path.join(ROOT, "paper_1605_06904_amd", "csrc", src)
    with open(path, "rb") as f:
        cur = hashlib.sha256(f.read()).hexdigest()[:16]
    return per_kernel.get(kernel) if cur == sha else None


def em_issued_flops(S, l, iters, nbk, split):
    """FLOPs the matrix-core EM issues for nbk models: per 16 models and
    32-window pair of a sequence (partial pairs padded), 2 ceil(MT/2) E-step
    MFMAs in each of iters + 1 E-steps and MT M-step MFMAs in each of iters
    M-steps, MT = ceil(l/4), each 16x16x32 (16 384 FLOPs), doubled by the
    split halves except the last E-step k-block when MT is odd (its hi and
    lo halves share one MFMA); models padded to groups of 16."""
    mt = (l + 3) // 4
    lb = (mt + 1) // 2
    pairs = sum((n - l + 1 + 31) // 32 for n in S.lens)
    groups = (nbk + 15) // 16
    e_step = 2 * (2 * lb - (mt & 1)) if split else 2 * lb
    m_step = mt * (2 if split else 1)
    per_pair = e_step * (iters + 1) + m_step * iters
    return float(groups) * pairs * per_pair * 16384.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also run one plain device copy of this many bytes (counter calibration)")
    ap.add_argument("--instances", type=int, default=256,
                    help="(15,4) instances for the instances/s leg (0: skip it)")
    ap.add_argument("--no-extra-hash", action="store_true",
                    help="skip the hash rooflines of the (21,7) DNA and (20,6) protein workloads")
    ap.add_argument("--c3-chunk", type=int, default=250,
                    help="trials per instance per chunk of the 512-instance uneven workload at m=1000 (0: skip)")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the timings of the sorted selection, ZOOPS/TCM, Gibbs and length-range rows")
    ap.add_argument("--uneven", type=int, default=0,
                    help="also run the 512-instance uneven batch with this many trials per instance")
    ap.add_argument("--c5", action="store_true",
                    help="also run one (21,7) instance (t=50, n=2000, k=9, s=3, m=10000) with and without triage")
    ap.add_argument("--c4", action="store_true",
                    help="also time the protein (20,6) EM (t=30, n=1000, k=4, s=3, m=2000): the matrix-core "
                         "precision form against the FP64 vector path, with its error")
    return ap.parse_args()


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_events(torch, n):
    return [torch.cuda.Event(enable_timing=True) for _ in range(n)]


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the benchmark runs the path on exactly one GPU (the multi-GPU split is not implemented); --gpus must be 1"}), flush=True)
        sys.exit(2)
    import torch

    import paper_1605_06904_amd as pm
    from synth import make_config

    torch.cuda.set_device(0)
    PREC = pm.PM_F16X2
    inst, masks = make_config("c2", seed=args.seed)
    cfg = inst.meta
    A, l, k, s, m, iters = 4, cfg["l"], cfg["k"], cfg["s"], cfg["m"], cfg["iters"]
    beta = 1.0
    bg = np.full(4, 0.25)
    S = pm.Seqs(A, inst.seqs)
    x = S.nwin(l)

    # size the bucket lists once (untimed), then allocate the pass buffers
    P0 = pm.Pipeline(S, l, k, s, masks, iters, beta, PREC, bg, cap_b=0, cap_m=0)
    P0.hash()
    P0.select()
    torch.cuda.synchronize()
    nbk, nmem = [int(v) for v in P0.b.n_out.cpu()]
    del P0
    torch.cuda.empty_cache()
    P = pm.Pipeline(S, l, k, s, masks, iters, beta, PREC, bg, cap_b=nbk, cap_m=nmem)

    for _ in range(args.warmup):
        P.run()
    torch.cuda.synchronize()
    # pick the EM tile shape for this workload (timed on its own buckets)
    b = P.b
    tune_th, tune_J = torch.zeros_like(b.theta), torch.zeros_like(b.J)
    # on all the pass's buckets: the shapes differ in workgroup size, so how
    # well the bucket count fills the device is part of what is timed
    tile_shape = pm.em_autotune(P.S, l, b.theta0, P.bg, nbk, iters, beta, PREC, tune_th, tune_J, ws=P.em_ws)
    shape_g, shape_ppb = tile_shape // 10, tile_shape % 10
    del tune_th, tune_J
    P.run()
    torch.cuda.synchronize()

    # timed region: K whole passes; per-stage HIP events on the launch stream
    names = ["hash+select", "profile+theta0", "em", "best"]
    per_stage = np.zeros(len(names))
    t_all0 = torch.cuda.Event(enable_timing=True)
    t_all1 = torch.cuda.Event(enable_timing=True)
    evs = [stage_events(torch, len(names) + 1) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_all0.record()
    for st in range(args.steps):
        e = evs[st]
        b, Sx = P.b, P.S
        e[0].record()
        P.hash_select()
        e[1].record()
        pm.bucket_profile(Sx, l, b.buckets, b.members, b.cap_m, b.cap_b, b.n_out, b.profile)
        pm.theta_init(A, l, b.profile, b.cap_b, b.n_out, P.bg, beta, b.theta0)
        e[2].record()
        pm.em_refine(Sx, l, b.theta0, P.bg, b.cap_b, b.n_out, iters, beta, P.precision, b.theta,
                     b.J, b.llr, b.sites, ws=P.em_ws)
        e[3].record()
        pm.em_best(b.J, b.cap_b, b.n_out, iters, b.theta, A, l, b.best, b.consensus)
        e[4].record()
    t_all1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    for e in evs:
        per_stage += [e[i].elapsed_time(e[i + 1]) for i in range(len(names))]
    per_stage /= args.steps
    ms_step = t_all0.elapsed_time(t_all1) / args.steps
    res = P.result()
    if res["status"] != 0:
        raise SystemExit(f"device status {res['status']}")

    lmers = m * x
    value = lmers / (ms_step / 1e3)
    stage = dict(zip(names, [round(float(v), 4) for v in per_stage]))
    # the hash kernel and the selection as separate calls (outside the timed
    # passes): the hash kernel's own rate, and what the fused call saves
    split = split_stages_leg(torch, P)

    # hashing: algorithmic bytes = 4 B key per l-mer + the dense u32 counts
    hash_bytes = 4.0 * lmers + 4.0 * m * A ** k
    hash_gbs = hash_bytes / (split["hash"] / 1e3) / 1e9
    # EM, algorithmic work: the column updates the method needs, l per
    # window-model in every E-step (iters + 1) and every M-step (iters), each
    # counted as one FLOP-equivalent against the FP16 matrix-core peak
    em_updates = float(nbk) * x * l * (2 * iters + 1)
    em_alg_tfs = em_updates / (stage["em"] / 1e3) / 1e12
    # what the matrix cores actually issue (MFMA utilisation): per 16 models and
    # 32-window pair, 2 ceil(ceil(l/4)/2) E-step and ceil(l/4) M-step
    # 16x16x32 MFMAs (16 384 FLOPs each), twice over in the split form
    em_mfma = em_issued_flops(S, l, iters, nbk, split=True)
    em_mfma_tfs = em_mfma / (stage["em"] / 1e3) / 1e12
    em_kernel = f"k_em_mfma<{(l + 3) // 4},2,true,{shape_ppb},{shape_g}>"
    dominant = max(stage, key=stage.get)
    if dominant == "hash+select":
        roof = {"kernel": "k_hash<4,8>", "bound": "hbm", "achieved": round(hash_gbs, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hash_gbs / HBM_PEAK_GBS, 4), "traffic": traffic("hash.hip", "k_hash<4,8>")}
    else:
        roof = {"kernel": em_kernel, "bound": "mfma", "achieved": round(em_alg_tfs, 3),
                "peak": FP16_MFMA_PEAK, "unit": "TFLOP/s", "frac": round(em_alg_tfs / FP16_MFMA_PEAK, 5),
                "traffic": traffic("em_mfma.hip", em_kernel),
                "work": "column updates (l per window-model per E- and M-step) as FLOP-equivalents",
                "updates_per_launch": em_updates,
                "mfma_util": {"issued_flops_per_launch": em_mfma, "achieved_tflops": round(em_mfma_tfs, 2),
                              "frac_of_peak": round(em_mfma_tfs / FP16_MFMA_PEAK, 4),
                              "note": "dense one-hot contractions as issued: split FP16 halves and padding included"}}
    out = {
        "metric": "projected l-mers/s (whole PROJECTION+EM pass, (18,6) DNA workload)",
        "value": round(value, 1),
        "unit": "l-mers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "wall_s": round(wall, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 keys/counts; EM on split-f16 MFMA with f32 accumulation, f64 per-sequence log-sum-exp",
        "data": "synthetic planted (18,6) motif, seeded",
        "config": {"workload": "(18,6) DNA: t=20, n=1000, k=8, s=4, m=5000 trials, 10 EM iterations",
                   "x_lmers_per_trial": x, "enriched_buckets": nbk, "members": nmem,
                   "em_tile_shape": f"{16 * shape_g} models per wave, {shape_ppb} window pairs per barrier "
                                    "(autotuned)",
                   "parallelism": "single GPU"},
        "stage_ms": stage,
        "separate_calls_ms": split,
        "roofline": roof,
        "roofline_hash": {"kernel": "k_hash<4,8>", "bound": "hbm", "achieved": round(hash_gbs, 2),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hash_gbs / HBM_PEAK_GBS, 4),
                          "traffic": traffic("hash.hip", "k_hash<4,8>"), "bytes_per_launch": hash_bytes},
        "hash_lmers_per_s": round(lmers / (split["hash"] / 1e3), 1),
        "em_column_updates_per_s": round(em_updates / (stage["em"] / 1e3), 1),
        "consensus": res.get("consensus"),
        "planted": inst.motif,
    }
    progress(f"pass timed: {ms_step:.3f} ms/step")
    out["fused_selection"] = fused_select_leg(torch, pm, P, l, k, s, m, nbk, nmem)
    if not args.no_next_rows:
        out["next_rows"] = next_rows_leg(torch, pm, P, inst, l, cfg, iters, beta, nbk)
    out["precision"] = precision_leg(torch, pm, P, l, iters, beta, nbk, ms_em=stage["em"])
    if args.instances > 0:
        out["instances"] = instances_leg(torch, pm, args.instances)
    if not args.no_extra_hash:
        out["roofline_hash_c5"] = hash_roofline(torch, pm, "c5")
        out["roofline_hash_c4"] = hash_roofline(torch, pm, "c4")
    if args.c3_chunk > 0:
        out["uneven_full_m"] = c3_full_leg(torch, pm, chunk=args.c3_chunk)
    if args.uneven > 0:
        out["uneven_batch"] = uneven_leg(torch, pm, args.uneven)
    if args.c5:
        out["triage_21_7"] = c5_leg(torch, pm)
    if args.c4:
        out["protein_20_6"] = c4_leg(torch, pm)
    if args.copy_probe:
        # a plain copy of known size, read once and written once, for scaling
        # the HBM byte counters of the kernels above
        src = torch.ones(args.copy_probe, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = args.copy_probe
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(inst, masks, cfg, bg, beta, nbk, args.cpu_budget)
    print(json.dumps(out), flush=True)


def split_stages_leg(torch, P, reps=5):
    """projection_hash and bucket_select as two calls on the pass's buffers
    (the pass runs projection_hash_select), in turn as a pass would make them:
    the hash kernel's own time, for its HBM roofline, and the selection with
    its counting pass."""
    P.hash()
    P.select()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
    for e in ev:
        e[0].record()
        P.hash()
        e[1].record()
        P.select()
        e[2].record()
    torch.cuda.synchronize()
    return {"hash": round(sum(e[0].elapsed_time(e[1]) for e in ev) / reps, 4),
            "select": round(sum(e[1].elapsed_time(e[2]) for e in ev) / reps, 4)}


def fused_select_leg(torch, pm, P, l, k, s, m, nbk, nmem, reps=5):
    """The same trials through the fused selection (projection, histogram and
    enriched-bucket lists with keys and counts kept on chip): its time beside
    the pass's hash + selection stage, and its lists against the pass's
    (records equal, members equal as sets per bucket)."""
    b = P.b
    nbytes = pm.pm_hash_select_workspace(P.S, l, k, m)
    ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    bk = torch.zeros((nbk, 4), dtype=torch.int32, device="cuda")
    mem = torch.zeros(nmem, dtype=torch.int32, device="cuda")
    pm.bucket_hash_select(P.S, l, k, P.masks, m, s, bk, nbk, mem, nmem, n_out, ws, nbytes)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pm.bucket_hash_select(P.S, l, k, P.masks, m, s, bk, nbk, mem, nmem, n_out, ws, nbytes)
    e1.record()
    torch.cuda.synchronize()
    same = bool(torch.equal(bk, b.buckets[:nbk]))
    if same:
        # members of every bucket as a set: sort within each bucket's slice
        seg = torch.repeat_interleave(torch.arange(nbk, device="cuda"), b.buckets[:nbk, 2].long())
        key = seg * (1 << 32) + mem.long().view(-1) % (1 << 32)
        ref = seg * (1 << 32) + b.members[:nmem].long() % (1 << 32)
        same = bool(torch.equal(torch.sort(key).values, torch.sort(ref).values))
    return {"ms": round(e0.elapsed_time(e1) / reps, 4), "lists_equal_to_pass": same,
            "note": "bucket_hash_select over the pass's trials: keys and counts never leave LDS"}


def next_rows_leg(torch, pm, P, inst, l, cfg, iters, beta, nbk, sample=4096, sort_m=1000, sort_k=14,
                  range_m=500):
    """The rows beyond the plain pass, on the (18,6) workload's sequences:
    ZOOPS and TCM EM (FP32 vector kernel, 10 iterations) and Gibbs site
    sampling (10 sweeps) of the first `sample` enriched buckets of the pass;
    the sorted selection at k = 14 (|Sigma|^k = 2^28, no count table) over
    `sort_m` trials; the motif-length range 16..20 (projection_run, host in
    and host out, `range_m` trials per length)."""
    S = P.S
    nb = min(sample, nbk)
    th0 = P.b.theta0[:nb].contiguous()
    dbg = P.bg
    out = {"buckets": nb}
    progress(f"next rows: ZOOPS/TCM, Gibbs on {nb} buckets, sorted selection k={sort_k}, length range 16..20")

    def timed(fn):
        fn()  # warm
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    th = torch.empty_like(th0)
    mix = torch.empty(nb, dtype=torch.float64, device="cuda")
    J = torch.empty((nb, iters + 1), dtype=torch.float64, device="cuda")
    for name, model in (("zoops", pm.PM_ZOOPS), ("tcm", pm.PM_TCM)):
        ms = timed(lambda: pm.em_refine_model(S, l, model, 0.5, th0, dbg, nb, None, iters, beta, pm.PM_FP32, th,
                                              mix, J))
        out[name] = {"ms": round(ms, 3), "us_per_model": round(1e3 * ms / nb, 3), "precision": "fp32 vector"}
    ms = timed(lambda: pm.em_refine(S, l, th0, dbg, nb, None, iters, beta, pm.PM_FP32, th, J))
    out["oops_fp32_vector"] = {"ms": round(ms, 3), "us_per_model": round(1e3 * ms / nb, 3)}
    F = torch.empty((nb, iters + 1), dtype=torch.float64, device="cuda")
    sites = torch.empty((nb, S.t), dtype=torch.int32, device="cuda")
    ms = timed(lambda: pm.gibbs_refine(S, l, th0, dbg, nb, None, iters, beta, 7, th, F, sites))
    out["gibbs"] = {"ms": round(ms, 3), "us_per_chain": round(1e3 * ms / nb, 3), "sweeps": iters}
    del th, mix, J, F, sites

    # sorted selection (large key space)
    rng = np.random.default_rng(5)
    from synth import projection_masks
    mk = projection_masks(rng, l, sort_k, sort_m)
    dm = torch.from_numpy(np.ascontiguousarray(mk, dtype=np.uint32).view(np.int32)).cuda()
    nbytes = pm.pm_sort_select_workspace(S, l, sort_k, sort_m)
    ws = torch.empty(max(nbytes, 16), dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    pm.bucket_sort_select(S, l, sort_k, dm, sort_m, 2, None, 0, None, 0, n_out, ws, nbytes)
    torch.cuda.synchronize()
    nb2, nm2 = [int(v) for v in n_out.cpu()]
    bk = torch.empty((max(nb2, 1), 4), dtype=torch.int32, device="cuda")
    mem = torch.empty(max(nm2, 1), dtype=torch.int32, device="cuda")
    ms = timed(lambda: pm.bucket_sort_select(S, l, sort_k, dm, sort_m, 2, bk, nb2, mem, nm2, n_out, ws, nbytes))
    x = S.nwin(l)
    out["sorted_selection"] = {"k": sort_k, "s": 2, "trials": sort_m, "ms": round(ms, 3),
                               "lmers_per_s": round(sort_m * x / (ms / 1e3), 1), "buckets": nb2, "members": nm2}
    del ws, bk, mem
    torch.cuda.empty_cache()

    # motif-length range, host in and host out
    prob = pm.Problem(seqs=inst.seqs, alphabet=4, l=cfg["l"], d=cfg["d"], k=0, s=0, m=range_m, seed=11)
    pm.projection_run_range(prob, 16, 20, em_iters=iters, precision=pm.PM_F16X2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, chosen = pm.projection_run_range(prob, 16, 20, em_iters=iters, precision=pm.PM_F16X2)
    sec = time.perf_counter() - t0
    out["length_range"] = {"lengths": "16..20", "trials_per_length": range_m, "s": round(sec, 3),
                           "chosen_l": chosen, "consensus": res[chosen - 16]["consensus"] if chosen >= 16 else "",
                           "k_per_length": [r["k"] for r in res], "note": "projection_run_range, host in and out"}
    return out


def precision_leg(torch, pm, P, l, iters, beta, nbk, ms_em, sample=512):
    """EM of the same enriched buckets in the single-FP16 form (timed), and
    the error of both matrix-core forms against the FP64 path on a sample of
    buckets (every (nbk / sample)-th one)."""
    b, S = P.b, P.S
    A = S.alphabet
    th16 = torch.zeros_like(b.theta)
    J16 = torch.zeros_like(b.J)
    pm.em_refine(S, l, b.theta0, P.bg, b.cap_b, b.n_out, iters, beta, pm.PM_F16, th16, J16, None, None, ws=P.em_ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        pm.em_refine(S, l, b.theta0, P.bg, b.cap_b, b.n_out, iters, beta, pm.PM_F16, th16, J16, None, None,
                     ws=P.em_ws)
    e1.record()
    torch.cuda.synchronize()
    ms16 = e0.elapsed_time(e1) / reps
    idx = torch.linspace(0, nbk - 1, steps=min(sample, nbk), device="cuda").round().long().unique()
    ns = int(idx.numel())
    th0s = b.theta0[idx].contiguous()
    th64 = torch.zeros_like(th0s)
    J64 = torch.zeros((ns, iters + 1), dtype=torch.float64, device="cuda")
    pm.em_refine(S, l, th0s, P.bg, ns, None, iters, beta, pm.PM_FP64, th64, J64, None, None)
    torch.cuda.synchronize()
    ref = J64[:, -1].cpu().numpy()
    out = {"sample_buckets": ns, "reference": "FP64 path (parity-pinned to the oracle at 1e-12)"}
    for name, J, th in (("f16x2", b.J, b.theta), ("f16", J16, th16)):
        got = J[idx, -1].cpu().numpy()
        rel = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
        c_got = th[idx].cpu().numpy().argmax(axis=1)
        c_ref = th64.cpu().numpy().argmax(axis=1)
        out[name] = {"max_rel_dJ": float(rel.max()), "mean_rel_dJ": float(rel.mean()),
                     "consensus_identical": float(np.mean(np.all(c_got == c_ref, axis=1)))}
    out["f16x2"]["em_ms"] = round(ms_em, 4)
    out["f16"]["em_ms"] = round(ms16, 4)
    return out


def uneven_leg(torch, pm, m, count=512, seed=1):
    """The uneven batching shape (t~U[10,40], n~U[300,2000], l~U[11,21],
    d = floor(l/4)+1, k = clamp(l-d-4, 6, 9), s = 3) with m trials per
    instance: one batch per shape class, all classes captured in one HIP
    graph and replayed."""
    from synth import batch_config
    insts = batch_config(seed, count=count, m=m)
    classes = {}
    for inst, masks in insts:
        classes.setdefault(inst.meta["l"], []).append((inst, masks))
    bg = np.full(4, 0.25)
    pipes, nbk_tot, lmers = [], 0, 0
    for l in sorted(classes):
        group = classes[l]
        meta = group[0][0].meta
        B = pm.Batch(4, l, meta["k"], [i.seqs for i, _ in group], [mk for _, mk in group])
        nbk, nmem = pm.size_batch(B, meta["s"])
        nbk_tot += nbk
        lmers += sum(B.x[p] * B.m[p] for p in range(B.P))
        pipes.append((B, pm.BatchPipeline(B, meta["s"], meta["iters"], 1.0, pm.PM_F16X2, bg, nbk, nmem)))
    progress(f"uneven: {len(pipes)} shape classes, {nbk_tot} enriched buckets")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for _, P in pipes:
            P.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _, P in pipes:
            P.run()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    solved = 0
    for (B, P), l in zip(pipes, sorted(classes)):
        for r, (inst, _) in zip(P.results(), classes[l]):
            solved += r.get("consensus") == inst.motif
    return {"workload": f"{count} uneven DNA instances (t~U[10,40], n~U[300,2000], l~U[11,21]), m={m} trials each "
                        "(of 1000 in the full shape), 5 EM iterations, one graph over all shape classes",
            "ms": round(ms, 2), "instances_per_s": round(count / (ms / 1e3), 1),
            "projected_lmers_per_s": round(lmers / (ms / 1e3), 1), "enriched_buckets": nbk_tot,
            "shape_classes": len(pipes), "solved": int(solved)}


def c4_leg(torch, pm, seed=4, n_f16=131072, n_f64=16384):
    """The protein (20,6) workload's EM: its enriched buckets (hash and
    selection on the GPU), then the first n_f16 of them refined in the
    matrix-core precision form (20-letter one-hot, FP16 operands, FP32
    accumulation, FP64 log-sum-exp) and the first n_f64 in the FP64 vector
    path; time per model of each, the full EM extrapolated, and the precision
    form's error against FP64 on the common models (every iteration's J)."""
    from synth import make_config
    inst, masks = make_config("c4", seed=seed)
    cfg = inst.meta
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    # the generator's background in the library's code order
    bg = np.array([inst.bg[c] for c in pm.PROTEIN_CODE_ORDER], dtype=np.float64)
    bg /= bg.sum()
    S = pm.Seqs(20, inst.seqs)
    P0 = pm.Pipeline(S, l, k, s, masks, iters, 1.0, pm.PM_FP32, bg, 0, 0)
    P0.hash()
    P0.select()
    torch.cuda.synchronize()
    nbk, nmem = [int(v) for v in P0.b.n_out.cpu()]
    del P0
    P = pm.Pipeline(S, l, k, s, masks, iters, 1.0, pm.PM_FP32, bg, nbk, nmem)
    P.hash()
    P.select()
    b = P.b
    pm.bucket_profile(S, l, b.buckets, b.members, b.cap_m, b.cap_b, b.n_out, b.profile)
    pm.theta_init(20, l, b.profile, b.cap_b, b.n_out, P.bg, 1.0, b.theta0)
    progress(f"c4: {nbk} enriched buckets")
    out = {"workload": f"(20,6) protein: t=30, n=1000, k={k}, s={s}, m={len(masks)}, {iters} EM iterations",
           "enriched_buckets": nbk}
    Js = {}
    for prec, name, nb in ((pm.PM_F16, "f16_mfma", min(n_f16, nbk)), (pm.PM_FP64, "fp64_vector", min(n_f64, nbk))):
        th = torch.zeros((nb, 20, l), dtype=torch.float64, device="cuda")
        J = torch.zeros((nb, iters + 1), dtype=torch.float64, device="cuda")
        pm.em_refine(S, l, b.theta0, P.bg, nb, None, iters, 1.0, prec, th, J)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        pm.em_refine(S, l, b.theta0, P.bg, nb, None, iters, 1.0, prec, th, J)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out[name] = {"models": nb, "ms": round(ms, 3), "us_per_model": round(ms * 1e3 / nb, 4),
                     "full_em_s": round(ms / nb * nbk / 1e3, 3)}
        Js[name] = J[:min(n_f16, n_f64, nbk)].cpu().numpy()
        progress(f"c4: {name} {ms / nb * 1e3:.3f} us/model")
    d = np.abs(Js["f16_mfma"] - Js["fp64_vector"]) / np.abs(Js["fp64_vector"])
    out["f16_vs_fp64"] = {"models": int(d.shape[0]), "max_rel_dJ": float(d.max()), "mean_rel_dJ": float(d.mean())}
    out["speedup"] = round(out["fp64_vector"]["us_per_model"] / out["f16_mfma"]["us_per_model"], 2)
    return out


def c5_leg(torch, pm, seed=1):
    """One (21,7) instance, the shape the triage network is meant for: the full
    path (every enriched bucket refined) against the triaged one (top 5% of
    the buckets by the network, fallback on a weak winner), same buckets."""
    import os
    from synth import make_config
    inst, masks = make_config("c5", seed=seed)
    cfg = inst.meta
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    bg = np.full(4, 0.25)
    progress("c5: generated")
    B = pm.Batch(4, l, k, [inst.seqs], [masks])
    nbk, nmem = pm.size_batch(B, s)
    progress(f"c5: {nbk} enriched buckets")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {"workload": "(21,7) DNA: t=50, n=2000, k=9, s=3, m=10000, 5 EM iterations, one instance",
           "enriched_buckets": nbk, "planted": inst.motif}
    full = pm.BatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nbk, nmem)
    full.run()
    torch.cuda.synchronize()
    e0.record()
    full.run()
    e1.record()
    torch.cuda.synchronize()
    r = full.results()[0]
    out["full"] = {"ms": round(e0.elapsed_time(e1), 2), "consensus": r.get("consensus"),
                   "solved": r.get("consensus") == inst.motif}
    progress(f"c5: full pass {out['full']['ms']} ms")
    del full
    torch.cuda.empty_cache()
    path = pm.default_triage_path()
    if os.path.exists(path):
        TP = pm.TriagedBatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nbk, nmem, pm.Triage.load(path), 0.05)
        TP.run()
        torch.cuda.synchronize()
        e0.record()
        TP.run()
        e1.record()
        torch.cuda.synchronize()
        r = TP.results()[0]
        out["triaged"] = {"ms": round(e0.elapsed_time(e1), 2), "consensus": r.get("consensus"),
                          "solved": r.get("consensus") == inst.motif, "refined_buckets": int(TP.refined),
                          "fell_back": bool(r["fell_back"]), "z": r["z"]}
        out["speedup"] = round(out["full"]["ms"] / out["triaged"]["ms"], 3)
        progress(f"c5: triaged pass {out['triaged']['ms']} ms")
    return out


def hash_roofline(torch, pm, name, seed=1, reps=3):
    """projection_hash (keys and dense counts of every trial) on one
    configuration's full trial set, timed on its launch stream: algorithmic
    bytes per launch = 4 B per projected l-mer key + 4 B per count bin."""
    from synth import make_config
    inst, masks = make_config(name, seed=seed)
    cfg = inst.meta
    A = 20 if cfg.get("alphabet") == "protein" else 4
    l, k, m = cfg["l"], cfg["k"], len(masks)
    S = pm.Seqs(A, inst.seqs)
    x = S.nwin(l)
    dm = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).cuda()
    keys = torch.empty((m, x), dtype=torch.int32, device="cuda")
    counts = torch.empty((m, A ** k), dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.projection_hash(S, l, k, dm, m, keys, counts, st)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pm.projection_hash(S, l, k, dm, m, keys, counts, st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = 4.0 * m * x + 4.0 * m * A ** k
    gbs = nbytes / (ms / 1e3) / 1e9
    del keys, counts
    torch.cuda.empty_cache()
    kern = f"k_hash<{A},{k}>"  # counter width chosen by the library per launch
    progress(f"{name} hash: {ms:.3f} ms, {gbs:.0f} GB/s")
    return {"kernel": kern, "bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic("hash.hip", kern), "bytes_per_launch": nbytes,
            "ms": round(ms, 4),
            "workload": f"{'protein' if A == 20 else 'DNA'} ({l},{cfg['d']}): t={len(inst.seqs)}, "
                        f"n={cfg['n']}, k={k}, m={m} trials, keys and counts of every trial",
            "lmers_per_s": round(m * x / (ms / 1e3), 1)}


def c3_full_leg(torch, pm, m=1000, chunk=250, count=512, seed=1):
    """The 512-instance uneven workload with all m = 1000 trials of every
    instance: per shape class (motif length), the trials in chunks of
    `chunk` per instance through key and count buffers reused from chunk to
    chunk; every chunk hashed (keys + dense counts), its enriched buckets
    selected from them, the same trials through the fused selection (keys
    and counts kept on chip), and through projection_hash_select (keys and
    counts written, the selection's bitmap formed by the hash kernel).  Times on the launch stream; hash bytes
    algorithmic (4 B per key, 4 B per count bin)."""
    from synth import batch_config
    insts = batch_config(seed, count=count, m=m)
    classes = {}
    for inst, masks in insts:
        classes.setdefault(inst.meta["l"], []).append((inst, masks))
    progress(f"c3: {count} instances, {len(classes)} shape classes generated")
    ev = lambda: torch.cuda.Event(enable_timing=True)
    # one set of buffers for the largest chunk of any class
    plans, keys_max, counts_max, items_max = [], 0, 0, 0
    for l in sorted(classes):
        group = classes[l]
        meta = group[0][0].meta
        xs = [i.meta["t"] * (i.meta["n"] - l + 1) for i, _ in group]
        nb = 4 ** meta["k"]
        items = len(group) * chunk
        keys_max = max(keys_max, sum(xs) * chunk)
        counts_max = max(counts_max, items * nb)
        items_max = max(items_max, items)
        plans.append((l, meta, group))
    keys = torch.empty(keys_max, dtype=torch.int32, device="cuda")
    counts = torch.empty(counts_max, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    bk = torch.empty((1, 4), dtype=torch.int32, device="cuda")
    mem = torch.empty(1, dtype=torch.int32, device="cuda")
    t_hash = t_sel = t_fused = t_one = 0.0
    nbytes = lmers = 0.0
    nbk_tot = nmem_tot = 0
    for l, meta, group in plans:
        k, s = meta["k"], meta["s"]
        for c0 in range(0, m, chunk):
            B = pm.Batch(4, l, k, [i.seqs for i, _ in group], [mk[c0:c0 + chunk] for _, mk in group])
            nb = 4 ** k
            # sizes of the chunk's lists (untimed), then its buffers
            sws0 = pm.pm_select_workspace(4, k, B.items, 0)
            ws = torch.empty(max(sws0, 16), dtype=torch.uint8, device="cuda")
            pm.projection_hash_batch(B, B.masks, keys, counts, status)
            pm.bucket_select_batch(B, keys, counts, s, None, 0, None, 0, n_out, ws, sws0, None)
            torch.cuda.synchronize()
            nbk, nmem = [int(v) for v in n_out.cpu()]
            if bk.shape[0] < nbk:
                bk = torch.empty((int(nbk * 1.1) + 1, 4), dtype=torch.int32, device="cuda")
            if mem.numel() < nmem:
                mem = torch.empty(int(nmem * 1.1) + 1, dtype=torch.int32, device="cuda")
            sws = pm.pm_select_workspace(4, k, B.items, nbk)
            ws = torch.empty(max(sws, 16), dtype=torch.uint8, device="cuda")
            hws = pm.pm_hash_select_batch_workspace(B)
            hw = torch.empty(max(hws, 16), dtype=torch.uint8, device="cuda")
            e = [ev() for _ in range(6)]
            e[0].record()
            pm.projection_hash_batch(B, B.masks, keys, counts, status)
            e[1].record()
            pm.bucket_select_batch(B, keys, counts, s, bk, nbk, mem, nmem, n_out, ws, sws, status)
            e[2].record()
            e[3].record()
            pm.bucket_hash_select_batch(B, B.masks, s, bk, nbk, mem, nmem, n_out, hw, hws, status)
            e[4].record()
            pm.projection_hash_select_batch(B, B.masks, keys, counts, s, bk, nbk, mem, nmem, n_out, ws, sws, status)
            e[5].record()
            torch.cuda.synchronize()
            t_hash += e[0].elapsed_time(e[1])
            t_sel += e[1].elapsed_time(e[2])
            t_fused += e[3].elapsed_time(e[4])
            t_one += e[4].elapsed_time(e[5])
            nbytes += 4.0 * B.keys_total + 4.0 * B.items * nb
            lmers += float(sum(B.x[p] * B.m[p] for p in range(B.P)))
            nbk_tot += nbk
            nmem_tot += nmem
        progress(f"c3: class l={l} done ({len(group)} instances)")
    if int(status.item()) != 0:
        raise SystemExit(f"c3 device status {int(status.item())}")
    gbs = nbytes / (t_hash / 1e3) / 1e9
    del keys, counts, bk, mem
    torch.cuda.empty_cache()
    return {"workload": f"{count} uneven DNA instances (t~U[10,40], n~U[300,2000], l~U[11,21], d=floor(l/4)+1, "
                        f"k=clamp(l-d-4,6,9), s=3), all m={m} trials of every instance, {len(plans)} shape classes, "
                        f"trials in chunks of {chunk} per instance through reused key/count buffers",
            "projected_lmers": lmers, "enriched_buckets": nbk_tot, "members": nmem_tot,
            "hash_ms": round(t_hash, 2), "select_ms": round(t_sel, 2), "fused_select_ms": round(t_fused, 2),
            "hash_then_select_one_call_ms": round(t_one, 2),
            "roofline_hash": {"kernel": "k_hash<4,k,*> (11 classes)", "bound": "hbm", "achieved": round(gbs, 2),
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                              "traffic": None, "bytes": nbytes},
            "lmers_per_s_hash": round(lmers / (t_hash / 1e3), 1),
            "lmers_per_s_hash_and_select": round(lmers / ((t_hash + t_sel) / 1e3), 1),
            "lmers_per_s_fused_select": round(lmers / (t_fused / 1e3), 1),
            "lmers_per_s_hash_then_select_one_call": round(lmers / (t_one / 1e3), 1)}


def perf_coefficient(starts, sites, l):
    """|planted residues & predicted residues| / |union|, over the sequences
    of one instance (windows of length l)."""
    inter = union = 0
    for a, b in zip(starts, sites):
        ov = max(0, min(a, b) + l - max(a, b))
        inter += ov
        union += 2 * l - ov
    return inter / union


def instances_leg(torch, pm, count):
    """(15,4) instances solved per second: every instance through the plain
    per-instance pipeline (FP64 EM, all enriched buckets), and the same
    instances as one graph-captured batch (EM on the split-FP16 matrix cores).
    Solved = consensus equals the planted motif."""
    from synth import make_config
    insts = [make_config("c1", seed=i) for i in range(count)]
    cfg = insts[0][0].meta
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    bg = np.full(4, 0.25)
    beta = 1.0

    def score(cons, sites, inst):
        return (cons == inst.motif), perf_coefficient(inst.starts, sites, l)

    progress(f"instances leg: {count} instances generated")

    def plain_leg(precision, label):
        # one pipeline per instance, run one after another
        pipes = []
        for inst, masks in insts:
            S = pm.Seqs(4, inst.seqs)
            P0 = pm.Pipeline(S, l, k, s, masks, iters, beta, precision, bg, cap_b=0, cap_m=0)
            P0.hash()
            P0.select()
            nbk, nmem = [int(v) for v in P0.b.n_out.cpu()]
            del P0
            pipes.append(pm.Pipeline(S, l, k, s, masks, iters, beta, precision, bg, cap_b=nbk, cap_m=nmem))
        for P in pipes[:2]:
            P.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for P in pipes:
            P.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        solved = pcs = 0.0
        for P, (inst, _) in zip(pipes, insts):
            r = P.result()
            ok, pc = score(r.get("consensus"), r.get("sites", [0] * len(inst.starts)), inst)
            solved += ok
            pcs += pc
        del pipes
        torch.cuda.empty_cache()
        progress(f"plain leg ({label}): {ms:.1f} ms")
        return {"instances_per_s": round(count / (ms / 1e3), 2), "ms": round(ms, 3),
                "solved": int(solved), "solved_per_s": round(solved / (ms / 1e3), 2),
                "mean_pc": round(pcs / count, 4), "em": f"{label}, all enriched buckets, one instance at a time"}

    plain = plain_leg(pm.PM_FP64, "fp64 vector")
    # the same per-instance pipeline with the batched leg's EM form, so that the
    # gain of batching is measured apart from the gain of the matrix cores
    plain_mc = plain_leg(pm.PM_F16X2, "split-f16 matrix cores")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # ---- batched: all instances in one pass of launches, captured in a graph
    B = pm.Batch(4, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])
    nbk, nmem = pm.size_batch(B, s)
    BP = pm.BatchPipeline(B, s, iters, beta, pm.PM_F16X2, bg, cap_b=nbk, cap_m=nmem)
    tile_shape = pick_shape(torch, pm, l, BP.run)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        BP.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        BP.run()
    g.replay()
    torch.cuda.synchronize()
    reps = 3
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1) / reps
    solved = pcs = 0.0
    for r, (inst, _) in zip(BP.results(), insts):
        ok, pc = score(r.get("consensus"), r.get("sites", [0] * len(inst.starts)), inst)
        solved += ok
        pcs += pc
    batched = {"instances_per_s": round(count / (batch_ms / 1e3), 2), "ms": round(batch_ms, 3),
               "solved": int(solved), "solved_per_s": round(solved / (batch_ms / 1e3), 2),
               "mean_pc": round(pcs / count, 4), "enriched_buckets": nbk, "em_tile_shape": tile_shape,
               "em": "split-f16 matrix cores, all enriched buckets, one HIP graph"}
    out = {"workload": f"(15,4) DNA: t=20, n=600, k=7, s=4, m=200, 5 EM iterations; {count} instances, seeds 0..{count - 1}",
           "plain": plain, "plain_f16x2": plain_mc, "batched": batched,
           "speedup_batched": round(batched["instances_per_s"] / plain["instances_per_s"], 3),
           "speedup_batched_vs_plain_f16x2": round(batched["instances_per_s"] / plain_mc["instances_per_s"], 3)}
    del BP, g
    torch.cuda.empty_cache()

    progress(f"batched leg: {batch_ms:.1f} ms")
    # ---- batched + triaged: the trained network picks 5% of each instance's buckets
    import os
    path = pm.default_triage_path()
    if not os.path.exists(path):
        out["triaged"] = None
        return out
    tri = pm.Triage.load(path)
    TP = pm.TriagedBatchPipeline(B, s, iters, beta, pm.PM_F16X2, bg, nbk, nmem, tri, frac=0.05)
    tri_shape = pick_shape(torch, pm, l, TP.run)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        TP.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        TP.run()
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    tri_ms = e0.elapsed_time(e1) / reps
    res = TP.results()
    solved = pcs = 0.0
    for r, (inst, _) in zip(res, insts):
        ok, pc = score(r.get("consensus"), r.get("sites", [0] * len(inst.starts)), inst)
        solved += ok
        pcs += pc
    out["triaged"] = {"instances_per_s": round(count / (tri_ms / 1e3), 2), "ms": round(tri_ms, 3),
                      "solved": int(solved), "solved_per_s": round(solved / (tri_ms / 1e3), 2),
                      "mean_pc": round(pcs / count, 4), "refined_buckets": int(TP.refined),
                      "fallbacks": int(sum(r["fell_back"] for r in res)), "frac": 0.05,
                      "em_tile_shape": tri_shape,
                      "em": "split-f16 matrix cores on the triaged buckets, BF16 network, one HIP graph"}
    out["speedup_triaged"] = round(out["triaged"]["instances_per_s"] / plain["instances_per_s"], 3)
    out["speedup_triaged_vs_plain_f16x2"] = round(out["triaged"]["instances_per_s"] / plain_mc["instances_per_s"], 3)
    out["pc_delta_triaged_vs_plain"] = round(out["triaged"]["mean_pc"] - plain["mean_pc"], 4)
    return out


def pick_shape(torch, pm, l, run):
    """Tile shape of the batched matrix-core EM, chosen on the whole batch: each
    candidate pinned in turn, the pipeline run eagerly (once to warm up, once
    timed), the fastest kept for the graph captured next."""
    times = {}
    for shape in (11, 12, 14, 21, 22, 24):
        try:
            pm.em_set_tuning(l, pm.PM_F16X2, shape)
        except pm.PmError:
            continue
        run()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times[shape] = e0.elapsed_time(e1)
    best = min(times, key=times.get)
    pm.em_set_tuning(l, pm.PM_F16X2, best)
    progress("batch tile shapes (ms): " + ", ".join(f"{k}: {v:.2f}" for k, v in times.items()))
    return best


def cpu_baseline(inst, masks, cfg, bg, beta, nbk, budget):
    """The oracle, untuned, on the same pass: hashing and selection of every
    trial in full (in chunks of trials, all host threads), EM of a sample of
    the enriched buckets timed and extrapolated linearly to all of them; the
    same again on one thread with the hashing and selection of a prefix of
    the trials extrapolated too."""
    import oracle
    l, k, s, iters, m = cfg["l"], cfg["k"], cfg["s"], cfg["iters"], cfg["m"]
    ref = oracle.Seqs(4, inst.seqs)
    x = ref.nwin(l)
    cores = oracle.set_threads(0)

    def hash_select(trials):
        th0 = None
        for j0 in range(0, len(trials), 500):
            K, N = oracle.hash_trials(ref, l, k, trials[j0:j0 + 500])
            bk, mem, _, _ = oracle.select(ref, l, k, K, N, s)
            if th0 is None:
                th0 = oracle.theta0(oracle.profile(ref, l, bk, mem), bg, beta)
        return th0

    def em_per_bucket(th0, seconds):
        nb = max(1, min(len(th0), 8))
        t3 = time.perf_counter()
        oracle.em(ref, l, th0[:nb], bg, iters, beta)
        per = (time.perf_counter() - t3) / nb
        nb2 = int(min(len(th0), max(nb, seconds / max(per, 1e-9))))
        if nb2 > nb:
            t3 = time.perf_counter()
            oracle.em(ref, l, th0[:nb2], bg, iters, beta)
            per = (time.perf_counter() - t3) / nb2
        return per, max(nb, nb2)

    t0 = time.perf_counter()
    th0 = hash_select(masks)
    t_hs = time.perf_counter() - t0
    per, nb_em = em_per_bucket(th0, max(2.0, 0.5 * budget - t_hs))
    est = t_hs + per * nbk
    # one thread: a prefix of the trials and a smaller EM sample
    oracle.set_threads(1)
    try:
        mt1 = max(8, m // 50)
        t0 = time.perf_counter()
        hash_select(masks[:mt1])
        t_hs1 = (time.perf_counter() - t0) * m / mt1
        per1, nb_em1 = em_per_bucket(th0, max(1.0, 0.25 * budget))
    finally:
        oracle.set_threads(cores)
    est1 = t_hs1 + per1 * nbk
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), cpu_model)
    except OSError:
        pass
    return {"value": round(m * x / est, 1), "unit": "l-mers/s", "cores": cores, "kind": "oracle",
            "sample": f"hash+select of all {m} trials timed in full; EM of {nb_em}/{nbk} buckets, "
                      "extrapolated linearly",
            "est_s_per_step": round(est, 2), "hash_select_s": round(t_hs, 2),
            "em_s_per_bucket": per,
            "one_thread": {"value": round(m * x / est1, 1), "est_s_per_step": round(est1, 2),
                           "sample": f"hash+select of {mt1}/{m} trials and EM of {nb_em1} buckets, "
                                     "extrapolated linearly"},
            "cpu_model": cpu_model, "nproc": os.cpu_count()}


if __name__ == "__main__":
    main()
