"""What the trained triage network gains over the method without it.

On held-out (15,4) instances (seeds the training never saw): the network's
ranking against an untrained one at the same 5% of refined buckets, and the
triaged pipeline with its fallback against full refinement (the method
without the network).  Training outcome: parity unpinned (stochastic); this
test states the gain.
"""
import os
import sys

import numpy as np
import pytest

import paper_1605_06904_amd as pm
from synth import make_config

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def trained():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    path = pm.default_triage_path()
    if not os.path.exists(path):
        pytest.skip("no trained triage weights (python -m paper_1605_06904_amd.triage_train)")
    return pm.Triage.load(path)


def _solved(results, insts):
    return sum(r.get("consensus") == inst.motif for r, (inst, _) in zip(results, insts))


def _run(B, s, iters, bg, nb_, nm_, tri, threshold):
    TP = pm.TriagedBatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_, tri, frac=0.05)
    if threshold is not None:
        TP.threshold = threshold
    TP.run()
    res = TP.results()
    return res, TP.refined


def test_trained_triage_gain_on_held_out_instances(trained):
    """On 64 held-out (15,4) instances the triaged pipeline with its fallback
    recovers the planted motif within one instance of full refinement (the
    method without the network) while refining fewer buckets.  The ranking
    alone (no fallback, 5% refined) is reported against an untrained network
    and not asserted: on this shape the profile of a bucket says little about
    where its refinement ends (parity unpinned; measured)."""
    n = 64
    insts = [make_config("c1", seed=20000 + i) for i in range(n)]
    cfg = insts[0][0].meta
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    bg = np.full(4, 0.25)
    say(f"triage gain on {n} held-out (15,4) instances")
    B = pm.Batch(4, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])
    nb_, nm_ = pm.size_batch(B, s)
    full = pm.BatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_)
    full.run()
    solved_full = _solved(full.results(), insts)

    rng = np.random.default_rng(0)
    sizes = (pm.PM_TRIAGE_INPUTS, 256, 256, 1)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts += [rng.normal(0, np.sqrt(2.0 / a), size=a * b), np.zeros(b)]
    untrained = pm.Triage(np.concatenate(parts).astype(np.float32), trained.mu.cpu().numpy(),
                          trained.sd.cpu().numpy(), -np.inf)
    res_u, ref_u = _run(B, s, iters, bg, nb_, nm_, untrained, -np.inf)
    res_t, ref_t = _run(B, s, iters, bg, nb_, nm_, trained, -np.inf)
    res_f, ref_f = _run(B, s, iters, bg, nb_, nm_, trained, None)
    su, st, sf = _solved(res_u, insts), _solved(res_t, insts), _solved(res_f, insts)
    fell = sum(r["fell_back"] for r in res_f)
    print(f"[gain] {n} instances, {nb_} buckets: full EM solved {solved_full}; 5% by untrained network "
          f"{su} ({ref_u} refined); 5% by trained network {st} ({ref_t} refined); trained + fallback {sf} "
          f"({ref_f} refined = {ref_f / nb_:.3f}, {fell} fallbacks)", flush=True)
    assert sf >= solved_full - 1
    assert ref_f < nb_
