"""What the trained triage network gains over the method without it.

On held-out (15,4) instances (seeds the training never saw), the triaged
pipeline refines about 5% of the enriched buckets and must recover the planted
motif as often as full refinement (the method without the network) up to one
instance, while the same machinery driven by an untrained network (a ranking
with no information) recovers fewer.  Training outcome: parity unpinned
(stochastic); this test states the gain.
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


def test_trained_triage_keeps_recovery_at_a_fraction_of_the_work(trained):
    insts = [make_config("c1", seed=20000 + i) for i in range(32)]
    cfg = insts[0][0].meta
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    bg = np.full(4, 0.25)
    say("triage gain on 32 held-out (15,4) instances")
    B = pm.Batch(4, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])
    nb_, nm_ = pm.size_batch(B, s)
    full = pm.BatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_)
    full.run()
    solved_full = _solved(full.results(), insts)

    TP = pm.TriagedBatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_, trained, frac=0.05)
    TP.run()
    res = TP.results()
    solved_tri = _solved(res, insts)
    fell = sum(r["fell_back"] for r in res)

    rng = np.random.default_rng(0)
    sizes = (pm.PM_TRIAGE_INPUTS, 256, 256, 1)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts += [rng.normal(0, np.sqrt(2.0 / a), size=a * b), np.zeros(b)]
    untrained = pm.Triage(np.concatenate(parts).astype(np.float32), trained.mu.cpu().numpy(),
                          trained.sd.cpu().numpy(), -np.inf)
    RP = pm.TriagedBatchPipeline(B, s, iters, 1.0, pm.PM_F16X2, bg, nb_, nm_, untrained, frac=0.05)
    RP.run()
    solved_rand = _solved(RP.results(), insts)
    print(f"[gain] buckets {nb_}: full EM solved {solved_full}/32; trained triage solved {solved_tri}/32 "
          f"refining {TP.refined} buckets ({TP.refined / nb_:.3f}), {fell} fallbacks; "
          f"untrained ranking solved {solved_rand}/32", flush=True)
    assert solved_tri >= solved_full - 1
    assert TP.refined <= 0.5 * nb_
    assert solved_tri > solved_rand
