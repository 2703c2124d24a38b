"""projection_run, the host-in/host-out entry point over many problems
(Alg. 2 / Alg. 3 INPUT and OUTPUT), through the C ABI: batched and unbatched
runs agree, a mixed-shape batch agrees with the oracle problem by problem, and
the triaged batched run gives the same bits as the binding's triaged batch
pipeline (the same kernels called in the same order)."""
import sys
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm
from synth import planted_instance, projection_masks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield
    torch.cuda.synchronize()


def _problems(name, shapes, bg=np.full(4, 0.25)):
    """One planted DNA problem per (l, k, d, s) in `shapes`: t in [4, 9], ragged
    n, 3-12 trials with explicit masks."""
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    out, insts = [], []
    for l, k, d, s in shapes:
        t = int(rng.integers(4, 10))
        lens = [int(v) for v in rng.integers(l + 20, 320, size=t)]
        inst = planted_instance(rng, t, lens, l, d)
        masks = projection_masks(rng, l, k, int(rng.integers(3, 13)))
        out.append(pm.Problem(inst.seqs, 4, l, d=d, k=k, s=s, masks=masks, bg=bg))
        insts.append(inst)
    return out, insts


def test_projection_run_fig1_toy():
    """Example 1: PROJECTION + EM on Fig. 1 returns ATGCAACT at Fig. 2's sites,
    unbatched and batched."""
    from tests.conftest import read_golden
    seqs = [r[0] for r in read_golden("fig1_sequences.txt")]
    say("projection_run toy")
    pr = pm.Problem(seqs, 4, 8, k=5, s=4, masks=np.array([0b1100111]), bg=np.full(4, 0.25))
    for batched in (False, True):
        r = pm.projection_run(pr, em_iters=5, beta=1.0, batched=batched)[0]
        assert r["consensus"] == "ATGCAACT"
        assert list(r["sites"]) == [7, 18, 2, 4, 30, 26, 14]
        assert r["n_enriched"] == 2 and r["n_refined"] == 2 and not r["fallback_used"]
        assert r["best_trial"] == 0 and r["best_key"] == 177  # ATGAC (Sec. 6 integer)


@pytest.mark.parametrize("prec", [pm.PM_FP64, pm.PM_F16X2], ids=["fp64", "f16x2"])
def test_projection_run_batched_equals_unbatched_and_oracle(prec):
    """Problems of three shape classes in one call: batched (one batch per
    class) and unbatched give the same answers bit for bit; the FP64 answers
    match the oracle's whole path."""
    shapes = [(11, 5, 2, 2), (13, 6, 3, 3), (11, 5, 2, 2), (15, 7, 4, 3), (13, 6, 3, 3)]
    probs, insts = _problems("run mixed", shapes)
    say("projection_run mixed", prec)
    a = pm.projection_run(probs, em_iters=4, beta=1.0, precision=prec, batched=False)
    b = pm.projection_run(probs, em_iters=4, beta=1.0, precision=prec, batched=True)
    for p, (ra, rb) in enumerate(zip(a, b)):
        for key in ("consensus", "J", "llr", "best_trial", "best_key", "n_enriched", "n_refined", "k", "s", "m"):
            assert ra[key] == rb[key], (p, key, ra[key], rb[key])
        assert np.array_equal(ra["sites"], rb["sites"]) and np.array_equal(ra["theta"], rb["theta"])
    if prec != pm.PM_FP64:
        return
    for p, (pr, r) in enumerate(zip(probs, b)):
        ref = oracle.run(pr.seqs, 4, pr.l, pr.k, pr.s, pr.masks, 4, beta=1.0, bg=pr.bg)
        assert r["n_enriched"] == len(ref["buckets"]), p
        if ref["best"] < 0:
            assert r["consensus"] == "" and r["best_trial"] == -1
            continue
        assert r["consensus"] == ref["consensus"], p
        np.testing.assert_allclose(r["J"], ref["J"][ref["best"], -1], rtol=1e-12)
        bk = ref["buckets"][ref["best"]]
        assert (r["best_trial"], r["best_key"]) == (int(bk[0]), int(bk[1]))
        assert np.array_equal(r["sites"], ref["sites"][ref["best"]])
        np.testing.assert_allclose(r["theta"], ref["theta"][ref["best"]], rtol=1e-12, atol=1e-14)


def test_projection_run_triaged_matches_triaged_pipeline():
    """n_problems > 1 with learned triage (the shipped weights): the same
    answers, bit for bit, as TriagedBatchPipeline over the same batch, with the
    number of refined buckets and the fallback flag of every problem."""
    shapes = [(15, 7, 4, 3)] * 6
    probs, insts = _problems("run triaged", shapes)
    say("projection_run triaged")
    iters, beta = 4, 1.0
    r = pm.projection_run(probs, em_iters=iters, beta=beta, precision=pm.PM_F16X2, batched=True, triage=True,
                          triage_frac=0.05)
    B = pm.Batch(4, 15, 7, [p.seqs for p in probs], [p.masks for p in probs])
    nb_, nm_ = pm.size_batch(B, 3)
    TP = pm.TriagedBatchPipeline(B, 3, iters, beta, pm.PM_F16X2, np.full(4, 0.25), nb_, nm_,
                                 pm.Triage.load(pm.default_triage_path()), 0.05)
    TP.run()
    torch.cuda.synchronize()
    tr = TP.results()
    bk = TP.b.buckets.cpu().numpy().view(np.uint32)[:nb_]
    L1, L2 = TP.lists
    n1, n2 = int(L1["n"].item()), int(L2["n"].item())
    item_inst = B.item_inst.cpu().numpy()
    refined = np.bincount(item_inst[np.concatenate([L1["buckets"].cpu().numpy().view(np.uint32)[:n1, 0],
                                                    L2["buckets"].cpu().numpy().view(np.uint32)[:n2, 0]])],
                          minlength=B.P)
    enriched = np.bincount(item_inst[bk[:, 0]], minlength=B.P)
    for p in range(B.P):
        assert r[p]["n_enriched"] == enriched[p], p
        assert r[p]["n_refined"] == refined[p], p
        assert r[p]["fallback_used"] == tr[p]["fell_back"], p
        if tr[p]["best"] < 0:
            assert r[p]["best_trial"] == -1
            continue
        assert r[p]["consensus"] == tr[p]["consensus"], p
        assert r[p]["J"] == tr[p]["J"], p
        assert np.array_equal(r[p]["sites"], tr[p]["sites"]), p
        w = bk[tr[p]["best"]]
        assert (r[p]["best_trial"], r[p]["best_key"]) == (int(w[0]) - B.first_item[p], int(w[1])), p


def test_projection_run_rejects_bad_options():
    probs, _ = _problems("run bad", [(11, 5, 2, 2)])
    say("projection_run bad options")
    with pytest.raises(pm.PmError):
        pm.projection_run(probs, triage=True, triage_weights="/nonexistent/weights.bin")
    with pytest.raises(pm.PmError):
        pm.projection_run(probs, precision=7)
    prot = pm.Problem(["ARNDCQEGHILKMFPSTWYV" * 3] * 3, 20, 10, k=2, s=2, masks=np.array([0b11]),
                      bg=np.full(20, 0.05))
    with pytest.raises(pm.PmError):
        pm.projection_run(prot, triage=True)  # triage is for DNA
    with pytest.raises(pm.PmError):
        pm.projection_run(prot, precision=pm.PM_F16, batched=True)


def test_projection_run_range_matches_oracle():
    """A motif-length range (Sec. 2) over one planted (11,2) problem at
    l = 10..12 (k and s from the Sec. 5 rules, 40 Park-Miller trials per
    length): every length's answer and the chosen length equal the oracle's,
    unbatched and batched."""
    rng = np.random.default_rng(71)
    inst = planted_instance(rng, 14, 300, 11, 2)
    pr = pm.Problem(inst.seqs, 4, 11, d=2, m=40, seed=7)
    ref, rchosen = oracle.run_range(inst.seqs, 4, 10, 12, 2, 7, 3, 1.0, m=40)
    assert rchosen > 0
    for batched in (False, True):
        say("projection_run_range batched" if batched else "projection_run_range")
        res, chosen = pm.projection_run_range(pr, 10, 12, em_iters=3, beta=1.0, precision=pm.PM_FP64,
                                              batched=batched)
        assert chosen == rchosen
        for r, q in zip(res, ref):
            assert (r["k"], r["s"], r["m"], r["n_enriched"]) == (q["k"], q["s"], q["m"], q["n_enriched"])
            assert r["consensus"] == q["consensus"]
            assert abs(r["llr"] - q["llr"]) <= 1e-12 * abs(q["llr"])
            assert np.array_equal(r["sites"], q["sites"])
