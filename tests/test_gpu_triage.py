"""Triage kernels against the triage oracle.

Features and FP32 training gradients within FP32 rounding of the FP64 oracle;
the BF16 serving forward against the oracle's emulation of the same roundings;
selection bit-exact against the oracle's top fraction of the GPU's own scores
(the same numbers decide on both sides); the triaged pipeline against the full
one under the settings where they must agree.
"""
import math
import sys
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm
from oracle import triage as T
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


def dev(a, dt=None):
    return torch.from_numpy(np.ascontiguousarray(a if dt is None else a.astype(dt))).cuda()


def _profiles(rng, B, l):
    sizes = rng.integers(3, 40, size=B)
    prof = np.zeros((B, 4, l), dtype=np.uint32)
    for b in range(B):
        for p in range(l):
            prof[b, :, p] = rng.multinomial(sizes[b], rng.dirichlet(np.ones(4) * 0.5))
    return prof


def test_features_match_oracle():
    rng = np.random.default_rng(1)
    for l, bg in [(15, np.full(4, 0.25)), (21, np.array([0.3, 0.2, 0.2, 0.3])), (5, np.full(4, 0.25))]:
        prof = _profiles(rng, 300, l)
        say("features", l)
        feat = torch.zeros((300, 87), dtype=torch.float32, device="cuda")
        pm.triage_features(l, dev(prof.view(np.int32)), 300, None, dev(bg), None, None, feat)
        mu = rng.normal(size=87).astype(np.float32)
        sd = (0.5 + rng.random(87)).astype(np.float32)
        feat2 = torch.zeros_like(feat)
        pm.triage_features(l, dev(prof.view(np.int32)), 300, None, dev(bg), dev(mu), dev(sd), feat2)
        torch.cuda.synchronize()
        ref = T.features(prof, bg)
        np.testing.assert_allclose(feat.cpu().numpy(), ref, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(feat2.cpu().numpy(), (ref - mu) / sd, rtol=1e-5, atol=1e-5)


def _params(seed):
    rng = np.random.default_rng(seed)
    P = T.init_params(rng)
    P = [p + 0.02 * rng.normal(size=p.shape) for p in P]
    return P, T.flat(P).astype(np.float32)


def test_serving_forward_matches_bf16_emulation():
    P, v = _params(2)
    P32 = T.unflat(v.astype(np.float64))  # the FP32 values the GPU holds
    rng = np.random.default_rng(3)
    for B in (1, 31, 129, 1000):
        X = rng.normal(size=(B, 87)).astype(np.float32)
        say("forward", B)
        dp = dev(v)
        packed = torch.zeros(pm.pm_triage_packed_bytes(), dtype=torch.uint8, device="cuda")
        pm.triage_pack(dp, packed)
        score = torch.full((B,), np.nan, dtype=torch.float32, device="cuda")
        pm.triage_forward(packed, dev(X), B, None, score)
        torch.cuda.synchronize()
        got = score.cpu().numpy()
        ref = T.forward_bf16(P32, X.astype(np.float64))
        # FP32 sums of exact BF16 products: bound by the magnitude of the terms
        W1, b1, W2, b2, W3, b3 = P32
        H1 = np.maximum(T.bf16_round(X) @ T.bf16_round(W1) + b1, 0)
        mag = (np.abs(T.bf16_round(H1)) @ np.abs(T.bf16_round(W2)) + np.abs(b2)) @ np.abs(W3)[:, 0] + 1.0
        # (a first-layer unit whose FP32 sum sits on a BF16 rounding boundary
        # may round the other way: one unit in the 8th bit of one H1 entry)
        assert np.all(np.abs(got - ref) <= 1e-4 * mag), (np.abs(got - ref) / mag).max()
        # and the full-precision network is close (BF16 is a lossy form)
        full = T.forward(P32, X.astype(np.float64))[0]
        assert np.corrcoef(got, full)[0, 1] > 0.99 if B > 30 else True


def _train_buffers(N):
    ws_b = pm.pm_triage_workspace(N)
    ws = torch.zeros((ws_b + 3) // 4, dtype=torch.float32, device="cuda")
    return ws, ws_b


def test_training_gradients_match_oracle():
    P, v = _params(4)
    P32 = T.unflat(v.astype(np.float64))
    rng = np.random.default_rng(5)
    for N in (1, 7, 64, 300):
        X = rng.normal(size=(N, 87)).astype(np.float32)
        t = rng.normal(size=N).astype(np.float32)
        say("gradients", N)
        ws, ws_b = _train_buffers(N)
        g = torch.zeros(pm.PM_TRIAGE_PARAMS, dtype=torch.float32, device="cuda")
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        dp = dev(v)
        pm.triage_train_step(dp, None, None, 0, dev(X), dev(t), N, 0.0, loss, g, ws, ws_b)
        torch.cuda.synchronize()
        y, cache = T.forward(P32, X.astype(np.float64))
        ref = T.flat(T.backward(P32, cache, y, t.astype(np.float64)))
        got = g.cpu().numpy()
        # FP32 sums over N examples and 256 units: a relative bound on the
        # largest gradient entry of each tensor
        o = 0
        for p in P32:
            seg = slice(o, o + p.size)
            scale = np.abs(ref[seg]).max() + 1e-12
            assert np.abs(got[seg] - ref[seg]).max() <= 1e-4 * scale, (o, np.abs(got[seg] - ref[seg]).max() / scale)
            o += p.size
        assert math.isclose(float(loss.item()), T.loss(y, t), rel_tol=1e-4)
        assert torch.equal(dp, dev(v))  # lr = 0: no update


def test_adam_update_matches_oracle():
    P, v = _params(6)
    P32 = T.unflat(v.astype(np.float64))
    rng = np.random.default_rng(7)
    N = 128
    X = rng.normal(size=(N, 87)).astype(np.float32)
    t = rng.normal(size=N).astype(np.float32)
    say("adam")
    ws, ws_b = _train_buffers(N)
    dp = dev(v)
    m = torch.zeros_like(dp)
    vv = torch.zeros_like(dp)
    ref_p = [p.copy() for p in P32]
    ref_m = [np.zeros_like(p) for p in P32]
    ref_v = [np.zeros_like(p) for p in P32]
    for step in (1, 2, 3):
        pm.triage_train_step(dp, m, vv, step, dev(X), dev(t), N, 1e-3, None, None, ws, ws_b)
        y, cache = T.forward(ref_p, X.astype(np.float64))
        T.adam_step(ref_p, T.backward(ref_p, cache, y, t.astype(np.float64)), ref_m, ref_v, step, lr=1e-3)
    torch.cuda.synchronize()
    got = dp.cpu().numpy().astype(np.float64)
    ref = T.flat(ref_p)
    # each Adam step moves a parameter by at most about lr; compare the moves
    moved_ref, moved_got = ref - T.flat(P32), got - T.flat(P32)
    assert np.abs(moved_ref).max() <= 3.5e-3
    assert np.abs(moved_got - moved_ref).max() <= 2e-4, np.abs(moved_got - moved_ref).max()
    assert np.mean(np.sign(moved_got) == np.sign(moved_ref)) > 0.99


def test_training_reduces_loss():
    rng = np.random.default_rng(8)
    N = 512
    X = rng.normal(size=(N, 87)).astype(np.float32)
    w = rng.normal(size=87)
    t = (np.tanh(X @ w / 9.0) * 2).astype(np.float32)
    _, v = _params(9)
    say("training loss")
    ws, ws_b = _train_buffers(N)
    dp = dev(v)
    m, vv = torch.zeros_like(dp), torch.zeros_like(dp)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    dX, dt = dev(X), dev(t)
    first = None
    for step in range(1, 301):
        pm.triage_train_step(dp, m, vv, step, dX, dt, N, 1e-3, loss, None, ws, ws_b)
        if step == 1:
            torch.cuda.synchronize()
            first = float(loss.item())
    torch.cuda.synchronize()
    assert float(loss.item()) < 0.1 * first


# ------------------------------------------------------------------ selection
def _batch(name, P, l, k, d):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    insts = []
    for p in range(P):
        t = int(rng.integers(3, 8))
        inst = planted_instance(rng, t, [int(v) for v in rng.integers(l + 2, 200, size=t)], l, d)
        insts.append((inst, projection_masks(rng, l, k, int(rng.integers(2, 7)))))
    return insts, pm.Batch(4, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])


@pytest.mark.parametrize("frac", [0.05, 0.3, 1.0])
def test_select_matches_oracle_top_fraction(frac):
    insts, B = _batch("triage select", 5, 11, 5, 3)
    s, iters = 2, 2
    bg = np.full(4, 0.25)
    say("triage select", frac)
    nb_, nm_ = pm.size_batch(B, s)
    PP = pm.BatchPipeline(B, s, iters, 1.0, pm.PM_FP64, bg, nb_, nm_)
    PP.hash()
    PP.select()
    PP.profile()
    b = PP.b
    # scores with many ties
    rng = np.random.default_rng(10)
    sc = np.round(rng.normal(size=nb_), 1).astype(np.float32)
    score = dev(sc)
    taken = torch.zeros(nb_, dtype=torch.uint8, device="cuda")
    sel_b = torch.full((nb_, 4), -1, dtype=torch.int32, device="cuda")
    sel_t = torch.zeros((nb_, 4, 11), dtype=torch.float64, device="cuda")
    sel_i = torch.full((nb_,), -1, dtype=torch.int64, device="cuda")
    n_sel = torch.zeros(1, dtype=torch.int64, device="cuda")
    wsb = pm.pm_triage_select_workspace(B.P, nb_)
    ws = torch.zeros((wsb + 7) // 8, dtype=torch.int64, device="cuda")
    pm.triage_select(B, b.buckets, score, nb_, b.n_out, frac, b.theta0, 4, 11, taken, sel_b, sel_t, sel_i, n_sel,
                     ws, wsb)
    torch.cuda.synchronize()
    bk = b.buckets.cpu().numpy().view(np.uint32)[:nb_]
    item_inst = B.item_inst.cpu().numpy()
    group = item_inst[bk[:, 0]]
    keep = T.top_fraction(sc.astype(np.float64), group, frac)
    n = int(n_sel.item())
    want = np.nonzero(keep)[0]
    assert n == len(want)
    assert np.array_equal(sel_i.cpu().numpy()[:n], want)
    assert np.array_equal(sel_b.cpu().numpy()[:n], b.buckets.cpu().numpy()[want])
    assert torch.equal(sel_t[:n], b.theta0[torch.from_numpy(want).cuda()])
    assert np.array_equal(taken.cpu().numpy().astype(bool), keep)

    # fallback: the z-score of each instance's winner among its list-1
    # objectives against a threshold; made-up objectives and winners
    sel_items = sel_b.cpu().numpy().view(np.uint32)[:n, 0]
    g1 = item_inst[sel_items]
    Jv = np.round(rng.normal(size=max(n, 1)) * 3, 2)
    winners = {}
    for p in range(B.P):
        idx = np.nonzero(g1 == p)[0]
        if len(idx) and p % 3 != 2:
            winners[p] = int(idx[np.argmax(Jv[idx])]) if p % 2 == 0 else int(idx[0])
    best = torch.tensor([winners.get(p, -1) for p in range(B.P)], dtype=torch.int64, device="cuda")
    J = torch.zeros((max(n, 1), iters + 1), dtype=torch.float64, device="cuda")
    J[:, -1] = torch.from_numpy(Jv)
    zref = T.winner_z(Jv[:n], g1, winners)
    finite = [v for v in zref.values() if np.isfinite(v)]
    thr = float(np.median(finite)) if finite else 0.0
    fb = torch.zeros(B.P, dtype=torch.int32, device="cuda")
    zz = torch.zeros(B.P, dtype=torch.float64, device="cuda")
    sel2_b = torch.full((nb_, 4), -1, dtype=torch.int32, device="cuda")
    sel2_t = torch.zeros_like(sel_t)
    sel2_i = torch.full((nb_,), -1, dtype=torch.int64, device="cuda")
    n2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    pm.triage_fallback_select(B, b.buckets, nb_, b.n_out, sel_b, n_sel, best, J, iters, thr, b.theta0, 4, 11, taken,
                              sel2_b, sel2_t, sel2_i, n2, fb, zz, ws, wsb)
    torch.cuda.synchronize()
    flags = fb.cpu().numpy()
    zg = zz.cpu().numpy()
    has = np.array([np.any(group == p) for p in range(B.P)])
    exp_flags = np.zeros(B.P, dtype=int)
    for p in range(B.P):
        zp = zref.get(p, -np.inf)
        if np.isfinite(zp):
            assert abs(zg[p] - zp) <= 1e-9 * max(1.0, abs(zp)), (p, zg[p], zp)
        else:
            assert zg[p] == -np.inf
        exp_flags[p] = int(has[p] and not (zp >= thr))
    assert np.array_equal(flags, exp_flags)
    want2 = np.nonzero(~keep & exp_flags[group].astype(bool))[0]
    assert int(n2.item()) == len(want2)
    assert np.array_equal(sel2_i.cpu().numpy()[:len(want2)], want2)


def _triaged_vs_full(threshold, frac, prec=pm.PM_FP64):
    insts, B = _batch("triaged pipeline", 6, 13, 6, 3)
    s, iters, beta = 2, 3, 1.0
    bg = np.full(4, 0.25)
    nb_, nm_ = pm.size_batch(B, s)
    full = pm.BatchPipeline(B, s, iters, beta, prec, bg, nb_, nm_)
    full.run()
    rng = np.random.default_rng(11)
    P = T.init_params(rng)
    tri = pm.Triage(T.flat(P).astype(np.float32), np.zeros(87), np.ones(87), threshold)
    TP = pm.TriagedBatchPipeline(B, s, iters, beta, prec, bg, nb_, nm_, tri, frac=frac)
    TP.run()
    torch.cuda.synchronize()
    return B, full, TP, nb_


def test_triaged_pipeline_always_fallback_equals_full():
    """Threshold +inf: every instance refines all of its buckets (triaged ones
    first, then the rest); the winner must be the full pipeline's."""
    say("triaged = full (threshold inf)")
    B, full, TP, nb_ = _triaged_vs_full(np.inf, 0.05)
    fr, tr = full.results(), TP.results()
    assert TP.refined == nb_
    Jf = full.b.J.cpu().numpy()
    for p in range(B.P):
        assert fr[p]["best"] == tr[p]["best"], p
        if fr[p]["best"] >= 0:
            assert fr[p]["consensus"] == tr[p]["consensus"]
            assert tr[p]["J"] == Jf[fr[p]["best"], -1]


def test_triaged_pipeline_fraction_one_equals_full():
    say("triaged = full (frac 1)")
    B, full, TP, nb_ = _triaged_vs_full(-np.inf, 1.0)
    fr, tr = full.results(), TP.results()
    assert TP.refined == nb_
    for p in range(B.P):
        assert fr[p]["best"] == tr[p]["best"] and not tr[p]["fell_back"], p


def test_triaged_pipeline_refines_the_fraction():
    say("triaged refines top fraction")
    B, full, TP, nb_ = _triaged_vs_full(-np.inf, 0.05)
    tr = TP.results()
    bk = full.b.buckets.cpu().numpy().view(np.uint32)[:nb_]
    group = B.item_inst.cpu().numpy()[bk[:, 0]]
    # buckets with equal features score equal and ties are all kept: the count
    # is the oracle's top fraction of the GPU's own scores
    scores = TP.score_buf.cpu().numpy()[:nb_].astype(np.float64)
    expect = int(T.top_fraction(scores, group, 0.05).sum())
    assert TP.refined == expect
    assert expect >= sum(max(1, math.ceil(0.05 * np.sum(group == p))) for p in range(B.P) if np.any(group == p))
    for p in range(B.P):
        assert not tr[p]["fell_back"]
