"""Batched path (many uneven instances of one shape class in one set of
launches) against the CPU oracle run instance by instance.

Keys, counts, bucket lists, members and profiles bit-exact; EM within the
tolerances of the single-instance parity tests; per-instance best model and
consensus as the oracle's.  A graph-captured pass replays to the eager result.
"""
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


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def _instances(name, P, l, k, d, alphabet="dna", tiny_last=True):
    """P uneven instances: t in [3, 8], ragged n, m in [2, 8]; the last one
    (optionally) too small to fill any bucket."""
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    out = []
    for p in range(P):
        if tiny_last and p == P - 1:
            t, lens = 1, [l + 2]
        else:
            t = int(rng.integers(3, 9))
            lens = [int(v) for v in rng.integers(l + 2, 260, size=t)]
        inst = planted_instance(rng, t, lens, l, d, alphabet,
                                dirichlet_alpha=2.0 if alphabet == "protein" else None)
        masks = projection_masks(rng, l, k, int(rng.integers(2, 9)))
        out.append((inst, masks))
    return out


def _batch(insts, A, l, k):
    return pm.Batch(A, l, k, [i.seqs for i, _ in insts], [mk for _, mk in insts])


def _pipeline(B, s, iters, beta, precision, bg):
    nb_, nm_ = pm.size_batch(B, s)
    P = pm.BatchPipeline(B, s, iters, beta, precision, bg, cap_b=nb_, cap_m=nm_)
    return P, nb_, nm_


def _oracle_instance(inst, masks, A, l, k, s):
    ref = oracle.Seqs(A, inst.seqs)
    K, N = oracle.hash_trials(ref, l, k, masks)
    bk, mem, (nb_, nm_), _ = oracle.select(ref, l, k, K, N, s)
    prof = oracle.profile(ref, l, bk, mem)
    return ref, K, N, bk, mem, prof


BATCH_CASES = [
    # name, alphabet, P, l, k, d, s
    ("dna l=11 k=5 s=2", 4, 7, 11, 5, 3, 2),
    ("dna l=15 k=7 s=3", 4, 5, 15, 7, 4, 3),
    ("protein l=10 k=2 s=3", 20, 4, 10, 2, 2, 3),
]


@pytest.mark.parametrize("case", BATCH_CASES, ids=[c[0] for c in BATCH_CASES])
def test_batch_hash_select_profile_bit_exact(case):
    name, A, P, l, k, d, s = case
    insts = _instances(name, P, l, k, d, "dna" if A == 4 else "protein")
    say("batch select", name)
    B = _batch(insts, A, l, k)
    bg = np.full(A, 1.0 / A)
    Pp, nb_, nm_ = _pipeline(B, s, 0, 1.0, pm.PM_FP64, bg)
    Pp.hash()
    Pp.select()
    Pp.profile()
    torch.cuda.synchronize()
    b = Pp.b
    assert int(b.status.item()) == 0
    keys, counts = u32(b.keys), u32(b.counts)
    bk, mem, prof = u32(b.buckets)[:nb_], u32(b.members)[:nm_], u32(b.profile)[:nb_]
    th0 = b.theta0.cpu().numpy()[:nb_]
    tot_b = tot_m = 0
    for p, (inst, masks) in enumerate(insts):
        ref, RK, RN, rbk, rmem, rprof = _oracle_instance(inst, masks, A, l, k, s)
        f, x, m = B.first_item[p], B.x[p], B.m[p]
        got_k = keys[B.key_base[p]:B.key_base[p] + m * x].reshape(m, x)
        assert np.array_equal(got_k, RK), p
        assert np.array_equal(counts[f:f + m], RN), p
        sel = (bk[:, 0] >= f) & (bk[:, 0] < f + m)
        gb = bk[sel]
        assert len(gb) == len(rbk), p
        if len(rbk):
            assert np.array_equal(gb[:, 0] - f, rbk[:, 0]) and np.array_equal(gb[:, 1:3], rbk[:, 1:3]), p
            for g, r in zip(gb, rbk):
                assert np.array_equal(mem[g[3]:g[3] + g[2]], rmem[r[3]:r[3] + r[2]]), p
            assert np.array_equal(prof[sel], rprof), p
            np.testing.assert_allclose(th0[sel], oracle.theta0(rprof, bg, 1.0), rtol=1e-15, atol=0)
        tot_b += len(rbk)
        tot_m += int(rbk[:, 2].sum()) if len(rbk) else 0
    assert (nb_, nm_) == (tot_b, tot_m)
    # buckets ascend by item, members of a bucket follow its first slot
    assert np.all(np.diff(bk[:, 0].astype(np.int64)) >= 0)


def _same_best(got, ref, rJ, tol):
    if got != ref:
        assert abs(rJ[got, -1] - rJ[ref, -1]) <= tol * max(1.0, abs(rJ[ref, -1])), (got, ref)


@pytest.mark.parametrize("prec", [pm.PM_FP64, pm.PM_FP32, pm.PM_F16X2], ids=["fp64", "fp32", "f16x2"])
@pytest.mark.parametrize("case", BATCH_CASES, ids=[c[0] for c in BATCH_CASES])
def test_batch_em_and_best_match_oracle(case, prec):
    name, A, P, l, k, d, s = case
    if prec == pm.PM_F16X2 and A != 4:
        pytest.skip("the split-FP16 matrix-core path is for DNA")
    insts = _instances(name, P, l, k, d, "dna" if A == 4 else "protein")
    iters, beta = 4, 1.0
    bg = np.full(A, 1.0 / A)
    say("batch em", name, prec)
    B = _batch(insts, A, l, k)
    Pp, nb_, nm_ = _pipeline(B, s, iters, beta, prec, bg)
    Pp.run()
    torch.cuda.synchronize()
    b = Pp.b
    bk = u32(b.buckets)[:nb_]
    J, th = b.J.cpu().numpy()[:nb_], b.theta.cpu().numpy()[:nb_]
    sites = b.sites.cpu().numpy()[:nb_]
    res = Pp.results()
    tol = 1e-12 if prec == pm.PM_FP64 else 1e-5
    # theta after several EM steps moves more than J: J is flat in theta near a
    # fixed point, while a window pair with nearly equal scores passes a score
    # rounding of ~l * 2^-24 * |W| on to its posteriors; over the iterations
    # that reaches ~1e-4 on 20-letter columns (J stays within 1e-5)
    th_tol = 1e-12 if prec == pm.PM_FP64 else 1e-4
    multi = 0
    for p, (inst, masks) in enumerate(insts):
        ref, RK, RN, rbk, rmem, rprof = _oracle_instance(inst, masks, A, l, k, s)
        f, m = B.first_item[p], B.m[p]
        sel = np.nonzero((bk[:, 0] >= f) & (bk[:, 0] < f + m))[0]
        if len(rbk) == 0:
            assert len(sel) == 0 and res[p]["best"] == -1, p
            continue
        multi += len(rbk) > 64
        rth0 = oracle.theta0(rprof, bg, beta)
        rth, rJ, rLL, rsites = oracle.em(ref, l, rth0, bg, iters, beta)
        np.testing.assert_allclose(J[sel], rJ, rtol=tol, atol=tol * np.abs(rJ).max())
        np.testing.assert_allclose(th[sel], rth, rtol=0, atol=th_tol)
        if prec == pm.PM_FP64:
            assert np.array_equal(sites[sel, :B.t[p]], rsites), p
        rbest, rcons = oracle.best(rJ, rth)
        got = res[p]["best"] - sel[0]
        assert 0 <= got < len(sel)
        _same_best(got, rbest, rJ, tol)
        if got == rbest:
            assert res[p]["consensus"] == rcons or prec != pm.PM_FP64, p
    if A == 4 and name.startswith("dna l=11"):
        assert multi >= 1  # some instance spans several matrix-core workgroups



def _first_largest(Jf):
    """The winning index by definition: the largest final objective, the
    smallest index among equals, NaN skipped, -1 when nothing is left."""
    ok = ~np.isnan(Jf)
    if not ok.any():
        return -1
    return int(np.flatnonzero(ok & (Jf == Jf[ok].max()))[0])


def test_batch_best_is_each_instance_first_largest_final_objective():
    """Per instance: the winner among that instance's buckets only, by the
    pick rule, with crafted objectives (ties, NaN, -inf, an instance whose
    objectives are all NaN, one with no bucket) and a valid count that cuts
    an instance short."""
    name, A, P, l, k, d, s = next(c for c in BATCH_CASES if c[1] == 4 and c[0].startswith("dna l=11"))
    insts = _instances(name, P, l, k, d)
    say("batch best", name)
    B = _batch(insts, A, l, k)
    Pp, nb_, nm_ = _pipeline(B, s, 1, 1.0, pm.PM_FP64, np.full(A, 0.25))
    Pp.hash()
    Pp.select()
    torch.cuda.synchronize()
    trial = u32(Pp.b.buckets)[:nb_, 0].astype(np.int64)
    iters = 2
    rng = np.random.default_rng(5)
    Jf = rng.integers(0, 6, nb_).astype(np.float64)
    Jf[rng.random(nb_) < 0.2] = np.nan
    Jf[rng.random(nb_) < 0.1] = -np.inf
    ranges = [np.nonzero((trial >= f) & (trial < f + m))[0] for f, m in zip(B.first_item, B.m)]
    filled = [p for p in range(P) if len(ranges[p])]
    Jf[ranges[filled[0]]] = np.nan
    Jf[ranges[filled[1]]] = -np.inf
    J = np.concatenate([np.full((nb_, iters), 1e300), Jf[:, None]], axis=1)
    theta = rng.random((nb_, A, l))
    d_J = torch.from_numpy(np.ascontiguousarray(J)).cuda()
    d_th = torch.from_numpy(theta).cuda()
    for nvalid in (nb_, nb_ - 5):
        d_n = torch.tensor([nvalid], dtype=torch.int64, device="cuda")
        best = torch.full((P,), -7, dtype=torch.int64, device="cuda")
        cons = torch.full((P, l + 1), 0xFF, dtype=torch.uint8, device="cuda")
        pm.em_best_batch(B, Pp.b.buckets, d_J, nb_, d_n, iters, d_th, best, cons)
        torch.cuda.synchronize()
        got, gcons = best.cpu().numpy(), cons.cpu().numpy()
        for p in range(P):
            r = ranges[p][ranges[p] < nvalid]
            w = _first_largest(Jf[r]) if len(r) else -1
            ref = int(r[w]) if w >= 0 else -1
            assert int(got[p]) == ref, (nvalid, p)
            want = ("".join("ACTG"[c] for c in theta[ref].argmax(axis=0)).encode() if ref >= 0 else bytes(l)) + b"\0"
            assert bytes(gcons[p]) == want, (nvalid, p)
    assert len(filled) < P  # the last instance has no bucket


def test_batch_em_every_tile_shape_bit_identical():
    """The batch plan cuts every instance into workgroups of the tile shape's
    size (64 or 128 models); each shape gives the same bits, with instances
    that span several workgroups and ones that fill part of one."""
    name, A, P, l, k, d, s = next(c for c in BATCH_CASES if c[1] == 4 and c[0].startswith("dna l=11"))
    insts = _instances(name, P, l, k, d)
    bg = np.full(4, 0.25)
    say("batch em tile shapes", name)
    B = _batch(insts, A, l, k)
    out = {}
    try:
        for shape in (11, 12, 14, 21, 22, 24):
            pm.em_set_tuning(l, pm.PM_F16X2, shape)
            Pp, nb_, nm_ = _pipeline(B, s, 3, 1.0, pm.PM_F16X2, bg)
            Pp.run()
            torch.cuda.synchronize()
            b = Pp.b
            out[shape] = (b.J.cpu().numpy()[:nb_], b.theta.cpu().numpy()[:nb_], b.sites.cpu().numpy()[:nb_],
                          [r["best"] for r in Pp.results()])
    finally:
        pm.em_set_tuning(l, pm.PM_F16X2, 14)
    trial = u32(b.buckets)[:nb_, 0]
    per_inst = [int(((trial >= f) & (trial < f + m)).sum()) for f, m in zip(B.first_item, B.m)]
    assert max(per_inst) > 64 and min(per_inst) < 64, per_inst
    for shape in (12, 14, 21, 22, 24):
        for x, y in zip(out[11][:3], out[shape][:3]):
            assert np.array_equal(x, y), shape
        assert out[11][3] == out[shape][3], shape


def test_batch_graph_replays_match_eager():
    name, A, P, l, k, d, s = BATCH_CASES[0]
    insts = _instances(name, P, l, k, d)
    bg = np.full(4, 0.25)
    say("batch graph")
    B = _batch(insts, A, l, k)
    Pp, nb_, nm_ = _pipeline(B, s, 3, 1.0, pm.PM_F16X2, bg)
    Pp.run()
    torch.cuda.synchronize()
    eager_J = Pp.b.J.clone()
    eager_best = Pp.b.best.clone()
    eager_mem = Pp.b.members.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        Pp.run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Pp.run()
    for rep in range(3):
        Pp.b.J.fill_(-1.0)
        Pp.b.best.fill_(-7)
        Pp.b.members.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Pp.b.J, eager_J), rep
        assert torch.equal(Pp.b.best, eager_best), rep
        assert torch.equal(Pp.b.members, eager_mem), rep
        # eager work between replays
        _ = (torch.arange(1000, device="cuda") * 2).sum().item()


def test_batch_rejects_bad_tables():
    """Host checks of the batch table (no launch)."""
    insts = _instances("bad tables", 2, 11, 5, 3, tiny_last=False)
    B = _batch(insts, 4, 11, 5)
    say("batch checks")
    B.tab_host[1].first_item = 0
    with pytest.raises(pm.PmError):
        pm.pm_batch_check(B)
    B.tab_host[1].first_item = B.m[0]
    B.tab_host[1].x += 1
    with pytest.raises(pm.PmError):
        pm.pm_batch_check(B)
    B.tab_host[1].x -= 1
    pm.pm_batch_check(B)


def test_uneven_shape_classes_in_one_graph_match_oracle():
    """The uneven batching workload's rules at test size: motif lengths 11, 14,
    17 and 20 with d = floor(l/4) + 1 and k = clamp(l - d - 4, 6, 9), ragged t
    and n, two or three trials per instance (s = 2, so that every class fills
    buckets at this size); one batch per length, all four captured in one HIP
    graph and replayed twice with eager work between.  Per instance of every
    class: keys and counts bit-exact, J of every model (split FP16) within
    1e-5 of the oracle, the winner the oracle's (or tied with it in J) with
    its consensus."""
    rng = np.random.default_rng(2024)
    bg = np.full(4, 0.25)
    iters, s = 4, 2
    classes = []
    for l in (11, 14, 17, 20):
        d = l // 4 + 1
        k = min(max(l - d - 4, 6), 9)
        insts = []
        for _ in range(3):
            t = int(rng.integers(5, 13))
            lens = [int(v) for v in rng.integers(120, 420, size=t)]
            insts.append((planted_instance(rng, t, lens, l, d), projection_masks(rng, l, k, int(rng.integers(2, 4)))))
        B = _batch(insts, 4, l, k)
        Pp, nb_, nm_ = _pipeline(B, s, iters, 1.0, pm.PM_F16X2, bg)
        assert nb_ > 0, l
        classes.append((l, k, insts, B, Pp, nb_))
    say("uneven classes in one graph", [(c[0], c[5]) for c in classes])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        for c in classes:
            c[4].run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for c in classes:
            c[4].run()
    for rep in range(2):
        for c in classes:
            c[4].b.J.fill_(-1.0)
            c[4].b.best.fill_(-7)
            c[4].b.keys.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (torch.arange(1000, device="cuda") * 3).sum().item()
        for l, k, insts, B, Pp, nb_ in classes:
            b = Pp.b
            assert int(b.status.item()) == 0
            keys, counts = u32(b.keys), u32(b.counts)
            bk = u32(b.buckets)[:nb_]
            J = b.J.cpu().numpy()[:nb_]
            res = Pp.results()
            for p, (inst, masks) in enumerate(insts):
                ref, RK, RN, rbk, rmem, rprof = _oracle_instance(inst, masks, 4, l, k, s)
                f, x, m = B.first_item[p], B.x[p], B.m[p]
                assert np.array_equal(keys[B.key_base[p]:B.key_base[p] + m * x].reshape(m, x), RK), (rep, l, p)
                assert np.array_equal(counts[f:f + m], RN), (rep, l, p)
                sel = np.nonzero((bk[:, 0] >= f) & (bk[:, 0] < f + m))[0]
                assert len(sel) == len(rbk), (rep, l, p)
                if len(rbk) == 0:
                    assert res[p]["best"] == -1
                    continue
                rth, rJ, _, _ = oracle.em(ref, l, oracle.theta0(rprof, bg, 1.0), bg, iters, 1.0)
                np.testing.assert_allclose(J[sel], rJ, rtol=1e-5, atol=1e-5 * np.abs(rJ).max())
                rbest, rcons = oracle.best(rJ, rth)
                got = res[p]["best"] - sel[0]
                _same_best(got, rbest, rJ, 1e-5)
                if got == rbest:
                    assert res[p]["consensus"] == rcons, (rep, l, p)
