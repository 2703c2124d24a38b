"""projection_hash_select: keys, counts, the enriched-bucket list and its
members in one call, the selection's passing-key bitmap and per-trial totals
formed by the hash pass while each trial's histogram is in LDS (Alg. 2 steps
2(b), 2(c) and 3; Sec. 6's threshold s).

Every output must be bit-exact against the CPU oracle and equal to
projection_hash followed by bucket_select: in every member-placement form of
the selection, with one and with two key-range slices per trial, with 4-, 8-
and 32-bit LDS counters, with 4- and 8-bit counters that wrap (the slice
counted again in u32, its bitmap formed from those counts), truncated to
capacities, with a bad mask, on a reused workspace and over a batch.
"""
import sys
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm
from synth import random_sequences, projection_masks

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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def _fused(S, A, l, k, s, masks, cap_b, cap_m, ws=None):
    m, x = len(masks), S.nwin(l)
    keys = torch.full((m, x), -1, dtype=torch.int32, device="cuda")
    counts = torch.full((m, A ** k), -1, dtype=torch.int32, device="cuda")
    bk = torch.full((max(cap_b, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(cap_m, 1),), -1, dtype=torch.int32, device="cuda")
    nout = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    if ws is None:
        ws = torch.zeros(pm.pm_select_workspace(A, k, m, cap_b) // 4 + 1, dtype=torch.int32, device="cuda")
    pm.projection_hash_select(S, l, k, _dev(masks), m, keys, counts, s, bk, cap_b, mem, cap_m, nout, ws,
                              ws.numel() * 4, st)
    torch.cuda.synchronize()
    return dict(keys=u32(keys), counts=u32(counts), buckets=u32(bk), members=u32(mem),
                n_out=[int(v) for v in nout.cpu()], status=int(st.item()))


def _separate(S, A, l, k, s, masks, cap_b, cap_m):
    m, x = len(masks), S.nwin(l)
    keys = torch.full((m, x), -1, dtype=torch.int32, device="cuda")
    counts = torch.full((m, A ** k), -1, dtype=torch.int32, device="cuda")
    bk = torch.full((max(cap_b, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(cap_m, 1),), -1, dtype=torch.int32, device="cuda")
    nout = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = torch.zeros(pm.pm_select_workspace(A, k, m, cap_b) // 4 + 1, dtype=torch.int32, device="cuda")
    pm.projection_hash(S, l, k, _dev(masks), m, keys, counts, st)
    pm.bucket_select(S, l, k, keys, counts, m, s, bk, cap_b, mem, cap_m, nout, ws, ws.numel() * 4, st)
    torch.cuda.synchronize()
    return dict(keys=u32(keys), counts=u32(counts), buckets=u32(bk), members=u32(mem),
                n_out=[int(v) for v in nout.cpu()], status=int(st.item()))


def _random_case(name, A, t, n, l, k, m):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    lens = [int(v) for v in rng.integers(n - n // 5, n + n // 5, size=t)]
    return random_sequences(rng, t, lens, "dna" if A == 4 else "protein"), projection_masks(rng, l, k, m)


def _runs_case(name, A, l, k, runs, m):
    """Random sequences plus one-letter runs: a run of c windows puts c
    windows on one key under every mask (counts at a narrow counter's limit)."""
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    alpha = "dna" if A == 4 else "protein"
    seqs = random_sequences(rng, 8, [2500] * 8, alpha) + [ch * (l + c - 1) for ch, c in runs]
    return seqs, projection_masks(rng, l, k, m)


CASES = [
    # name, alphabet, t, n, l, k, s, m, runs (None: random sequences only).
    # Counter width and slices on a device with 160 KB of LDS per workgroup,
    # and the selection's member placement, in the name.
    ("u8 one slice, chunks, few passing", 4, 10, 1300, 15, 7, 3, 3, None),
    ("u8 one slice, many passing, second launch", 4, 10, 2000, 12, 6, 1, 2, None),
    ("many passing, device-memory rows", 4, 10, 3500, 12, 7, 1, 2, None),
    ("protein, second launch", 20, 10, 2000, 8, 3, 1, 2, None),
    ("protein k=4, u4 two balanced slices", 20, 12, 1500, 10, 4, 2, 3, None),
    ("DNA k=9, u4 two balanced slices", 4, 8, 2000, 12, 9, 2, 3, None),
    ("DNA k=5, u32 table", 4, 6, 300, 10, 5, 2, 4, None),
    ("DNA k=2, one bitmap word", 4, 5, 100, 8, 2, 3, 3, None),
    ("DNA s=0 as s=1", 4, 6, 400, 11, 6, 0, 3, None),
    ("u4 count 16 wraps, two slices recounted", 4, 0, 0, 12, 9, 3, 3, [("C", 15), ("T", 16), ("G", 40)]),
    ("u4 protein count 17 wraps", 20, 0, 0, 10, 4, 3, 3, [("A", 17), ("W", 15)]),
    ("u8 counts 255 and 256", 4, 0, 0, 11, 8, 4, 3, [("C", 255), ("A", 256)]),
]


def _inputs(case):
    name, A, t, n, l, k, s, m, runs = case
    if runs is None:
        return _random_case(name, A, t, n, l, k, m)
    return _runs_case(name, A, l, k, runs, m)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_hash_select_matches_oracle_and_separate_calls(case):
    name, A, t, n, l, k, s, m, runs = case
    seqs, masks = _inputs(case)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    say("hash+select", name, "x", RK.shape[1], "buckets", rnb, "members", rnm)
    S = pm.Seqs(A, seqs)
    F = _fused(S, A, l, k, s, masks, rnb, rnm)
    assert F["status"] == 0 and F["n_out"] == [rnb, rnm]
    assert np.array_equal(F["keys"], RK) and np.array_equal(F["counts"], RN)
    assert np.array_equal(F["buckets"][:rnb], rbk)
    assert np.array_equal(F["members"][:rnm], rmem)
    G = _separate(S, A, l, k, s, masks, rnb, rnm)
    for key in F:
        assert np.array_equal(np.asarray(F[key]), np.asarray(G[key])), key
    if runs is not None:
        assert RN.max() >= max(c for _, c in runs)


def test_hash_select_sizing_call_then_reused_workspace():
    """Zero capacities size the lists; two full calls on one workspace (the
    per-trial totals start again from zero) give the oracle's lists."""
    name, A, t, n, l, k, s, m, _ = CASES[1]
    seqs, masks = _inputs(CASES[1])
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    say("hash+select sizing and reuse", name)
    S = pm.Seqs(A, seqs)
    Z = _fused(S, A, l, k, s, masks, 0, 0)
    assert Z["n_out"] == [rnb, rnm] and Z["status"] == pm.PM_STATUS_CAPACITY
    ws = torch.zeros(pm.pm_select_workspace(A, k, m, rnb) // 4 + 1, dtype=torch.int32, device="cuda")
    for _ in range(2):
        F = _fused(S, A, l, k, s, masks, rnb, rnm, ws=ws)
        assert F["status"] == 0 and F["n_out"] == [rnb, rnm]
        assert np.array_equal(F["buckets"][:rnb], rbk) and np.array_equal(F["members"][:rnm], rmem)


@pytest.mark.parametrize("which", [0, 2, 5], ids=[CASES[i][0] for i in (0, 2, 5)])
def test_hash_select_truncated_like_separate_calls(which):
    case = CASES[which]
    name, A, t, n, l, k, s, m, _ = case
    seqs, masks = _inputs(case)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    _, _, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    cap_b, cap_m = rnb // 2 + 3, rnm // 3
    say("hash+select truncated", name, cap_b, cap_m)
    S = pm.Seqs(A, seqs)
    F = _fused(S, A, l, k, s, masks, cap_b, cap_m)
    G = _separate(S, A, l, k, s, masks, cap_b, cap_m)
    assert F["status"] & pm.PM_STATUS_CAPACITY and F["n_out"] == [rnb, rnm]
    for key in F:
        assert np.array_equal(np.asarray(F[key]), np.asarray(G[key])), key


def test_hash_select_bad_mask_trial_gives_no_buckets():
    """A mask with the wrong number of kept positions: PM_STATUS_BAD_MASK and
    no buckets from that trial; the other trials' lists as the oracle's."""
    A, l, k, s = 4, 12, 6, 2
    seqs, masks = _random_case("bad mask", A, 6, 600, l, k, 3)
    bad = np.array(masks, dtype=np.uint32)
    bad[1] = (1 << (k + 1)) - 1  # k + 1 positions
    good = [0, 2]
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, bad[good])
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    rbk = rbk.copy()
    rbk[:, 0] = np.array(good, dtype=np.uint32)[rbk[:, 0]]
    say("hash+select bad mask")
    S = pm.Seqs(A, seqs)
    F = _fused(S, A, l, k, s, bad, rnb, rnm)
    assert F["status"] & pm.PM_STATUS_BAD_MASK
    assert F["n_out"] == [rnb, rnm]
    assert np.array_equal(F["buckets"][:rnb], rbk) and np.array_equal(F["members"][:rnm], rmem)
    assert np.array_equal(F["keys"][good], RK) and np.array_equal(F["counts"][good], RN)


def test_hash_select_batch_equals_separate_batch_calls():
    """One batch of three instances (trials of both selection launches):
    BatchPipeline.hash_select against hash then select, every output."""
    A, l, k, s = 4, 12, 6, 1
    insts = [_random_case("light", A, 3, 200, l, k, 3), _random_case("heavy", A, 10, 2000, l, k, 2),
             _random_case("light 2", A, 4, 150, l, k, 2)]
    say("hash+select batch")
    B = pm.Batch(A, l, k, [sq for sq, _ in insts], [mk for _, mk in insts])
    nb_, nm_ = pm.size_batch(B, s)
    out = []
    for fused in (True, False):
        P = pm.BatchPipeline(B, s, 0, 1.0, pm.PM_FP64, np.full(A, 0.25), cap_b=nb_, cap_m=nm_)
        if fused:
            P.hash_select()
        else:
            P.hash()
            P.select()
        torch.cuda.synchronize()
        b = P.b
        out.append(dict(status=int(b.status.item()), n_out=[int(v) for v in b.n_out.cpu()], keys=u32(b.keys),
                        counts=u32(b.counts), buckets=u32(b.buckets)[:nb_], members=u32(b.members)[:nm_]))
    F, G = out
    assert F["status"] == 0 and F["n_out"] == [nb_, nm_]
    for key in F:
        assert np.array_equal(np.asarray(F[key]), np.asarray(G[key])), key
    # and per instance against the oracle
    bk, mem = F["buckets"], F["members"]
    tot = 0
    for p, (seqs, masks) in enumerate(insts):
        ref = oracle.Seqs(A, seqs)
        RK, RN = oracle.hash_trials(ref, l, k, masks)
        rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
        f, mp = B.first_item[p], B.m[p]
        sel = (bk[:, 0] >= f) & (bk[:, 0] < f + mp)
        gb = bk[sel]
        assert len(gb) == rnb, p
        assert np.array_equal(gb[:, 0] - f, rbk[:, 0]) and np.array_equal(gb[:, 1:3], rbk[:, 1:3]), p
        for g, r in zip(gb, rbk):
            assert np.array_equal(mem[g[3]:g[3] + g[2]], rmem[r[3]:r[3] + r[2]]), p
        tot += rnb
    assert tot == nb_
