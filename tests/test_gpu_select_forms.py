"""bucket_select on trials large enough to use every form of its member
placement, against the CPU oracle (Alg. 2 step 3; Sec. 6's threshold s).

The selection keeps each trial's member cursors in LDS when its buckets fit
there (a first launch with a small LDS footprint), in further launches with
LDS rows for four, two and one workgroups per CU for trials with more
buckets, in ranges of buckets taken by separate workgroups beyond that;
windows go by in chunks of 2048, or by wave quarters in two passes when a
trial has more buckets than half a chunk's windows, and a wave groups its passing windows by key with one
ballot per key when few pass and with ballots over the key bits when many
do.  Bucket lists and members must match the oracle bit for bit in every
form, also truncated to a capacity and in a batch whose instances take
different forms.
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


def _case(name, A, t, n, l, k, m):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    lens = [int(v) for v in rng.integers(n - n // 5, n + n // 5, size=t)]
    seqs = random_sequences(rng, t, lens, "dna" if A == 4 else "protein")
    return seqs, projection_masks(rng, l, k, m)


def _select(S, A, l, k, s, K, N, cap_b=None, cap_m=None):
    m = K.shape[0]
    dK = torch.from_numpy(K.view(np.int32)).cuda()
    dN = torch.from_numpy(N.view(np.int32)).cuda()
    nout = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    if cap_b is None:
        ws = torch.zeros(pm.pm_select_workspace(A, k, m, 0) // 4 + 1, dtype=torch.int32, device="cuda")
        pm.bucket_select(S, l, k, dK, dN, m, s, None, 0, None, 0, nout, ws, ws.numel() * 4, st)
        torch.cuda.synchronize()
        cap_b, cap_m = [int(v) for v in nout.cpu()]
        st.zero_()
    bk = torch.full((max(cap_b, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(cap_m, 1),), -1, dtype=torch.int32, device="cuda")
    ws = torch.zeros(pm.pm_select_workspace(A, k, m, cap_b) // 4 + 1, dtype=torch.int32, device="cuda")
    pm.bucket_select(S, l, k, dK, dN, m, s, bk, cap_b, mem, cap_m, nout, ws, ws.numel() * 4, st)
    torch.cuda.synchronize()
    return u32(bk), u32(mem), [int(v) for v in nout.cpu()], int(st.item())


CASES = [
    # name, alphabet, t, n, l, k, s, m; the form each trial takes on a device
    # with 160 KB of LDS per workgroup is in the name
    ("chunks, few passing, LDS rows", 4, 10, 1300, 15, 7, 3, 3),
    ("many passing, second launch, LDS rows", 4, 10, 2000, 12, 6, 1, 2),
    ("many passing, device-memory rows", 4, 10, 3500, 12, 7, 1, 2),
    ("protein, second launch, LDS rows", 20, 10, 2000, 8, 3, 1, 2),
    ("protein k=4, few passing", 20, 12, 1500, 10, 4, 3, 3),
    # more buckets than the first launch takes, few enough for the heavy
    # tier whose LDS rows let four workgroups share a CU
    ("tier of four workgroups per CU", 4, 6, 1500, 12, 6, 3, 3),
    ("tier of four workgroups per CU, protein", 20, 6, 1500, 8, 3, 2, 3),
    # about 58 000 buckets per trial: eight ranges of LDS rows, each taken by
    # its own workgroup over all of the trial's windows
    ("protein k=4, s=1, several bucket ranges", 20, 12, 6000, 10, 4, 1, 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_select_large_trials_match_oracle(case):
    name, A, t, n, l, k, s, m = case
    seqs, masks = _case(name, A, t, n, l, k, m)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    per_trial = np.bincount(rbk[:, 0], minlength=m)
    say("select forms", name, "x", RK.shape[1], "buckets per trial", per_trial.tolist())
    S = pm.Seqs(A, seqs)
    bk, mem, (nb_, nm_), st = _select(S, A, l, k, s, RK, RN)
    assert st == 0 and (nb_, nm_) == (rnb, rnm)
    assert np.array_equal(bk[:nb_], rbk)
    assert np.array_equal(mem[:nm_], rmem)


@pytest.mark.parametrize("which", [0, 1, 2, 3, 7], ids=[CASES[i][0] for i in (0, 1, 2, 3, 7)])
def test_select_truncated_to_capacity(which):
    """Capacities that end inside a trial's buckets and inside a bucket's
    members, in every placement form: the kept records and every member slot
    of a kept bucket below the member capacity as the oracle's."""
    name, A, t, n, l, k, s, m = CASES[which]
    seqs, masks = _case(name, A, t, n, l, k, m)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    cap_b, cap_m = rnb // 2 + 3, rnm // 3
    say("select forms truncated", name, cap_b, cap_m)
    S = pm.Seqs(A, seqs)
    bk, mem, (nb_, nm_), st = _select(S, A, l, k, s, RK, RN, cap_b=cap_b, cap_m=cap_m)
    assert st & pm.PM_STATUS_CAPACITY and (nb_, nm_) == (rnb, rnm)
    assert np.array_equal(bk[:cap_b], rbk[:cap_b])
    # every member slot below the capacity that belongs to a kept bucket
    slots = np.zeros(cap_m, dtype=bool)
    for b in rbk[:cap_b]:
        slots[b[3]:min(b[3] + b[2], cap_m)] = True
    assert slots.any()
    assert np.array_equal(mem[:cap_m][slots], rmem[:cap_m][slots])


def test_select_batch_mixes_light_and_heavy_trials():
    """One batch, s = 1, k = 6: a small instance whose trials fit the first
    launch and a large one whose trials go to the second."""
    A, l, k, s = 4, 12, 6, 1
    insts = [_case("light", A, 3, 200, l, k, 3), _case("heavy", A, 10, 2000, l, k, 2),
             _case("light 2", A, 4, 150, l, k, 2)]
    say("select forms batch")
    B = pm.Batch(A, l, k, [sq for sq, _ in insts], [mk for _, mk in insts])
    nb_, nm_ = pm.size_batch(B, s)
    P = pm.BatchPipeline(B, s, 0, 1.0, pm.PM_FP64, np.full(A, 0.25), cap_b=nb_, cap_m=nm_)
    P.hash()
    P.select()
    torch.cuda.synchronize()
    b = P.b
    assert int(b.status.item()) == 0
    bk, mem = u32(b.buckets)[:nb_], u32(b.members)[:nm_]
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


def _check_batch_against_oracle(B, insts, A, l, k, s, bk, mem, nb_):
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


def test_select_batch_spans_every_heavy_tier():
    """One batch, DNA k = 7, s = 1, whose trials fall in the first launch and
    in every heavy tier of one call (LDS rows for four, two and one
    workgroups per CU, and several bucket ranges), all taken from the tiers'
    work queues; every instance's list bit-exact against the oracle, through
    bucket_select_batch and through projection_hash_select_batch."""
    A, l, k, s = 4, 12, 7, 1
    insts = [_case("tier first launch", A, 2, 400, l, k, 2), _case("tier four per CU", A, 2, 800, l, k, 2),
             _case("tier two per CU", A, 4, 880, l, k, 2), _case("tier one per CU", A, 6, 1500, l, k, 2),
             _case("tier ranges", A, 15, 2000, l, k, 2)]
    buckets = []
    for seqs, masks in insts:
        ref = oracle.Seqs(A, seqs)
        RK, RN = oracle.hash_trials(ref, l, k, masks)
        buckets.append(int((RN >= s).sum(axis=1).max()))
    say("select forms, every heavy tier", buckets)
    # first launch <= 1024 buckets, then 2 144, 4 672 and 9 856 LDS rows on a
    # device with 160 KB of LDS per workgroup
    assert buckets[0] <= 1024 < buckets[1] <= 2144 < buckets[2] <= 4672 < buckets[3] <= 9856 < buckets[4]
    B = pm.Batch(A, l, k, [sq for sq, _ in insts], [mk for _, mk in insts])
    nb_, nm_ = pm.size_batch(B, s)
    for fused in (False, True):
        P = pm.BatchPipeline(B, s, 0, 1.0, pm.PM_FP64, np.full(A, 0.25), cap_b=nb_, cap_m=nm_)
        if fused:
            P.hash_select()
        else:
            P.hash()
            P.select()
        torch.cuda.synchronize()
        b = P.b
        assert int(b.status.item()) == 0
        _check_batch_against_oracle(B, insts, A, l, k, s, u32(b.buckets)[:nb_], u32(b.members)[:nm_], nb_)


def test_select_few_members_one_quarter_over_its_list():
    """A trial of few members whose passing windows crowd into the first
    quarter of its windows (a poly-A run of 400 windows first): that quarter
    holds more than its wave may list, so the trial falls back to the chunked
    placement; lists bit-exact against the oracle."""
    A, l, k, s, m = 4, 12, 8, 3, 3
    rng = np.random.default_rng(77)
    seqs = ["A" * (l + 399)] + random_sequences(rng, 7, [500] * 7, "dna")
    masks = projection_masks(rng, l, k, m)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    per_trial = np.bincount(rbk[:, 0], minlength=m, weights=rbk[:, 2])
    assert per_trial.max() <= 1024 and per_trial.min() >= 400
    say("select few members, crowded quarter", per_trial.tolist())
    S = pm.Seqs(A, seqs)
    bk, mem, (nb_, nm_), st = _select(S, A, l, k, s, RK, RN)
    assert st == 0 and (nb_, nm_) == (rnb, rnm)
    assert np.array_equal(bk[:nb_], rbk)
    assert np.array_equal(mem[:nm_], rmem)
