"""Fused projection + histogram + selection (bucket_hash_select and its
batch form) against the oracle: bucket records (trial, key, size, first)
bit-exact and in the oracle's order, the members of every bucket equal as a
set (the fused pass places them in no particular order; Alg. 2 step 3 defines
a bucket by its members, not their order), the required totals, capacity
truncation and bad masks."""
import sys
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm
from synth import planted_instance, projection_masks, random_sequences

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


def _fused(S, l, k, masks, s, cap_b=None, cap_m=None):
    m = len(masks)
    dm = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).cuda()
    nbytes = pm.pm_hash_select_workspace(S, l, k, m)
    assert nbytes > 0
    ws = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.bucket_hash_select(S, l, k, dm, m, s, None, 0, None, 0, n_out, ws, nbytes, None)
    torch.cuda.synchronize()
    nb_, nm_ = [int(v) for v in n_out.cpu()]
    cb = nb_ if cap_b is None else cap_b
    cm = nm_ if cap_m is None else cap_m
    bk = torch.full((max(cb, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(cm, 1),), -1, dtype=torch.int32, device="cuda")
    st.zero_()
    pm.bucket_hash_select(S, l, k, dm, m, s, bk, cb, mem, cm, n_out, ws, nbytes, st)
    torch.cuda.synchronize()
    return u32(bk)[:min(cb, nb_)], u32(mem)[:min(cm, nm_)], (nb_, nm_), int(st.item()), ws


def _check_against_oracle(bk, mem, totals, ref, l, k, masks, s, trial_map=None):
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, rtot, _ = oracle.select(ref, l, k, RK, RN, s)
    assert totals == rtot
    got = bk.copy()
    if trial_map is not None:
        got[:, 0] = trial_map(got[:, 0])
    assert np.array_equal(got, rbk)
    for b in rbk:
        f, n = int(b[3]), int(b[2])
        assert np.array_equal(np.sort(mem[f:f + n]), rmem[f:f + n])


FUSED_CASES = [
    # name, alphabet, t, lengths, l, k, m, s
    ("dna small ragged", 4, 6, [40, 33, 57, 19, 80, 26], 8, 5, 7, 2),
    ("dna several tiles", 4, 9, [700, 1500, 333, 64, 999, 1200, 41, 512, 2048], 15, 7, 11, 3),
    ("dna k=8 whole-trial histogram", 4, 8, [500] * 8, 12, 8, 5, 3),
    ("dna u32 histogram x>=65536", 4, 40, [1700] * 40, 12, 6, 3, 4),
    ("dna sliced k=9", 4, 10, [900] * 10, 21, 9, 4, 2),
    ("dna k=12 many slices", 4, 6, [300] * 6, 16, 12, 2, 2),
    ("dna s=1 every key", 4, 3, [90, 70, 50], 9, 4, 3, 1),
    ("protein k=3", 20, 7, [120, 31, 77, 64, 200, 23, 50], 10, 3, 5, 2),
    ("protein sliced k=4", 20, 12, [400] * 12, 20, 4, 3, 3),
    ("dna k=1", 4, 3, [10, 12, 9], 1, 1, 2, 2),
]


@pytest.mark.parametrize("case", FUSED_CASES, ids=[c[0] for c in FUSED_CASES])
def test_fused_select_matches_oracle(case):
    name, A, t, lens, l, k, m, s = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seqs = random_sequences(rng, t, lens, "dna" if A == 4 else "protein")
    masks = projection_masks(rng, l, k, m)
    say("fused select", name)
    S = pm.Seqs(A, seqs)
    bk, mem, totals, st, _ = _fused(S, l, k, masks, s)
    assert st == 0
    _check_against_oracle(bk, mem, totals, oracle.Seqs(A, seqs), l, k, masks, s)


def test_fused_select_planted_and_poly_a():
    """A planted instance (the enriched buckets of interest) and a poly-A
    sequence (every window of every trial in one bin: the largest bucket a
    trial can have and the most contended LDS counter)."""
    rng = np.random.default_rng(5)
    inst = planted_instance(rng, 12, 600, 15, 4)
    seqs = inst.seqs + ["A" * 900]
    masks = projection_masks(rng, 15, 7, 9)
    say("fused select planted + poly-A")
    S = pm.Seqs(4, seqs)
    bk, mem, totals, st, _ = _fused(S, 15, 7, masks, 3)
    assert st == 0
    _check_against_oracle(bk, mem, totals, oracle.Seqs(4, seqs), 15, 7, masks, 3)
    assert bk[:, 2].max() >= 886


def test_fused_select_capacity_and_bad_mask():
    rng = np.random.default_rng(6)
    seqs = random_sequences(rng, 5, [60, 80, 70, 90, 50], "dna")
    masks = projection_masks(rng, 10, 4, 5)
    say("fused select truncated")
    S = pm.Seqs(4, seqs)
    ref = oracle.Seqs(4, seqs)
    RK, RN = oracle.hash_trials(ref, 10, 4, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, 10, 4, RK, RN, 2)
    assert rnb > 8 and rnm > 20
    bk, mem, totals, st, _ = _fused(S, 10, 4, masks, 2, cap_b=8, cap_m=20)
    assert st & pm.PM_STATUS_CAPACITY and totals == (rnb, rnm)
    assert np.array_equal(bk[:8], rbk[:8])
    for b in rbk[:8]:
        f, n = int(b[3]), int(b[2])
        if f + n <= 20:
            assert np.array_equal(np.sort(mem[f:f + n]), rmem[f:f + n])
    # a mask keeping the wrong number of positions: flagged, that trial adds nothing
    bad = masks.copy()
    bad[2] = 0b111
    say("fused select bad mask")
    bk2, mem2, totals2, st2, _ = _fused(S, 10, 4, bad, 2)
    assert st2 & pm.PM_STATUS_BAD_MASK
    keep = np.array([0, 1, 3, 4])
    RK2, RN2 = oracle.hash_trials(ref, 10, 4, masks[keep])
    rbk2, rmem2, rtot2, _ = oracle.select(ref, 10, 4, RK2, RN2, 2)
    assert totals2 == rtot2
    mapped = bk2.copy()
    mapped[:, 0] = np.searchsorted(keep, mapped[:, 0])
    assert np.array_equal(mapped, rbk2)


def test_fused_select_batch_matches_per_instance_oracle():
    """The batch form over instances of one shape class: every instance's
    buckets (trial = item) equal the oracle's for that instance."""
    rng = np.random.default_rng(7)
    insts = []
    for p in range(5):
        t = int(rng.integers(3, 9))
        lens = [int(v) for v in rng.integers(20, 400, size=t)]
        inst = planted_instance(rng, t, lens, 13, 3)
        insts.append((inst, projection_masks(rng, 13, 6, int(rng.integers(2, 7)))))
    say("fused select batch")
    B = pm.Batch(4, 13, 6, [i.seqs for i, _ in insts], [mk for _, mk in insts])
    nbytes = pm.pm_hash_select_batch_workspace(B)
    ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.bucket_hash_select_batch(B, B.masks, 2, None, 0, None, 0, n_out, ws, nbytes, None)
    torch.cuda.synchronize()
    nb_, nm_ = [int(v) for v in n_out.cpu()]
    bk = torch.zeros((nb_, 4), dtype=torch.int32, device="cuda")
    mem = torch.zeros(nm_, dtype=torch.int32, device="cuda")
    pm.bucket_hash_select_batch(B, B.masks, 2, bk, nb_, mem, nm_, n_out, ws, nbytes, st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    bk, mem = u32(bk), u32(mem)
    for p, (inst, masks) in enumerate(insts):
        f0, m = B.first_item[p], B.m[p]
        sel = (bk[:, 0] >= f0) & (bk[:, 0] < f0 + m)
        mine = bk[sel]
        ref = oracle.Seqs(4, inst.seqs)
        RK, RN = oracle.hash_trials(ref, 13, 6, masks)
        rbk, rmem, _, _ = oracle.select(ref, 13, 6, RK, RN, 2)
        assert np.array_equal(mine[:, 0] - f0, rbk[:, 0]) and np.array_equal(mine[:, 1:3], rbk[:, 1:3])
        for a, b in zip(mine, rbk):
            assert np.array_equal(np.sort(mem[a[3]:a[3] + a[2]]), rmem[b[3]:b[3] + b[2]])
