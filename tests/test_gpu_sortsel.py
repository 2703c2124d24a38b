"""Sorted selection (bucket_sort_select and its batch form; bucket_hash_select
for DNA k > 12 and protein k > 5) against the oracle's selection from keys
alone: bucket records (trial, key, size, first) and the members of every
bucket, in order, bit-exact; the required totals; capacity truncation; bad
masks; one key holding more windows than a sort buffer; and, where both exist,
equality with the count-table selection."""
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


def _sorted(S, l, k, masks, s, cap_b=None, cap_m=None, via_hash_select=False):
    m = len(masks)
    dm = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).cuda()
    if via_hash_select:
        nbytes = pm.pm_hash_select_workspace(S, l, k, m)
        run = pm.bucket_hash_select
    else:
        nbytes = pm.pm_sort_select_workspace(S, l, k, m)
        run = pm.bucket_sort_select
    assert nbytes > 0
    ws = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device="cuda")
    n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    run(S, l, k, dm, m, s, None, 0, None, 0, n_out, ws, nbytes, None)
    torch.cuda.synchronize()
    nb_, nm_ = [int(v) for v in n_out.cpu()]
    cb = nb_ if cap_b is None else cap_b
    cm = nm_ if cap_m is None else cap_m
    bk = torch.full((max(cb, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(cm, 1),), -1, dtype=torch.int32, device="cuda")
    run(S, l, k, dm, m, s, bk, cb, mem, cm, n_out, ws, nbytes, st)
    torch.cuda.synchronize()
    return u32(bk)[:min(cb, nb_)], u32(mem)[:min(cm, nm_)], (nb_, nm_), int(st.item())


def _oracle_sorted(seqs, A, l, k, masks, s):
    ref = oracle.Seqs(A, seqs)
    RK, _ = oracle.hash_trials(ref, l, k, masks, counts=False)
    bk, mem, tot, _ = oracle.select_sorted(ref, l, RK, s)
    return bk, mem, tot


SORT_CASES = [
    # name, alphabet, t, lengths, l, k, m, s
    ("dna k=13 ragged", 4, 7, [300, 41, 777, 120, 64, 512, 1000], 16, 13, 6, 2),
    ("dna k=14 planted-size", 4, 20, [600] * 20, 18, 14, 5, 2),
    ("dna k=16 full 32-bit keys", 4, 9, [900] * 9, 20, 16, 4, 2),
    ("dna k=16 several slices", 4, 30, [1500] * 30, 21, 16, 3, 2),
    ("protein k=6", 20, 10, [400, 90, 300, 777, 150, 60, 500, 222, 333, 100], 12, 6, 5, 2),
    ("protein k=7", 20, 12, [600] * 12, 14, 7, 4, 2),
    ("dna k=14 s=1 every key", 4, 3, [200, 150, 90], 16, 14, 3, 1),
]


@pytest.mark.parametrize("case", SORT_CASES, ids=[c[0] for c in SORT_CASES])
def test_sorted_select_matches_oracle(case):
    name, A, t, lens, l, k, m, s = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seqs = random_sequences(rng, t, lens, "dna" if A == 4 else "protein")
    masks = projection_masks(rng, l, k, m)
    say("sorted select", name)
    S = pm.Seqs(A, seqs)
    rbk, rmem, rtot = _oracle_sorted(seqs, A, l, k, masks, s)
    bk, mem, tot, st = _sorted(S, l, k, masks, s)
    assert st == 0 and tot == rtot
    assert np.array_equal(bk, rbk) and np.array_equal(mem, rmem)
    # bucket_hash_select routes these key spaces to the same path
    say("sorted select via bucket_hash_select", name)
    bk2, mem2, tot2, st2 = _sorted(S, l, k, masks, s, via_hash_select=True)
    assert st2 == 0 and tot2 == rtot
    assert np.array_equal(bk2, rbk) and np.array_equal(mem2, rmem)


@pytest.mark.parametrize("A,l,k", [(4, 12, 8), (4, 16, 12), (20, 10, 4), (20, 12, 5)],
                         ids=["dna k=8", "dna k=12", "protein k=4", "protein k=5"])
def test_sorted_select_equals_count_table_selection(A, l, k):
    """Where the count table also applies, the sorted path gives the count
    table's bucket records and members (sorted), and both equal the oracle's
    count-table selection."""
    rng = np.random.default_rng(100 * A + k)
    seqs = planted_instance(rng, 12, 500, l, 2).seqs if A == 4 else random_sequences(rng, 12, [500] * 12, "protein")
    masks = projection_masks(rng, l, k, 5)
    say("sorted vs count table", A, l, k)
    S = pm.Seqs(A, seqs)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, rtot, _ = oracle.select(ref, l, k, RK, RN, 3)
    bk, mem, tot, st = _sorted(S, l, k, masks, 3)
    assert st == 0 and tot == rtot
    assert np.array_equal(bk, rbk) and np.array_equal(mem, rmem)


def test_sorted_select_one_key_beyond_the_sort_buffer():
    """Poly-A sequences: in every trial one key holds every window of them
    (more than the 8192 pairs a sort buffer takes), beside random sequences
    whose keys share its slice; the key range is narrowed down to that single
    key, which forms its bucket directly."""
    rng = np.random.default_rng(11)
    seqs = ["A" * 5000, "A" * 4000] + random_sequences(rng, 6, [700] * 6, "dna")
    masks = projection_masks(rng, 16, 13, 3)
    say("sorted select poly-A beyond the buffer")
    S = pm.Seqs(4, seqs)
    rbk, rmem, rtot = _oracle_sorted(seqs, 4, 16, 13, masks, 2)
    bk, mem, tot, st = _sorted(S, 16, 13, masks, 2)
    assert st == 0 and tot == rtot
    assert np.array_equal(bk, rbk) and np.array_equal(mem, rmem)
    assert rbk[:, 2].max() > 8192


def test_sorted_select_low_complexity_narrowing():
    """Tandem repeats crowd a few key ranges with many distinct keys (coarse
    bins over the buffer that hold more than one key), so ranges are narrowed
    several times before they fit."""
    rng = np.random.default_rng(12)
    unit = "ACGTTGCA"
    seqs = []
    for _ in range(6):
        q = list((unit * 1200)[:9000])
        for p in rng.choice(len(q), size=900, replace=False):
            q[p] = "ACGT"[int(rng.integers(4))]
        seqs.append("".join(q))
    masks = projection_masks(rng, 16, 14, 2)
    say("sorted select tandem repeats")
    S = pm.Seqs(4, seqs)
    rbk, rmem, rtot = _oracle_sorted(seqs, 4, 16, 14, masks, 2)
    bk, mem, tot, st = _sorted(S, 16, 14, masks, 2)
    assert st == 0 and tot == rtot
    assert np.array_equal(bk, rbk) and np.array_equal(mem, rmem)


def test_sorted_select_capacity_and_bad_mask():
    rng = np.random.default_rng(13)
    seqs = random_sequences(rng, 8, [500] * 8, "dna")
    masks = projection_masks(rng, 14, 9, 4)
    S = pm.Seqs(4, seqs)
    rbk, rmem, (rnb, rnm) = _oracle_sorted(seqs, 4, 14, 9, masks, 2)
    assert rnb > 6 and rnm > 14
    say("sorted select truncated")
    bk, mem, tot, st = _sorted(S, 14, 9, masks, 2, cap_b=6, cap_m=14)
    assert st & pm.PM_STATUS_CAPACITY and tot == (rnb, rnm)
    assert np.array_equal(bk[:6], rbk[:6]) and np.array_equal(mem[:14], rmem[:14])
    bad = masks.copy()
    bad[1] = 0b1011
    say("sorted select bad mask")
    bk2, mem2, tot2, st2 = _sorted(S, 14, 9, bad, 2)
    assert st2 & pm.PM_STATUS_BAD_MASK
    keep = np.array([0, 2, 3])
    rbk2, rmem2, rtot2 = _oracle_sorted(seqs, 4, 14, 9, masks[keep], 2)
    assert tot2 == rtot2
    mapped = bk2.copy()
    mapped[:, 0] = np.searchsorted(keep, mapped[:, 0])
    assert np.array_equal(mapped, rbk2) and np.array_equal(mem2, rmem2)


def test_sorted_select_batch_matches_per_instance_oracle():
    rng = np.random.default_rng(14)
    insts = []
    for p in range(4):
        t = int(rng.integers(3, 9))
        lens = [int(v) for v in rng.integers(30, 900, size=t)]
        inst = planted_instance(rng, t, lens, 17, 3)
        insts.append((inst, projection_masks(rng, 17, 13, int(rng.integers(2, 5)))))
    say("sorted select batch")
    B = pm.Batch(4, 17, 13, [i.seqs for i, _ in insts], [mk for _, mk in insts])
    for nbytes, run in ((pm.pm_sort_select_batch_workspace(B), pm.bucket_sort_select_batch),
                        (pm.pm_hash_select_batch_workspace(B), pm.bucket_hash_select_batch)):
        ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        n_out = torch.zeros(2, dtype=torch.int64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        run(B, B.masks, 2, None, 0, None, 0, n_out, ws, nbytes, None)
        torch.cuda.synchronize()
        nb_, nm_ = [int(v) for v in n_out.cpu()]
        bk = torch.zeros((max(nb_, 1), 4), dtype=torch.int32, device="cuda")
        mem = torch.zeros(max(nm_, 1), dtype=torch.int32, device="cuda")
        run(B, B.masks, 2, bk, nb_, mem, nm_, n_out, ws, nbytes, st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        bk, mem = u32(bk)[:nb_], u32(mem)[:nm_]
        for p, (inst, masks) in enumerate(insts):
            f0, m = B.first_item[p], B.m[p]
            mine = bk[(bk[:, 0] >= f0) & (bk[:, 0] < f0 + m)]
            rbk, rmem, _ = _oracle_sorted(inst.seqs, 4, 17, 13, masks, 2)
            assert np.array_equal(mine[:, 0] - f0, rbk[:, 0]) and np.array_equal(mine[:, 1:3], rbk[:, 1:3])
            for a, b in zip(mine, rbk):
                assert np.array_equal(mem[a[3]:a[3] + a[2]], rmem[b[3]:b[3] + b[2]])
