"""Parity of the HIP path with the CPU oracle, element by element.

Integer outputs (codes, keys, counts, bucket lists, members, profiles) must be
bit-exact.  EM: FP64 path within 1e-12 relative of the oracle; FP32 path within
1e-5 relative on J and LLR (the target of the FP32 form); consensus identical.
Inputs are seeded and synthetic.  Every case prints its name before it touches
the GPU.
"""
import sys
import zlib

import numpy as np
import pytest

import oracle
import paper_1605_06904_amd as pm
from synth import make_config, planted_instance, projection_masks, random_sequences
from tests.conftest import read_golden

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


def _bg(A, rng=None):
    if A == 4:
        return np.full(4, 0.25)
    return rng.dirichlet(np.full(20, 2.0)) if rng is not None else np.full(20, 0.05)


def _unpack(words, A, n):
    per, bits = (16, 2) if A == 4 else (6, 5)
    out = np.zeros(n, dtype=np.uint8)
    for g in range(n):
        w = int(words[g // per])
        out[g] = (w >> (32 - bits * (g % per + 1))) & ((1 << bits) - 1)
    return out


# ------------------------------------------------------------------ a1 pack
@pytest.mark.parametrize("A,alpha", [(4, "dna"), (20, "protein")])
def test_pack_matches_oracle_codes(A, alpha):
    rng = np.random.default_rng(100 + A)
    seqs = random_sequences(rng, 5, [37, 1, 64, 17, 250], alpha)
    seqs[1] = seqs[1].lower()
    say("pack", A)
    S = pm.Seqs(A, seqs)
    torch.cuda.synchronize()
    assert int(S.status.item()) == 0
    ref = oracle.Seqs(A, seqs)
    words = u32(S.packed)
    assert len(words) == pm.pm_packed_words(A, S.n_total)
    assert np.array_equal(_unpack(words, A, S.n_total), ref.codes[:S.n_total])
    per = 16 if A == 4 else 6
    assert np.all(words[(S.n_total + per - 1) // per:] == 0)


def test_pack_flags_foreign_symbols():
    say("pack bad symbol")
    S = pm.Seqs(4, ["ACGTNACGT", "ACGT"])
    torch.cuda.synchronize()
    assert int(S.status.item()) & pm.PM_STATUS_BAD_SYMBOL
    with pytest.raises(pm.PmError):
        S.check_status()


# ------------------------------------------------------------------ a3 + a4
def _hash_gpu(S, l, k, masks, keys=True, counts=True):
    m = len(masks)
    x, nb = S.nwin(l), S.alphabet ** k
    dm = torch.from_numpy(np.ascontiguousarray(masks, dtype=np.uint32).view(np.int32)).cuda()
    K = torch.full((m, x), -1, dtype=torch.int32, device="cuda") if keys else None
    N = torch.full((m, nb), -1, dtype=torch.int32, device="cuda") if counts else None
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    pm.projection_hash(S, l, k, dm, m, K, N, st)
    torch.cuda.synchronize()
    return (u32(K) if keys else None), (u32(N) if counts else None), int(st.item())


HASH_CASES = [
    # name, alphabet, t, lengths, l, k, m
    ("dna small ragged", 4, 6, [40, 33, 57, 19, 80, 26], 8, 5, 7),
    ("dna several tiles", 4, 9, [700, 1500, 333, 64, 999, 1200, 41, 512, 2048], 15, 7, 11),
    ("dna l=32 k=16 keys", 4, 3, [64, 40, 33], 32, 11, 3),
    ("dna u32 histogram x>=65536", 4, 40, [1700] * 40, 12, 6, 3),
    ("dna sliced k=9", 4, 10, [900] * 10, 21, 9, 4),
    ("dna k=8 two slices of a whole-trial histogram", 4, 8, [500] * 8, 12, 8, 3),
    ("protein k=3", 20, 7, [120, 31, 77, 64, 200, 23, 50], 10, 3, 5),
    ("protein sliced k=4", 20, 12, [400] * 12, 20, 4, 3),
    ("dna k=1", 4, 3, [10, 12, 9], 1, 1, 2),
]


@pytest.mark.parametrize("case", HASH_CASES, ids=[c[0] for c in HASH_CASES])
def test_hash_bit_exact(case):
    name, A, t, lens, l, k, m = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seqs = random_sequences(rng, t, lens, "dna" if A == 4 else "protein")
    masks = projection_masks(rng, l, k, m)
    say("hash", name)
    S = pm.Seqs(A, seqs)
    counts_on = A ** k <= (1 << 24) and not (A == 4 and k > 12)
    K, N, st = _hash_gpu(S, l, k, masks, counts=counts_on)
    assert st == 0
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks, counts=counts_on)
    assert np.array_equal(K, RK)
    if counts_on:
        assert np.array_equal(N, RN)
        assert np.all(N.sum(axis=1, dtype=np.int64) == S.nwin(l))


def test_hash_outputs_one_at_a_time():
    rng = np.random.default_rng(7)
    seqs = random_sequences(rng, 4, [300, 200, 250, 90], "dna")
    masks = projection_masks(rng, 14, 6, 5)
    say("hash keys-only / counts-only")
    S = pm.Seqs(4, seqs)
    K, _, _ = _hash_gpu(S, 14, 6, masks, counts=False)
    _, N, _ = _hash_gpu(S, 14, 6, masks, keys=False)
    RK, RN = oracle.hash_trials(oracle.Seqs(4, seqs), 14, 6, masks)
    assert np.array_equal(K, RK) and np.array_equal(N, RN)


def test_hash_bad_mask_sets_status_and_skips_trial():
    rng = np.random.default_rng(8)
    seqs = random_sequences(rng, 3, 100, "dna")
    masks = projection_masks(rng, 10, 4, 3)
    masks[1] = 0b1111100000  # five kept positions, k = 4
    say("hash bad mask")
    S = pm.Seqs(4, seqs)
    K, N, st = _hash_gpu(S, 10, 4, masks)
    assert st & pm.PM_STATUS_BAD_MASK
    RK, RN = oracle.hash_trials(oracle.Seqs(4, seqs), 10, 4, masks[[0, 2]])
    assert np.array_equal(K[[0, 2]], RK) and np.array_equal(N[[0, 2]], RN)
    assert np.all(K[1] == 0xFFFFFFFF) and np.all(N[1] == 0xFFFFFFFF)


def test_hash_degenerate_single_bucket():
    """Poly-A input: every l-mer lands in one bucket (all lanes of every wave
    collide on one bin)."""
    seqs = ["A" * 3000] * 8
    masks = projection_masks(np.random.default_rng(9), 11, 5, 2)
    say("hash poly-A")
    S = pm.Seqs(4, seqs)
    K, N, st = _hash_gpu(S, 11, 5, masks)
    x = S.nwin(11)
    assert np.all(K == 0) and np.all(N[:, 0] == x) and np.all(N[:, 1:] == 0)


@pytest.mark.parametrize("k,l,extra", [(3, 7, 0), (9, 12, 6), (8, 11, 3)],
                         ids=["one slice", "k=9 several slices", "k=8 two slices"])
def test_hash_count_past_u16_is_recounted(k, l, extra):
    """More than 65 535 windows share one key (poly-A, x >= 65 536): the LDS
    count of that bin wraps its 16 bits, so the slice holding it is counted
    again in u32; every count bit-exact against the oracle, beside random
    sequences whose keys fill the other bins and slices."""
    rng = np.random.default_rng(100 + k)
    seqs = ["A" * 40000, "A" * 36000] + random_sequences(rng, extra, [3000] * extra, "dna")
    masks = projection_masks(rng, l, k, 2)
    say(f"hash u16 wrap k={k}")
    S = pm.Seqs(4, seqs)
    K, N, st = _hash_gpu(S, l, k, masks)
    assert st == 0
    RK, RN = oracle.hash_trials(oracle.Seqs(4, seqs), l, k, masks)
    assert np.array_equal(K, RK) and np.array_equal(N, RN)
    assert N[:, 0].min() > 65535


NARROW_CASES = [
    # name, alphabet, l, k, runs: (letter, windows) of one-letter sequences
    ("u4 highest count 15", 4, 12, 9, [("C", 15), ("T", 7)]),
    ("u4 count 16 wraps", 4, 12, 9, [("C", 15), ("T", 16), ("G", 40)]),
    ("u4 protein count 17 wraps", 20, 10, 4, [("A", 17), ("W", 15)]),
    ("u8 counts 255 and 256", 4, 11, 8, [("C", 255), ("A", 256)]),
]


@pytest.mark.parametrize("case", NARROW_CASES, ids=[c[0] for c in NARROW_CASES])
def test_hash_narrow_counters_wrap_and_recount(case):
    """Count tables of 4- and 8-bit counters (chosen for |Sigma|^k too large
    for wider ones: DNA k = 9 and protein k = 4 take 4 bits, DNA k = 8 takes 8
    on a device with 160 KB of LDS per workgroup).  A one-letter sequence of
    c windows puts c windows on one key under every mask, so counts sit just
    below and at the counter's limit; a slice where one wrapped is counted
    again in u32.  Every count bit-exact against the oracle, beside random
    sequences that fill the other bins."""
    name, A, l, k, runs = case
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    alpha = "dna" if A == 4 else "protein"
    seqs = random_sequences(rng, 8, [2500] * 8, alpha) + [ch * (l + c - 1) for ch, c in runs]
    masks = projection_masks(rng, l, k, 3)
    say("hash narrow counters", name)
    S = pm.Seqs(A, seqs)
    K, N, st = _hash_gpu(S, l, k, masks)
    assert st == 0
    RK, RN = oracle.hash_trials(oracle.Seqs(A, seqs), l, k, masks)
    assert np.array_equal(K, RK) and np.array_equal(N, RN)
    assert RN.max() >= max(c for _, c in runs)


# ------------------------------------------------------------------ a5, a6
def _select_gpu(S, l, k, s, K, N, cap_b=None, cap_m=None):
    m = K.shape[0]
    dK = torch.from_numpy(K.view(np.int32)).cuda()
    dN = torch.from_numpy(N.view(np.int32)).cuda()
    nout = torch.zeros(2, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    if cap_b is None:
        ws = torch.zeros(pm.pm_select_workspace(S.alphabet, k, m, 0) // 4 + 1, dtype=torch.int32, device="cuda")
        pm.bucket_select(S, l, k, dK, dN, m, s, None, 0, None, 0, nout, ws, ws.numel() * 4, st)
        torch.cuda.synchronize()
        cap_b, cap_m = [int(v) for v in nout.cpu()]
    bk = torch.full((max(cap_b, 1), 4), -1, dtype=torch.int32, device="cuda")
    mem = torch.full((max(cap_m, 1),), -1, dtype=torch.int32, device="cuda")
    ws = torch.zeros(pm.pm_select_workspace(S.alphabet, k, m, cap_b) // 4 + 1, dtype=torch.int32, device="cuda")
    st.zero_()
    pm.bucket_select(S, l, k, dK, dN, m, s, bk, cap_b, mem, cap_m, nout, ws, ws.numel() * 4, st)
    torch.cuda.synchronize()
    nb_, nm_ = [int(v) for v in nout.cpu()]
    return bk, mem, nout, (nb_, nm_), int(st.item()), cap_b, cap_m


SELECT_CASES = [
    ("toy", None, 8, 5, 4),
    ("dna ragged s=2", 4, 12, 6, 2),
    ("dna s=1 every key", 4, 9, 4, 1),
    ("dna s=0 same as s=1", 4, 9, 4, 0),
    ("protein s=2", 20, 9, 2, 2),
    ("dna k=1 buckets of more than 128 members", 4, 8, 1, 3),
]


def _select_inputs(name, A, l, k):
    if name == "toy":
        seqs = [r[0] for r in read_golden("fig1_sequences.txt")]
        return 4, seqs, np.array([0b1100111], dtype=np.uint32)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    seqs = random_sequences(rng, 7, [90, 130, 61, 200, 45, 77, 150], "dna" if A == 4 else "protein")
    return A, seqs, projection_masks(rng, l, k, 6)


@pytest.mark.parametrize("case", SELECT_CASES, ids=[c[0] for c in SELECT_CASES])
def test_select_profile_theta0_bit_exact(case):
    name, A, l, k, s = case
    A, seqs, masks = _select_inputs(name, A, l, k)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, l, k, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, l, k, RK, RN, s)
    if "more than 128" in name:
        assert rbk[:, 2].min() > 128  # profiles read members 64 at a time
    say("select", name)
    S = pm.Seqs(A, seqs)
    bk, mem, nout, (nb_, nm_), st, cap_b, cap_m = _select_gpu(S, l, k, s, RK, RN)
    assert st == 0 and (nb_, nm_) == (rnb, rnm)
    assert np.array_equal(u32(bk)[:nb_], rbk)
    assert np.array_equal(u32(mem)[:nm_], rmem)
    # a6: profiles and theta0
    A_ = S.alphabet
    prof = torch.zeros((max(cap_b, 1), A_, l), dtype=torch.int32, device="cuda")
    pm.bucket_profile(S, l, bk, mem, cap_m, cap_b, nout, prof)
    rprof = oracle.profile(ref, l, rbk, rmem)
    bg = _bg(A_, np.random.default_rng(1))
    dbg = torch.from_numpy(bg).cuda()
    th0 = torch.zeros((max(cap_b, 1), A_, l), dtype=torch.float64, device="cuda")
    for beta in (0.0, 1.0, 2.5):
        pm.theta_init(A_, l, prof, cap_b, nout, dbg, beta, th0)
        torch.cuda.synchronize()
        assert np.array_equal(u32(prof)[:nb_], rprof)
        np.testing.assert_allclose(th0.cpu().numpy()[:nb_], oracle.theta0(rprof, bg, beta), rtol=1e-15, atol=0)


def test_select_truncates_to_capacity_and_reports():
    A, seqs, masks = _select_inputs("dna ragged s=2", 4, 12, 6)
    ref = oracle.Seqs(A, seqs)
    RK, RN = oracle.hash_trials(ref, 12, 6, masks)
    rbk, rmem, (rnb, rnm), _ = oracle.select(ref, 12, 6, RK, RN, 2)
    assert rnb > 5 and rnm > 11
    say("select truncated")
    S = pm.Seqs(A, seqs)
    bk, mem, nout, (nb_, nm_), st, _, _ = _select_gpu(S, 12, 6, 2, RK, RN, cap_b=5, cap_m=11)
    assert st & pm.PM_STATUS_CAPACITY and (nb_, nm_) == (rnb, rnm)
    assert np.array_equal(u32(bk)[:5], rbk[:5])
    got = u32(mem)[:11]
    # members of the buckets that were kept, up to the member capacity
    keep = rmem[:11]
    written = [i for i in range(11) if any(b[3] <= i < b[3] + b[2] for b in rbk[:5])]
    assert np.array_equal(got[written], keep[written])


# ------------------------------------------------------------------ a7 - a10
def _em_case(seed, A, t, n, l, d, nb):
    rng = np.random.default_rng(seed)
    inst = planted_instance(rng, t, n, l, d, "dna" if A == 4 else "protein",
                            dirichlet_alpha=2.0 if A == 20 else None)
    ref = oracle.Seqs(A, inst.seqs)
    bg = oracle.bg_vector(A, inst.bg)
    # models: random profiles plus one seeded at the planted sites
    th0 = np.stack([rng.dirichlet(np.ones(A) * 0.7, size=l).T for _ in range(nb)])
    th0 = 0.8 * th0 + 0.2 * bg[None, :, None]
    planted = np.zeros((A, l))
    L = oracle.letters(A)
    for x, a in zip(inst.seqs, inst.starts):
        for p in range(l):
            planted[L.index(x[a + p]), p] += 1
    th0[0] = (planted + bg[:, None]) / (t + 1)
    return inst, ref, bg, np.ascontiguousarray(th0)


def _em_gpu(S, l, th0, bg, iters, beta, precision, ws=None):
    B = th0.shape[0]
    A = S.alphabet
    d_th0 = torch.from_numpy(th0).cuda()
    d_bg = torch.from_numpy(bg).cuda()
    th = torch.zeros_like(d_th0)
    J = torch.zeros((B, iters + 1), dtype=torch.float64, device="cuda")
    LL = torch.zeros_like(J)
    sites = torch.zeros((B, S.t), dtype=torch.int32, device="cuda")
    pm.em_refine(S, l, d_th0, d_bg, B, None, iters, beta, precision, th, J, LL, sites, ws=ws)
    best = torch.zeros(1, dtype=torch.int64, device="cuda")
    cons = torch.zeros(l + 1, dtype=torch.uint8, device="cuda")
    pm.em_best(J, B, None, iters, th, A, l, best, cons)
    torch.cuda.synchronize()
    return (th.cpu().numpy(), J.cpu().numpy(), LL.cpu().numpy(), sites.cpu().numpy(),
            int(best.item()), bytes(cons.cpu().numpy()[:l]).decode())


def _same_best(got, ref, rJ, tol):
    """The winning model: the oracle's, or one whose final J ties it within the
    tolerance (several buckets often converge to the same motif)."""
    if got != ref:
        assert abs(rJ[got, -1] - rJ[ref, -1]) <= tol * max(1.0, abs(rJ[ref, -1])), (got, ref)


def _same_consensus(got, ref, theta_ref, A, tol):
    """Identical consensus, except that a column whose two largest oracle
    probabilities lie within the tolerance of the arithmetic counts as a tie
    (Sec. 2 lets ties go either way)."""
    L = oracle.letters(A)
    assert len(got) == len(ref)
    for p, (g, r) in enumerate(zip(got, ref)):
        if g != r:
            assert abs(theta_ref[L.index(g), p] - theta_ref[L.index(r), p]) <= tol, (p, g, r)


EM_CASES = [
    # name, seed, A, t, n, l, d, B, iters, beta
    ("dna small", 1, 4, 6, 90, 10, 2, 9, 5, 1.0),
    ("dna c1 shape", 2, 4, 20, 600, 15, 4, 6, 5, 1.0),
    ("dna ragged beta 0.3", 3, 4, 11, None, 13, 3, 5, 7, 0.3),
    ("protein", 4, 20, 8, 150, 12, 3, 4, 4, 1.0),
    ("dna l=32", 5, 4, 5, 120, 32, 6, 3, 3, 2.0),
    # odd numbers of 4-position tiles: the split form's last k-block holds the
    # hi and lo halves of its positions in one MFMA (two positions at l = 18,
    # four at l = 20, one at l = 9); more models than one group of 16
    ("dna l=18", 6, 4, 8, 200, 18, 6, 20, 4, 1.0),
    ("dna l=20", 7, 4, 7, 160, 20, 5, 37, 3, 0.5),
    ("dna l=9", 8, 4, 6, 110, 9, 2, 17, 4, 1.0),
]


PREC_NAMES = {pm.PM_FP64: "fp64", pm.PM_FP32: "fp32", pm.PM_F16X2: "f16x2"}


def _sites_valid(sites, rsites, rth, ref, l, bg, tol):
    """Sites equal the oracle's, except where the oracle's best score and the
    score at the chosen start tie within the tolerance."""
    if np.array_equal(sites, rsites):
        return
    L = ref.lens - l + 1
    cum = np.concatenate([[0], np.cumsum(L)])
    for b in range(len(sites)):
        if np.array_equal(sites[b], rsites[b]):
            continue
        _, s, _, _ = oracle.estep(ref, l, rth[b], bg)
        for i in range(len(L)):
            seg = s[cum[i]:cum[i + 1]]
            assert 0 <= sites[b, i] < L[i]
            assert seg.max() - seg[sites[b, i]] <= tol * max(1.0, abs(seg.max())), (b, i)


@pytest.mark.parametrize("prec", [pm.PM_FP64, pm.PM_FP32, pm.PM_F16X2], ids=["fp64", "fp32", "f16x2"])
@pytest.mark.parametrize("case", EM_CASES, ids=[c[0] for c in EM_CASES])
def test_em_matches_oracle(case, prec):
    name, seed, A, t, n, l, d, B, iters, beta = case
    if prec == pm.PM_F16X2 and A != 4:
        pytest.skip("the split-FP16 matrix-core path is for DNA")
    if n is None:
        rng = np.random.default_rng(seed)
        inst = planted_instance(rng, t, list(rng.integers(l + 3, 400, size=t)), l, d)
        ref = oracle.Seqs(A, inst.seqs)
        bg = np.full(4, 0.25)
        th0 = np.ascontiguousarray(np.stack([0.7 * rng.dirichlet(np.ones(4), size=l).T + 0.075
                                              for _ in range(B)]))
    else:
        inst, ref, bg, th0 = _em_case(seed, A, t, n, l, d, B)
    rth, rJ, rLL, rsites = oracle.em(ref, l, th0, bg, iters, beta)
    rbest, rcons = oracle.best(rJ, rth)
    say("em", name, PREC_NAMES[prec])
    S = pm.Seqs(A, inst.seqs)
    th, J, LL, sites, best, cons = _em_gpu(S, l, th0, bg, iters, beta, prec)
    tol = 1e-12 if prec == pm.PM_FP64 else 1e-5
    th_tol = 1e-12 if prec == pm.PM_FP64 else 2e-5
    np.testing.assert_allclose(J, rJ, rtol=tol, atol=tol * np.abs(rJ).max())
    np.testing.assert_allclose(LL, rLL, rtol=tol, atol=tol * np.abs(rLL).max())
    np.testing.assert_allclose(th, rth, rtol=0, atol=th_tol)
    assert np.all(np.diff(J, axis=1) >= -tol * np.abs(J).max())
    _same_best(best, rbest, rJ, tol)
    _same_consensus(cons, oracle.best(rJ[best:best + 1], rth[best:best + 1])[1], rth[best], A, th_tol)
    if prec == pm.PM_FP64:
        assert np.array_equal(sites, rsites)
    else:
        _sites_valid(sites, rsites, rth, ref, l, bg, 1e-5)


F16_CASES = EM_CASES + [
    # the protein matrix-core kernel at the (20,6) workload's shape (20 l = 400
    # contraction rows in 13 steps of 32, counts of all 26 row tiles in
    # registers), at l = 22 (the largest single sweep) and past it, where the
    # count rows are split over two sweeps (l = 23, 24); B = 70 spans two
    # workgroups of 64 models with a ragged tail
    ("protein l=20 c4 shape", 41, 20, 9, 160, 20, 6, 70, 3, 1.0),
    ("protein l=22", 42, 20, 5, 120, 22, 6, 20, 2, 1.0),
    ("protein l=23 two sweeps", 43, 20, 6, 140, 23, 6, 20, 3, 1.0),
    ("protein l=24 two sweeps", 44, 20, 7, 100, 24, 7, 70, 2, 0.5),
]


def _fp16_eval_bound(theta, bg, t):
    """Largest error of an objective that the single-FP16 form evaluates at a
    model theta it holds exactly (FP64): each log-odds entry W = ln(theta/bg)
    is rounded once to FP16 (relative error at most 2^-11, plus 2^-24 for the
    FP32 step before it), the l products are exact and summed in FP32, so a
    window's score moves by at most (2^-11 + 2^-22) sum_p max_c |W_cp|; the
    log-sum-exp of a sequence is 1-Lipschitz in its scores, and its FP32
    exponentials carry 2^-22 relative error each, summed in FP64; t sequences
    add up."""
    W = np.log(theta) - np.log(bg)[None, :, None]
    per_window = np.abs(W).max(axis=1).sum(axis=1)
    return t * ((2.0 ** -11 + 2.0 ** -22) * per_window + 2.0 ** -21)


@pytest.mark.parametrize("case", F16_CASES, ids=[c[0] for c in F16_CASES])
def test_em_single_fp16_form_error_against_fp64(case):
    """The precision form (one FP16 value per operand; protein cases run the
    20-letter one-hot kernel) against the FP64 oracle.  What the arithmetic
    fixes is asserted: the objective of theta^0 (held exactly on both sides)
    and the objective the kernel reports for its own final model theta^I
    (returned in FP64), each within the evaluation bound of _fp16_eval_bound
    of the oracle's FP64 value at that same model; every column of theta^I on
    the simplex.  The drift of later iterates from the oracle's trajectory
    (the FP16 rounding of the posteriors feeds each M-step) has no a-priori
    bound and is stated per case, not asserted."""
    name, seed, A, t, n, l, d, B, iters, beta = case
    if n is None:
        rng = np.random.default_rng(seed)
        inst = planted_instance(rng, t, list(rng.integers(l + 3, 400, size=t)), l, d)
        ref = oracle.Seqs(A, inst.seqs)
        bg = np.full(4, 0.25)
        th0 = np.ascontiguousarray(np.stack([0.7 * rng.dirichlet(np.ones(4), size=l).T + 0.075
                                              for _ in range(B)]))
    else:
        inst, ref, bg, th0 = _em_case(seed, A, t, n, l, d, B)
    rth, rJ, rLL, rsites = oracle.em(ref, l, th0, bg, iters, beta)
    say("em single fp16", name)
    S = pm.Seqs(A, inst.seqs)
    th, J, LL, sites, best, cons = _em_gpu(S, l, th0, bg, iters, beta, pm.PM_F16)
    assert np.all(np.isfinite(J)) and np.all(th > 0)
    np.testing.assert_allclose(th.sum(axis=1), 1.0, rtol=0, atol=1e-12)
    # J(theta^0): theta^0 is exact on both sides
    b0 = _fp16_eval_bound(th0, bg, t)
    assert np.all(np.abs(J[:, 0] - rJ[:, 0]) <= b0), (np.abs(J[:, 0] - rJ[:, 0]) / b0).max()
    # J(theta^I) at the kernel's own theta^I, against the oracle's FP64 value there
    _, eJ, eLL, _ = oracle.em(ref, l, np.ascontiguousarray(th), bg, 0, beta)
    bI = _fp16_eval_bound(th, bg, t)
    assert np.all(np.abs(J[:, -1] - eJ[:, 0]) <= bI), (np.abs(J[:, -1] - eJ[:, 0]) / bI).max()
    assert np.all(np.abs(LL[:, -1] - eLL[:, 0]) <= bI)
    rel = np.abs(J - rJ) / np.maximum(1.0, np.abs(rJ))
    print(f"[precision] {name}: J(theta^0) error {np.abs(J[:, 0] - rJ[:, 0]).max():.3e} "
          f"(bound {b0.min():.3e}..{b0.max():.3e}); J(theta^I) evaluation error "
          f"{np.abs(J[:, -1] - eJ[:, 0]).max():.3e} (bound {bI.min():.3e}..{bI.max():.3e}); "
          f"trajectory drift max |dJ|/|J| = {rel.max():.3e}, mean = {rel.mean():.3e}, "
          f"max |dtheta| = {np.abs(th - rth).max():.3e}", flush=True)


def test_em_theta_equal_background_gives_zero():
    rng = np.random.default_rng(11)
    seqs = random_sequences(rng, 5, 60, "dna")
    bg = np.array([0.1, 0.2, 0.3, 0.4])
    th0 = np.repeat(bg[None, :, None], 8, axis=2).repeat(2, axis=0)
    say("em theta = bg")
    S = pm.Seqs(4, seqs)
    for prec in (pm.PM_FP64, pm.PM_FP32, pm.PM_F16X2):
        th, J, LL, sites, best, cons = _em_gpu(S, 8, np.ascontiguousarray(th0), bg, 2, 0.0, prec)
        assert np.all(np.abs(LL[:, 0]) <= (0.0 if prec != pm.PM_F16X2 else 1e-9))



def _first_largest(Jf):
    """The winning index by definition: the largest final objective, the
    smallest index among equals, NaN skipped, -1 when nothing is left."""
    ok = ~np.isnan(Jf)
    if not ok.any():
        return -1
    return int(np.flatnonzero(ok & (Jf == Jf[ok].max()))[0])


BEST_CASES = [
    # name, buckets, valid buckets (None: all), final-J pattern
    ("empty", 0, None, "rand"),
    ("one", 1, None, "rand"),
    ("ragged tail", 8 * 1024 + 37, None, "rand"),
    ("ties over the whole range", 100_003, None, "ties"),
    ("nan and -inf", 5_000, None, "nan"),
    ("all nan", 300, None, "allnan"),
    ("all -inf", 300, None, "allninf"),
    ("n_dev below capacity", 20_000, 12_345, "ties"),
    ("(18,6) bucket count", 89_296, None, "ties"),
]


@pytest.mark.parametrize("case", BEST_CASES, ids=[c[0] for c in BEST_CASES])
def test_em_best_is_the_first_largest_final_objective(case):
    name, B, nvalid, pattern = case
    A, l, iters = 4, 12, 3
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    Jf = {"rand": lambda: rng.standard_normal(B),
          "ties": lambda: rng.integers(0, 40, B).astype(np.float64),
          "nan": lambda: np.where(rng.random(B) < 0.3, np.nan,
                                  np.where(rng.random(B) < 0.3, -np.inf, rng.integers(0, 9, B).astype(np.float64))),
          "allnan": lambda: np.full(B, np.nan),
          "allninf": lambda: np.full(B, -np.inf)}[pattern]()
    # earlier iterations hold larger values: only the final column may count
    J = np.concatenate([np.full((B, iters), 1e300), Jf[:, None]], axis=1)
    theta = rng.random((B, A, l))
    n = B if nvalid is None else nvalid
    ref = _first_largest(Jf[:n])
    say("em_best", name, B, n, ref)
    d_J = torch.from_numpy(np.ascontiguousarray(J)).cuda()
    d_th = torch.from_numpy(theta).cuda()
    d_n = None if nvalid is None else torch.tensor([nvalid], dtype=torch.int64, device="cuda")
    best = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    cons = torch.full((l + 1,), 0xFF, dtype=torch.uint8, device="cuda")
    pm.em_best(d_J, B, d_n, iters, d_th, A, l, best, cons)
    torch.cuda.synchronize()
    assert int(best.item()) == ref
    got = bytes(cons.cpu().numpy())
    want = ("".join("ACTG"[c] for c in theta[ref].argmax(axis=0)).encode() if ref >= 0 else bytes(l)) + b"\0"
    assert got == want


# ------------------------------------------------------------------ end to end
def _pipeline(inst, masks, cfg, precision, cap_factor=1):
    A = 4 if cfg["alphabet"] == "dna" else 20
    ref = oracle.Seqs(A, inst.seqs)
    bg = oracle.bg_vector(A, inst.bg)
    S = pm.Seqs(A, inst.seqs)
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    # size the lists with one counting pass
    P0 = pm.Pipeline(S, l, k, s, masks, iters, 1.0, precision, bg, cap_b=0, cap_m=0)
    P0.hash()
    P0.select()
    torch.cuda.synchronize()
    nb_, nm_ = [int(v) for v in P0.b.n_out.cpu()]
    del P0
    P = pm.Pipeline(S, l, k, s, masks, iters, 1.0, precision, bg, cap_b=nb_, cap_m=nm_)
    return A, ref, bg, S, P


def test_c1_full_pipeline_against_oracle():
    """The (15,4) plain workload at full size: every output against the oracle."""
    inst, masks = make_config("c1", seed=1)
    cfg = inst.meta
    A, ref, bg, S, P = _pipeline(inst, masks, cfg, pm.PM_FP64)
    say("c1 full pipeline")
    P.run()
    res = P.result()
    r = oracle.run(inst.seqs, A, cfg["l"], cfg["k"], cfg["s"], masks, cfg["iters"], 1.0, bg=bg)
    assert res["status"] == 0
    assert (res["n_buckets"], res["n_members"]) == (len(r["buckets"]), len(r["members"]))
    assert np.array_equal(u32(P.b.keys), r["keys"]) and np.array_equal(u32(P.b.counts), r["counts"])
    assert np.array_equal(u32(P.b.buckets), r["buckets"]) and np.array_equal(u32(P.b.members), r["members"])
    np.testing.assert_allclose(P.b.J.cpu().numpy(), r["J"], rtol=1e-12, atol=1e-10)
    _same_best(res["best"], r["best"], r["J"], 1e-12)
    b = res["best"]
    _same_consensus(res["consensus"], oracle.best(r["J"][b:b + 1], r["theta"][b:b + 1])[1],
                    r["theta"][b], A, 1e-12)
    assert np.array_equal(res["sites"], r["sites"][b])


def test_c2_full_size_sampled_against_oracle():
    """The (18,6) workload at full size (m = 5000) in the launch configuration
    the benchmark times: keys/counts and buckets of sampled trials bit-exact,
    FP32 EM of sampled buckets within 1e-5 of the FP64 oracle, and the
    invariants on every trial."""
    inst, masks = make_config("c2", seed=1)
    cfg = inst.meta
    A, ref, bg, S, P = _pipeline(inst, masks, cfg, pm.PM_F16X2)
    say("c2 full size", P.m, "trials", P.b.cap_b, "buckets")
    P.run()
    torch.cuda.synchronize()
    res = P.result()
    assert res["status"] == 0
    x = S.nwin(cfg["l"])
    assert torch.all(P.b.counts.sum(dim=1) == x).item()
    rng = np.random.default_rng(5)
    trials = np.sort(rng.choice(P.m, size=12, replace=False))
    RK, RN = oracle.hash_trials(ref, cfg["l"], cfg["k"], masks[trials])
    assert np.array_equal(u32(P.b.keys[trials]), RK)
    assert np.array_equal(u32(P.b.counts[trials]), RN)
    bk = u32(P.b.buckets)
    mem = u32(P.b.members)
    for i, j in enumerate(trials):
        rbk, rmem, _, _ = oracle.select(ref, cfg["l"], cfg["k"], RK[i:i + 1], RN[i:i + 1], cfg["s"])
        mine = bk[bk[:, 0] == j]
        assert np.array_equal(mine[:, 1:3], rbk[:, 1:3])
        for a, b in zip(mine, rbk):
            assert np.array_equal(mem[a[3]:a[3] + a[2]], rmem[b[3]:b[3] + b[2]])
    # EM on a sample of buckets, FP32 against the FP64 oracle
    sel = np.sort(rng.choice(len(bk), size=24, replace=False))
    th0 = P.b.theta0.cpu().numpy()[sel]
    rprof = oracle.profile(ref, cfg["l"], bk[sel], mem)
    np.testing.assert_allclose(th0, oracle.theta0(rprof, bg, 1.0), rtol=1e-15)
    rth, rJ, rLL, rsites = oracle.em(ref, cfg["l"], th0, bg, cfg["iters"], 1.0)
    np.testing.assert_allclose(P.b.J.cpu().numpy()[sel], rJ, rtol=1e-5, atol=1e-5 * np.abs(rJ).max())
    J = P.b.J.cpu().numpy()[: len(bk)]
    assert np.all(np.diff(J, axis=1) >= -1e-5 * np.abs(J).max())


def _full_size_sampled(name, precision, n_trials, n_buckets, seed):
    """Hash and selection of a whole configuration at full size, sampled trials
    bit-exact against the oracle, Sum counts = x on every trial; EM of sampled
    buckets (theta^0 rows of the full run) against the FP64 oracle."""
    inst, masks = make_config(name, seed=seed)
    cfg = inst.meta
    A, ref, bg, S, P = _pipeline(inst, masks, cfg, precision)
    l, k, s, iters = cfg["l"], cfg["k"], cfg["s"], cfg["iters"]
    say(name, "full size", P.m, "trials", P.b.cap_b, "buckets")
    P.hash()
    P.select()
    pm.bucket_profile(S, l, P.b.buckets, P.b.members, P.b.cap_m, P.b.cap_b, P.b.n_out, P.b.profile)
    pm.theta_init(A, l, P.b.profile, P.b.cap_b, P.b.n_out, P.bg, 1.0, P.b.theta0)
    torch.cuda.synchronize()
    assert int(P.b.status.item()) == 0
    x = S.nwin(l)
    assert torch.all(P.b.counts.sum(dim=1) == x).item()
    rng = np.random.default_rng(seed)
    trials = np.sort(rng.choice(P.m, size=n_trials, replace=False))
    RK, RN = oracle.hash_trials(ref, l, k, masks[trials])
    assert np.array_equal(u32(P.b.keys[trials]), RK)
    assert np.array_equal(u32(P.b.counts[trials]), RN)
    bk = u32(P.b.buckets)
    mem = u32(P.b.members)
    for i, j in enumerate(trials):
        rbk, rmem, _, _ = oracle.select(ref, l, k, RK[i:i + 1], RN[i:i + 1], s)
        mine = bk[bk[:, 0] == j]
        assert np.array_equal(mine[:, 1:3], rbk[:, 1:3])
        for a, b in zip(mine, rbk):
            assert np.array_equal(mem[a[3]:a[3] + a[2]], rmem[b[3]:b[3] + b[2]])
    sel = np.sort(rng.choice(len(bk), size=n_buckets, replace=False))
    th0 = P.b.theta0.cpu().numpy()[sel]
    rprof = oracle.profile(ref, l, bk[sel], mem)
    np.testing.assert_allclose(th0, oracle.theta0(rprof, bg, 1.0), rtol=1e-15)
    th, J, LL, sites, best, cons = _em_gpu(S, l, np.ascontiguousarray(th0), bg, iters, 1.0, precision)
    rth, rJ, rLL, rsites = oracle.em(ref, l, th0, bg, iters, 1.0)
    np.testing.assert_allclose(J, rJ, rtol=1e-5, atol=1e-5 * np.abs(rJ).max())
    assert np.all(np.diff(J, axis=1) >= -1e-5 * np.abs(J).max())


def test_c4_protein_full_size_sampled_against_oracle():
    """(20,6) protein, Dirichlet background, t=30, n=1000, k=4 (160 000 bins,
    key-range slices), m=2000; EM sample on the FP32 path."""
    _full_size_sampled("c4", pm.PM_FP32, n_trials=6, n_buckets=16, seed=4)


def test_c5_full_size_sampled_against_oracle():
    """(21,7) DNA, t=50, n=2000 (x = 99 000: u32 histogram in key-range slices),
    k=9, m=10000; EM sample on the split-FP16 matrix cores."""
    _full_size_sampled("c5", pm.PM_F16X2, n_trials=4, n_buckets=16, seed=5)


@pytest.mark.parametrize("case", [c for c in EM_CASES if c[2] == 4], ids=[c[0] for c in EM_CASES if c[2] == 4])
def test_em_precomputed_tables_match_the_in_kernel_build(case):
    """The DNA matrix-core forms read the one-hot tables of every window pair
    from the workspace (built once per call) or, without one, build them inside
    the EM kernel: the same tables, so the same bits, for ragged lengths,
    sequence tails and a workspace padded with garbage past its size."""
    name, seed, A, t, n, l, d, B, iters, beta = case
    if n is None:
        rng = np.random.default_rng(seed)
        inst = planted_instance(rng, t, list(rng.integers(l + 3, 400, size=t)), l, d)
        th0 = np.ascontiguousarray(np.stack([0.7 * rng.dirichlet(np.ones(4), size=l).T + 0.075
                                              for _ in range(B)]))
        bg = np.full(4, 0.25)
    else:
        inst, ref, bg, th0 = _em_case(seed, A, t, n, l, d, B)
    say("em tables", name)
    S = pm.Seqs(A, inst.seqs)
    for prec in (pm.PM_F16X2, pm.PM_F16):
        nbytes = pm.pm_em_workspace(S, l, prec)
        assert nbytes > 0
        ws = torch.full((nbytes + 4096,), 0x7F, dtype=torch.uint8, device="cuda")
        pre = _em_gpu(S, l, th0, bg, iters, beta, prec, ws=ws)
        built = _em_gpu(S, l, th0, bg, iters, beta, prec, ws=False)
        for x, y in zip(pre[:4], built[:4]):
            assert np.array_equal(x, y), (name, prec)
        assert pre[4:] == built[4:]


def test_em_instance_too_large_to_stage_builds_from_global_memory():
    """An instance of 150 000 symbols (more than the 32 KB of packed words the
    kernel stages in LDS): without a workspace the matrix-core EM builds the
    one-hot tables from the packed words in global memory (reads clamped to the
    buffer), with one it copies the precomputed tables; both give the same
    bits, within 1e-5 of the oracle."""
    inst, ref, bg, th0 = _em_case(31, 4, 5, 30000, 12, 3, 6)
    say("em large instance")
    S = pm.Seqs(4, inst.seqs)
    assert pm.pm_packed_words(4, S.n_total) * 4 > 32 * 1024
    iters = 2
    rth, rJ, rLL, rsites = oracle.em(ref, 12, th0, bg, iters, 1.0)
    pre = _em_gpu(S, 12, th0, bg, iters, 1.0, pm.PM_F16X2)
    built = _em_gpu(S, 12, th0, bg, iters, 1.0, pm.PM_F16X2, ws=False)
    for x, y in zip(pre[:4], built[:4]):
        assert np.array_equal(x, y)
    np.testing.assert_allclose(pre[1], rJ, rtol=1e-5, atol=1e-5 * np.abs(rJ).max())
    np.testing.assert_allclose(pre[0], rth, rtol=0, atol=2e-5)


def test_em_autotune_records_a_shape_and_keeps_results():
    """The tile-shape autotuner times the candidates on the caller's models and
    records the fastest; every shape gives bit-identical results (the shapes
    change how many models share a wave's one-hot operands and how many window
    pairs share a barrier, never the order of any model's arithmetic)."""
    inst, ref, bg, th0 = _em_case(21, 4, 12, 300, 18, 6, 200)
    say("em autotune")
    S = pm.Seqs(4, inst.seqs)
    for prec in (pm.PM_F16X2, pm.PM_F16):
        pm.em_set_tuning(18, prec, 11)
        base = _em_gpu(S, 18, th0, bg, 3, 1.0, prec)
        for shape in (12, 14, 21, 22, 24):
            pm.em_set_tuning(18, prec, shape)
            assert pm.em_tuning(18, prec) == shape
            got = _em_gpu(S, 18, th0, bg, 3, 1.0, prec)
            assert all(np.array_equal(x, y) for x, y in zip(base[:4], got[:4])), shape
        d_th0 = torch.from_numpy(th0).cuda()
        th = torch.zeros_like(d_th0)
        J = torch.zeros((th0.shape[0], 4), dtype=torch.float64, device="cuda")
        choice = pm.em_autotune(S, 18, d_th0, torch.from_numpy(bg).cuda(), th0.shape[0], 3, 1.0, prec, th, J)
        assert choice in (11, 12, 14, 21, 22, 24) and pm.em_tuning(18, prec) == choice
        after = _em_gpu(S, 18, th0, bg, 3, 1.0, prec)
        assert np.array_equal(base[1], after[1]) and np.array_equal(base[0], after[0])
    # G = 2 is limited to l <= 24; the default shape stays valid everywhere
    with pytest.raises(pm.PmError):
        pm.em_set_tuning(28, pm.PM_F16X2, 21)
    with pytest.raises(pm.PmError):
        pm.em_tuning(18, pm.PM_FP64)
