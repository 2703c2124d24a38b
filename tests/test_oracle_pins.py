"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here touches the GPU.  Each test names the passage of the paper it
rests on.  The brute-force side (``oracle.brute``) works on letters, not codes,
so a mistake in the C oracle cannot cancel against itself.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import planted_instance, projection_masks, random_sequences
from tests.conftest import read_golden

DNA = 4
PROT = 20


def _mask(positions_0based):
    m = 0
    for p in positions_0based:
        m |= 1 << p
    return m


def _key_to_string(key, k, A):
    L = oracle.letters(A)
    out = []
    for _ in range(k):
        out.append(L[key % A])
        key //= A
    return "".join(reversed(out))


# ---------------------------------------------------------------- Sec. 6 keys
def test_key_examples_printed():
    """Sec. 6: "AAAAAAAA" -> 0 and "AAAAAAACG" -> 7 under A0 C1 T2 G3."""
    for word, val in read_golden("key_examples.txt"):
        S = oracle.Seqs(DNA, [word])
        l = len(word)
        keys, counts = oracle.hash_trials(S, l, l, np.array([(1 << l) - 1]), counts=False)
        assert int(keys[0, 0]) == int(val)


def test_letters_in_code_order():
    assert oracle.letters(DNA) == "ACTG"
    assert len(set(oracle.letters(PROT))) == 20


def test_hash_rejects_bad_mask():
    S = oracle.Seqs(DNA, ["ACGTACGTAC"])
    with pytest.raises(ValueError):
        oracle.hash_trials(S, 4, 3, np.array([0b1111]))
    with pytest.raises(ValueError):
        oracle.hash_trials(S, 4, 2, np.array([0b10001]))


def test_encode_rejects_foreign_symbol():
    with pytest.raises(ValueError):
        oracle.Seqs(DNA, ["ACGTN"])
    with pytest.raises(ValueError):
        oracle.Seqs(PROT, ["ARNDB"])


# ------------------------------------------------ Fig. 1 / Fig. 2 / Example 1
TOY_MASK_READ = _mask([0, 1, 2, 5, 6])     # 1-based {1,2,3,6,7}
TOY_MASK_PRINTED = _mask([0, 1, 2, 4, 5])  # 1-based {1,2,3,5,6} as printed


def test_fig1_toy_buckets(fig1):
    """Example 1: bucket "ATGAC" is enriched (s = 4) with exactly the seven
    l-mers of Fig. 2.  Reading: the printed positions 1,2,3,5,6 do not produce
    that bucket; positions 1,2,3,6,7 do (checked below)."""
    l, k, s = 8, 5, 4
    g = read_golden("fig2_alignment.txt")
    starts = [int(v) - 1 for v in next(r for r in g if r[0] == "starts_1based")[1:]]
    S = oracle.Seqs(DNA, fig1)
    keys, counts = oracle.hash_trials(S, l, k, np.array([TOY_MASK_READ]))
    assert counts.sum() == 7 * 33
    bk, mem, (nb, nm), rc = oracle.select(S, l, k, keys, counts, s)
    assert rc == 0
    names = [_key_to_string(int(b[1]), k, DNA) for b in bk]
    assert "ATGAC" in names
    b = bk[names.index("ATGAC")]
    assert int(b[2]) == 7
    sites = [S.window_site(l, int(w)) for w in mem[b[3]:b[3] + b[2]]]
    assert sites == list(enumerate(starts))
    # brute force (letters, no integers): the same enriched set
    sizes = brute.bucket_sizes(fig1, l, TOY_MASK_READ)
    assert sorted(names) == sorted(w for w, c in sizes.items() if c >= s)
    # the printed positions do not give an "ATGAC" bucket of seven
    printed = brute.bucket_sizes(fig1, l, TOY_MASK_PRINTED)
    assert printed.get("ATGAC", 0) != 7


def test_fig2_profile_consensus_score(fig1):
    """Fig. 2 profile, consensus ATGCAACT and Score 53 (Sec. 2)."""
    g = {r[0] + (r[1] if r[0] == "profile" else ""): r for r in read_golden("fig2_alignment.txt")}
    l = 8
    starts = [int(v) - 1 for v in g["starts_1based"][1:]]
    S = oracle.Seqs(DNA, fig1)
    L = np.array([len(x) - l + 1 for x in fig1])
    cum = np.concatenate([[0], np.cumsum(L)])
    members = np.array([cum[i] + a for i, a in enumerate(starts)], dtype=np.uint32)
    bk = np.array([[0, 0, len(members), 0]], dtype=np.uint32)
    prof = oracle.profile(S, l, bk, members)[0]
    letters = oracle.letters(DNA)
    for ch in "ATCG":
        assert list(prof[letters.index(ch)]) == [int(v) for v in g["profile" + ch][2:]]
    rows = [fig1[i][a:a + l] for i, a in enumerate(starts)]
    assert rows == g["rows"][1:]
    assert brute.score(rows, "ACGT") == int(g["score"][1]) == 53
    th0 = oracle.theta0(prof[None], np.full(4, 0.25), 0.0)
    _, cons = oracle.best(np.zeros((1, 1)), th0)
    assert cons == g["consensus"][1]
    # Score bounds l*t (Sec. 2)
    assert brute.score(rows, "ACGT") <= l * len(rows)


def test_fig4_theta0(fig1):
    """Fig. 4: theta^0 of the ATGAC bucket at two decimals.  The caption's
    "Expectation = 8.58" (sum of column maxima) is inconsistent with its own
    table; the sum is 53/7 = 7.571 (five 1.00 and three 6/7)."""
    l = 8
    g = read_golden("fig4_theta0.txt")
    starts = [7, 18, 2, 4, 30, 26, 14]
    S = oracle.Seqs(DNA, fig1)
    cum = np.concatenate([[0], np.cumsum([len(x) - l + 1 for x in fig1])])
    members = np.array([cum[i] + a for i, a in enumerate(starts)], dtype=np.uint32)
    prof = oracle.profile(S, l, np.array([[0, 0, 7, 0]], dtype=np.uint32), members)
    th0 = oracle.theta0(prof, np.full(4, 0.25), 0.0)[0]
    letters = oracle.letters(DNA)
    for r in g:
        if r[0] != "theta":
            continue
        row = th0[letters.index(r[1])]
        assert float(r[2]) == 0.25
        assert [f"{v:.2f}" for v in row] == r[3:]
    assert math.isclose(th0.max(axis=0).sum(), 53 / 7, rel_tol=1e-12)


def test_toy_em_converges_to_printed_consensus(fig1):
    """Example 1: refinement of the planted bucket returns ATGCAACT; the
    sites are Fig. 2's start vector; the other enriched bucket loses."""
    l, k, s = 8, 5, 4
    bg = np.full(4, 0.25)
    for beta in (0.1, 1.0, 4.0):
        r = oracle.run(fig1, DNA, l, k, s, np.array([TOY_MASK_READ]), iters=5, beta=beta, bg=bg)
        assert r["consensus"] == "ATGCAACT"
        assert list(r["sites"][r["best"]]) == [7, 18, 2, 4, 30, 26, 14]
        assert np.all(np.diff(r["J"], axis=1) >= -1e-12)


# ------------------------------------------------ hashing vs brute force
@pytest.mark.parametrize("A,alpha", [(DNA, "dna"), (PROT, "protein")])
def test_counts_match_pairwise_and_dict(A, alpha):
    """Alg. 2 step 2(c) and Sec. 5.2: histogram counts (PROJECTION1) equal the
    all-pairs comparison counts (PROJECTION2) and a dictionary of projected
    strings, window by window; sum of counts = x."""
    rng = np.random.default_rng(1)
    for trial in range(4):
        lens = rng.integers(9, 30, size=4)
        seqs = random_sequences(rng, 4, lens, alpha)
        l = int(rng.integers(3, 9))
        k = int(rng.integers(1, min(l, 4 if A == 20 else 6) + 1))
        masks = projection_masks(rng, l, k, 3)
        S = oracle.Seqs(A, seqs)
        keys, counts = oracle.hash_trials(S, l, k, masks)
        x = S.nwin(l)
        assert keys.shape == (3, x)
        for j, mk in enumerate(masks):
            assert counts[j].sum() == x
            pw = brute.pairwise_sizes(seqs, l, int(mk))
            dic = brute.bucket_sizes(seqs, l, int(mk))
            proj = [brute.projected_string(seqs[i][a:a + l], int(mk)) for i, a in brute.windows(seqs, l)]
            for w in range(x):
                assert counts[j, keys[j, w]] == pw[w] == dic[proj[w]]
                assert _key_to_string(int(keys[j, w]), k, A) == proj[w]


def test_k_equals_l_gives_lmer_multiplicities():
    rng = np.random.default_rng(2)
    seqs = random_sequences(rng, 3, 40, "dna")
    l = 6
    S = oracle.Seqs(DNA, seqs)
    keys, counts = oracle.hash_trials(S, l, l, np.array([(1 << l) - 1]))
    dic = brute.bucket_sizes(seqs, l, (1 << l) - 1)
    for w, st in zip(keys[0], (s[a:a + l] for s in seqs for a in range(len(s) - l + 1))):
        assert counts[0, w] == dic[st]


def test_select_matches_brute():
    """Alg. 2 step 3: enriched buckets (size >= s), ordered by (trial, key),
    members in window order; s = 1 lists every distinct key."""
    rng = np.random.default_rng(3)
    seqs = random_sequences(rng, 5, [20, 25, 18, 30, 22], "dna")
    l, k = 7, 3
    masks = projection_masks(rng, l, k, 4)
    S = oracle.Seqs(DNA, seqs)
    keys, counts = oracle.hash_trials(S, l, k, masks)
    win = brute.windows(seqs, l)
    for s in (1, 2, 3, 5):
        bk, mem, (nb, nm), rc = oracle.select(S, l, k, keys, counts, s)
        exp = []
        for j, mk in enumerate(masks):
            groups = {}
            for w, (i, a) in enumerate(win):
                groups.setdefault(brute.projected_string(seqs[i][a:a + l], int(mk)), []).append(w)
            for name in sorted(groups, key=lambda z: int("".join(str("ACTG".index(c)) for c in z), 4)):
                if len(groups[name]) >= s:
                    exp.append((j, name, groups[name]))
        assert nb == len(exp)
        assert nm == sum(len(e[2]) for e in exp)
        for b, (j, name, ws) in zip(bk, exp):
            assert int(b[0]) == j and _key_to_string(int(b[1]), k, DNA) == name
            assert list(mem[b[3]:b[3] + b[2]]) == ws
        if s == 1:
            assert nb == sum(len(np.unique(keys[j])) for j in range(len(masks)))


def _brute_enriched(seqs, l, masks, s, A):
    """Enriched buckets by grouping the projected strings themselves (letters),
    ordered by trial, then by the base-|Sigma| value of the string (digit of a
    letter = its place in the code order), members in window order."""
    L = oracle.letters(A)
    win = brute.windows(seqs, l)
    exp = []
    for j, mk in enumerate(masks):
        groups = {}
        for w, (i, a) in enumerate(win):
            groups.setdefault(brute.projected_string(seqs[i][a:a + l], int(mk)), []).append(w)
        def val(z):
            v = 0
            for c in z:
                v = v * A + L.index(c)
            return v
        for name in sorted(groups, key=val):
            if len(groups[name]) >= s:
                exp.append((j, name, groups[name]))
    return exp


@pytest.mark.parametrize("A,alpha,l,k", [(DNA, "dna", 16, 14), (DNA, "dna", 18, 16), (PROT, "protein", 9, 6),
                                         (PROT, "protein", 10, 7)])
def test_select_sorted_matches_brute_large_k(A, alpha, l, k):
    """Alg. 2 step 3 without a count table (|Sigma|^k of 2^28 - 2^32 bins):
    the sorted-runs oracle against brute-force grouping of projected strings.
    Low-complexity sequences make buckets of every size at these k."""
    rng = np.random.default_rng(11 + k)
    L = oracle.letters(A)
    seqs = random_sequences(rng, 4, [40, 33, 51, 28], alpha)
    # a repeat-rich sequence over three letters, so that large k still gives
    # buckets of several l-mers
    seqs.append("".join(rng.choice(list(L[:3]), size=60)))
    seqs.append(L[1] * 45)
    masks = projection_masks(rng, l, k, 3)
    S = oracle.Seqs(A, seqs)
    keys, _ = oracle.hash_trials(S, l, k, masks, counts=False)
    for s in (1, 2, 3, 7):
        bk, mem, (nb, nm), rc = oracle.select_sorted(S, l, keys, s)
        assert rc == 0
        exp = _brute_enriched(seqs, l, masks, s, A)
        assert nb == len(exp) and nm == sum(len(e[2]) for e in exp)
        for b, (j, name, ws) in zip(bk, exp):
            assert int(b[0]) == j and _key_to_string(int(b[1]), k, A) == name
            assert int(b[2]) == len(ws)
            assert list(mem[b[3]:b[3] + b[2]]) == ws
        if s == 1:
            assert nb == sum(len(np.unique(keys[j])) for j in range(len(masks)))


def test_select_sorted_equals_count_table_select():
    """Where the count table fits, both definitions of the enriched list
    (table of counts, sorted runs) give the same bytes."""
    rng = np.random.default_rng(12)
    for A, alpha, l, k in ((DNA, "dna", 12, 7), (DNA, "dna", 9, 4), (PROT, "protein", 11, 3)):
        inst_seqs = random_sequences(rng, 6, [300, 120, 77, 410, 260, 90], alpha)
        masks = projection_masks(rng, l, k, 5)
        S = oracle.Seqs(A, inst_seqs)
        keys, counts = oracle.hash_trials(S, l, k, masks)
        for s in (1, 2, 4):
            b1, m1, n1, _ = oracle.select(S, l, k, keys, counts, s)
            b2, m2, n2, _ = oracle.select_sorted(S, l, keys, s)
            assert n1 == n2 and np.array_equal(b1, b2) and np.array_equal(m1, m2)


def test_select_capacity_truncates_and_reports():
    rng = np.random.default_rng(4)
    seqs = random_sequences(rng, 3, 30, "dna")
    S = oracle.Seqs(DNA, seqs)
    keys, counts = oracle.hash_trials(S, 6, 2, projection_masks(rng, 6, 2, 2))
    full_b, full_m, (nb, nm), rc = oracle.select(S, 6, 2, keys, counts, 2)
    assert rc == 0
    bk, mem, (nb2, nm2), rc2 = oracle.select(S, 6, 2, keys, counts, 2, cap_b=3, cap_m=5)
    assert rc2 == -3 and (nb2, nm2) == (nb, nm)
    assert np.array_equal(bk, full_b[:3]) and np.array_equal(mem, full_m[:5])


# ------------------------------------------------ EM (Sec. 5.1) vs brute force
def _rand_theta(rng, A, l):
    th = rng.dirichlet(np.ones(A), size=l).T
    return np.ascontiguousarray(th)


def _as_dict(th, A):
    L = oracle.letters(A)
    return {c: list(th[i]) for i, c in enumerate(L)}


@pytest.mark.parametrize("A,alpha", [(DNA, "dna"), (PROT, "protein")])
def test_estep_equals_explicit_products(A, alpha):
    """OOPS likelihood ratio and start posteriors by explicit products over
    whole sequences (no log-odds, no log-sum-exp) equal the oracle's E-step."""
    rng = np.random.default_rng(5)
    for _ in range(3):
        seqs = random_sequences(rng, 3, [9, 11, 10], alpha)
        l = 4
        S = oracle.Seqs(A, seqs)
        th = _rand_theta(rng, A, l)
        bg = rng.dirichlet(np.ones(A))
        llr, s, Z, lse = oracle.estep(S, l, th, bg)
        L = oracle.letters(A)
        ref = brute.oops_loglik_ratio(seqs, l, _as_dict(th, A), dict(zip(L, bg)))
        assert math.isclose(llr, ref, rel_tol=1e-11, abs_tol=1e-11)
        w0 = 0
        for seq in seqs:
            post = brute.oops_posterior(seq, l, _as_dict(th, A), dict(zip(L, bg)))
            np.testing.assert_allclose(Z[w0:w0 + len(post)], post, rtol=1e-11, atol=1e-14)
            w0 += len(post)


def test_theta_equal_bg_gives_zero_llr():
    rng = np.random.default_rng(6)
    seqs = random_sequences(rng, 4, 50, "dna")
    S = oracle.Seqs(DNA, seqs)
    bg = np.array([0.1, 0.2, 0.3, 0.4])
    th = np.repeat(bg[:, None], 9, axis=1)
    llr, s, Z, lse = oracle.estep(S, 9, th, bg)
    assert llr == 0.0 and np.all(s == 0.0)
    np.testing.assert_allclose(Z[:42], 1 / 42)


def test_mstep_maximises_expected_loglik():
    """The M-step maximises Q(theta) + beta * sum bg ln theta over the simplex
    (the EM of Dempster et al. with a Dirichlet prior): random moves that keep
    every column on the simplex never increase it."""
    rng = np.random.default_rng(7)
    seqs = random_sequences(rng, 3, [12, 10, 14], "dna")
    l, A = 4, DNA
    S = oracle.Seqs(A, seqs)
    bg = rng.dirichlet(np.ones(A))
    L = oracle.letters(A)
    th = _rand_theta(rng, A, l)
    post = [brute.oops_posterior(x, l, _as_dict(th, A), dict(zip(L, bg))) for x in seqs]
    Z = np.concatenate(post)
    for beta in (0.0, 0.5, 2.0):
        new = oracle.mstep(S, l, Z, bg, beta)
        np.testing.assert_allclose(new.sum(axis=0), 1.0, rtol=1e-13)

        def obj(t_):
            q = brute.expected_complete_loglik(seqs, l, post, _as_dict(t_, A))
            return q + beta * float(np.sum(bg[:, None] * np.log(t_)))

        base = obj(new)
        for _ in range(40):
            d = rng.normal(size=(A, l))
            d -= d.mean(axis=0)
            eps = 1e-3 * float(rng.uniform(0.1, 1.0))
            cand = new + eps * d
            if np.all(cand > 0):
                assert obj(cand) <= base + 1e-12


@pytest.mark.parametrize("beta", [0.1, 1.0, 4.0])
def test_em_objective_never_decreases(beta):
    rng = np.random.default_rng(8)
    inst = planted_instance(rng, 8, 80, 10, 2)
    S = oracle.Seqs(DNA, inst.seqs)
    bg = np.full(4, 0.25)
    th0 = np.stack([_rand_theta(rng, DNA, 10) for _ in range(6)])
    th, J, LL, sites = oracle.em(S, 10, th0, bg, 8, beta)
    assert np.all(np.diff(J, axis=1) >= -1e-10 * np.abs(J[:, 1:]).max())
    np.testing.assert_allclose(th.sum(axis=1), 1.0, rtol=1e-12)


def test_em_ml_mstep_increases_plain_llr():
    """beta = 0 in the M-step (smoothed theta^0): the plain log-likelihood ratio
    never decreases."""
    rng = np.random.default_rng(9)
    inst = planted_instance(rng, 6, 60, 8, 1)
    S = oracle.Seqs(DNA, inst.seqs)
    th0 = np.stack([_rand_theta(rng, DNA, 8) for _ in range(5)])
    th, J, LL, sites = oracle.em(S, 8, th0, np.full(4, 0.25), 6, 0.0)
    assert np.array_equal(J, LL)
    assert np.all(np.diff(LL, axis=1) >= -1e-10)


def test_sites_argmax_first_on_ties():
    S = oracle.Seqs(DNA, ["AAAAAAAA", "CACACACA"])
    bg = np.full(4, 0.25)
    th = np.full((1, 4, 2), 0.25)
    _, J, _, sites = oracle.em(S, 2, th, bg, 0, 1.0)
    assert list(sites[0]) == [0, 0]


# ------------------------------------------------ end to end, tiny brute force
def test_end_to_end_matches_exhaustive_search():
    """Tiny planted instances with exact copies (d = 0): the answer's Score
    reaches the exhaustive optimum l*t of Alg. 1, and the consensus is the
    unique (l,0) candidate."""
    rng = np.random.default_rng(10)
    done = 0
    for _ in range(10):
        inst = planted_instance(rng, 3, 9, 4, 0)
        cands = brute.ld_candidates(inst.seqs, 4, 0, "ACGT")
        assert inst.motif in cands
        if len(cands) != 1:
            continue
        masks = np.array([0b1101, 0b0111, 0b1110, 0b1011], dtype=np.uint32)
        r = oracle.run(inst.seqs, DNA, 4, 3, 3, masks, iters=5, beta=0.1, bg=np.full(4, 0.25))
        best_score, _ = brute.naive_mfp(inst.seqs, 4, "ACGT")
        rows = [inst.seqs[i][a:a + 4] for i, a in enumerate(r["sites"][r["best"]])]
        assert best_score == 4 * 3 == brute.score(rows, "ACGT")
        assert r["consensus"] == cands[0]
        done += 1
    assert done >= 3


def test_answer_score_never_beats_exhaustive():
    rng = np.random.default_rng(11)
    for _ in range(3):
        inst = planted_instance(rng, 3, 8, 4, 1)
        masks = projection_masks(rng, 4, 2, 6)
        r = oracle.run(inst.seqs, DNA, 4, 2, 2, masks, iters=3, beta=1.0, bg=np.full(4, 0.25))
        if r["best"] < 0:
            continue
        rows = [inst.seqs[i][a:a + 4] for i, a in enumerate(r["sites"][r["best"]])]
        best_score, _ = brute.naive_mfp(inst.seqs, 4, "ACGT")
        assert brute.score(rows, "ACGT") <= best_score


# ------------------------------------------------ Sec. 5 parameters, RNG
def test_p_hat_by_enumeration():
    """p_hat(l,d,k) = C(l-d,k)/C(l,k): the fraction of k-subsets of the l
    positions that avoid d fixed mutated positions."""
    for l, d, k in [(15, 4, 7), (10, 3, 4), (8, 2, 5)]:
        subsets = list(itertools.combinations(range(l), k))
        good = sum(1 for sub in subsets if not set(sub) & set(range(d)))
        assert math.isclose(oracle.p_hat(l, d, k), good / len(subsets), rel_tol=1e-15)


def test_b_below_is_binomial_cdf():
    from scipy.stats import binom
    for t, p, s in [(20, 2 / 39, 4), (50, 0.0068, 3), (30, 0.2, 3)]:
        assert math.isclose(oracle.b_below(t, p, s), binom.cdf(s - 1, t, p), rel_tol=1e-12)


def test_auto_params_rules():
    k, s, m = oracle.auto_params(15, 4, 20, 20 * 586, 4, q=0.95)
    assert k == 10 and s == 3
    B = oracle.b_below(20, oracle.p_hat(15, 4, 10), 3)
    assert m == math.ceil(math.log(0.05) / math.log(B))
    assert 1 - B ** m >= 0.95 > 1 - B ** (m - 1)
    # a mean bucket size above 1.5 makes twice the mean the threshold
    k, s, m = oracle.auto_params(8, 1, 20, 20 * 593, 4)
    assert k == 6 and s == math.ceil(2 * 20 * 593 / 4 ** 6) == 6
    with pytest.raises(ValueError):
        oracle.auto_params(8, 2, 20, 20 * 593, 4)


def test_parkmiller_published_check_value():
    """Park & Miller (1988): from seed 1, the 10000th value is 1043618065."""
    assert oracle.parkmiller(1, 10000) == 1043618065


def test_seeded_masks_are_uniform_k_subsets():
    l, k, m = 15, 7, 4000
    ms = oracle.masks_from_seed(12345, l, k, m)
    assert all(bin(int(v)).count("1") == k and int(v) < (1 << l) for v in ms)
    freq = np.array([[int(v) >> p & 1 for p in range(l)] for v in ms]).mean(axis=0)
    np.testing.assert_allclose(freq, k / l, atol=0.035)
    assert np.array_equal(ms, oracle.masks_from_seed(12345, l, k, m))
    assert not np.array_equal(ms, oracle.masks_from_seed(12346, l, k, m))


# ------------------------------------------------ theta^0 with pseudocounts
def test_theta0_pseudocounts_by_hand(fig1):
    """Sec. 5.1 / Fig. 4 with the pseudocount reading theta0 = (f + beta bg) /
    (size + beta), values worked out by hand from Fig. 2's profile (f = 7, 6,
    1 or 0 of size 7).  Uniform bg 0.25, beta = 1: 7.25/8, 6.25/8, 1.25/8,
    0.25/8.  A non-uniform bg (A .1, C .2, T .3, G .4) with beta = 2 makes each
    letter's own bg visible: column 1 (all A) gives A 7.2/9, C 0.4/9, T 0.6/9,
    G 0.8/9."""
    l = 8
    starts = [7, 18, 2, 4, 30, 26, 14]
    S = oracle.Seqs(DNA, fig1)
    cum = np.concatenate([[0], np.cumsum([len(x) - l + 1 for x in fig1])])
    members = np.array([cum[i] + a for i, a in enumerate(starts)], dtype=np.uint32)
    prof = oracle.profile(S, l, np.array([[0, 0, 7, 0]], dtype=np.uint32), members)
    L = oracle.letters(DNA)
    th = oracle.theta0(prof, np.full(4, 0.25), 1.0)[0]
    by_hand = {  # Fig. 2 rows: A 7 0 0 0 6 7 0 0 / T 0 7 0 0 0 0 0 6 / C 0 0 0 6 1 0 7 0 / G 0 0 7 1 0 0 0 1
        "A": [7.25, .25, .25, .25, 6.25, 7.25, .25, .25],
        "T": [.25, 7.25, .25, .25, .25, .25, .25, 6.25],
        "C": [.25, .25, .25, 6.25, 1.25, .25, 7.25, .25],
        "G": [.25, .25, 7.25, 1.25, .25, .25, .25, 1.25],
    }
    for ch, row in by_hand.items():
        np.testing.assert_allclose(th[L.index(ch)], np.array(row) / 8.0, rtol=1e-15, atol=0)
    bg = np.array([0.1, 0.2, 0.3, 0.4])  # code order A C T G
    th2 = oracle.theta0(prof, bg, 2.0)[0]
    np.testing.assert_allclose(th2[:, 0], [7.2 / 9, 0.4 / 9, 0.6 / 9, 0.8 / 9], rtol=1e-15)
    # column 4 (1-based 5): A 6, C 1 -> A 6.2/9, C 1.4/9, T 0.6/9, G 0.8/9
    np.testing.assert_allclose(th2[:, 4], [6.2 / 9, 1.4 / 9, 0.6 / 9, 0.8 / 9], rtol=1e-15)


def test_example1_objective_at_beta_one(fig1):
    """Example 1 at beta = 1, bg = 0.25, EM from the ATGAC bucket.  The
    oracle's J of theta^0 .. theta^5 equals a letter-level EM written with
    explicit products (no log-odds, no log-sum-exp, dictionaries of letters),
    and the values 19.806893 (theta^0) and 19.806909 (theta^5) obtained by an
    independent computation on the Fig. 1 data.  The plain LLR dips
    (39.702425 -> 39.695728) while J rises: the monotone quantity is J."""
    l, k, s, beta = 8, 5, 4, 1.0
    bg = np.full(4, 0.25)
    r = oracle.run(fig1, DNA, l, k, s, np.array([TOY_MASK_READ]), iters=5, beta=beta, bg=bg)
    names = [_key_to_string(int(b[1]), k, DNA) for b in r["buckets"]]
    b = names.index("ATGAC")
    J, LL = r["J"][b], r["llr"][b]
    assert round(J[0], 6) == 19.806893 and round(J[5], 6) == 19.806909
    assert round(LL[0], 6) == 39.702425 and round(LL[5], 6) == 39.695728
    L = oracle.letters(DNA)
    bgd = {c: 0.25 for c in "ACGT"}
    th = _as_dict(r["theta0"][b], DNA)
    for it in range(6):
        np.testing.assert_allclose(J[it], brute.oops_objective(fig1, l, th, bgd, beta), rtol=1e-12)
        post = [brute.oops_posterior(x, l, th, bgd) for x in fig1]
        th = brute.oops_mstep(fig1, l, post, bgd, beta)
    # theta^5 itself
    got = r["theta"][b]
    th5 = _as_dict(r["theta0"][b], DNA)
    for _ in range(5):
        th5 = brute.oops_mstep(fig1, l, [brute.oops_posterior(x, l, th5, bgd) for x in fig1], bgd, beta)
    for c in "ACGT":
        np.testing.assert_allclose(got[L.index(c)], th5[c], rtol=1e-12)


def test_best_and_consensus_tie_rules():
    """Sec. 5.1 (highest objective wins) and Sec. 2 (consensus ties may go
    either way): the reading taken is the lowest bucket index among equal J
    and the lowest code (A C T G order) among equal probabilities."""
    L = oracle.letters(DNA)
    th = np.zeros((3, 4, 3))
    # model 1 (the winner): column 0 ties A/G, column 1 ties C/T, column 2 ties T/G
    for b in range(3):
        th[b, L.index("A"), 0] = th[b, L.index("G"), 0] = 0.4
        th[b, L.index("C"), 0] = th[b, L.index("T"), 0] = 0.1
        th[b, L.index("C"), 1] = th[b, L.index("T"), 1] = 0.45
        th[b, L.index("A"), 1] = th[b, L.index("G"), 1] = 0.05
        th[b, L.index("T"), 2] = th[b, L.index("G"), 2] = 0.35
        th[b, L.index("A"), 2] = th[b, L.index("C"), 2] = 0.15
    th[2, L.index("G"), 0] = 0.41  # model 2 would read G in column 0
    th[2, L.index("A"), 0] = 0.39
    J = np.array([[0.0, 1.0], [0.0, 3.0], [0.0, 3.0]])
    b, cons = oracle.best(J, th)
    assert b == 1 and cons == "ACT"
    J[1, 1] = np.nan
    b, cons = oracle.best(J, th)
    assert b == 2 and cons == "GCT"


# ------------------------------------------- Sec. 2 motif-length range (l-, l+)
def test_length_range_is_the_per_length_runs_and_the_per_column_choice():
    """run_range at every length equals a plain run at that length (auto
    parameters of Sec. 5, Park-Miller masks of Sec. 6), and the chosen length
    is the argmax of LLR / l over lengths that found a bucket, the longer on
    ties."""
    rng = np.random.default_rng(31)
    inst = planted_instance(rng, 14, 300, 11, 2)
    out, chosen = oracle.run_range(inst.seqs, DNA, 10, 12, 2, 7, 3, 1.0, m=40)
    S = oracle.Seqs(DNA, inst.seqs)
    for r in out:
        k, s, _ = oracle.auto_params(r["l"], 2, 14, S.nwin(r["l"]), DNA)
        assert (r["k"], r["s"], r["m"]) == (k, s, 40)
        ref = oracle.run(inst.seqs, DNA, r["l"], k, s, oracle.masks_from_seed(7, r["l"], k, 40), 3, 1.0)
        assert r["consensus"] == ref["consensus"]
        assert r["llr"] == ref["llr"][ref["best"], -1]
    per_col = {r["l"]: r["llr"] / r["l"] for r in out if r["best"] >= 0}
    top = max(per_col.values())
    assert chosen == max(l for l, v in per_col.items() if v == top)
