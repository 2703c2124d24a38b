"""Brute-force checks on tiny inputs -- TEST INFRASTRUCTURE ONLY.

Pure Python, deliberately independent of ``oracle.c``: these routines work on
the letters themselves (no codes, no base-|Sigma| integers, no logarithms of
odds) so that a mistake in the C oracle cannot hide behind the same mistake
here.
"""
from __future__ import annotations

import itertools
import math
from collections import Counter
from typing import Dict, List, Sequence, Tuple


def projected_string(lmer: str, mask: int) -> str:
    """h_k of an l-mer (Sec. 5): the kept letters, in order."""
    return "".join(ch for p, ch in enumerate(lmer) if mask >> p & 1)


def bucket_sizes(seqs: Sequence[str], l: int, mask: int) -> Counter:
    """PROJECTION1-style dictionary of projected strings -> multiplicity."""
    c = Counter()
    for S in seqs:
        for a in range(len(S) - l + 1):
            c[projected_string(S[a:a + l], mask)] += 1
    return c


def pairwise_sizes(seqs: Sequence[str], l: int, mask: int) -> List[int]:
    """PROJECTION2 (Sec. 5.2 / Sec. 6): every projected k-mer compared with all
    others; the bucket size of l-mer w is 1 + the number of other l-mers with
    an equal projection.  Returned in window order."""
    ks = [projected_string(S[a:a + l], mask) for S in seqs for a in range(len(S) - l + 1)]
    return [1 + sum(1 for v, u in enumerate(ks) if v != w and u == ks[w]) for w in range(len(ks))]


def windows(seqs: Sequence[str], l: int) -> List[Tuple[int, int]]:
    return [(i, a) for i, S in enumerate(seqs) for a in range(len(S) - l + 1)]


def profile_of(lmers: Sequence[str], letters: str) -> Dict[str, List[int]]:
    """Profile matrix P(s) (Sec. 2): per letter, count in each column."""
    l = len(lmers[0])
    return {c: [sum(1 for x in lmers if x[p] == c) for p in range(l)] for c in letters}


def score(lmers: Sequence[str], letters: str) -> int:
    """Score(s) = sum over columns of the largest letter count (Sec. 2)."""
    P = profile_of(lmers, letters)
    return sum(max(P[c][p] for c in letters) for p in range(len(lmers[0])))


def naive_mfp(seqs: Sequence[str], l: int, letters: str) -> Tuple[int, Tuple[int, ...]]:
    """Alg. 1: exhaust every start vector, keep the best Score.  Exponential;
    only for t <= 4 and short sequences."""
    best, arg = -1, None
    ranges = [range(len(S) - l + 1) for S in seqs]
    for st in itertools.product(*ranges):
        v = score([S[a:a + l] for S, a in zip(seqs, st)], letters)
        if v > best:
            best, arg = v, st
    return best, arg


def hamming(u: str, v: str) -> int:
    return sum(1 for a, b in zip(u, v) if a != b)


def ld_candidates(seqs: Sequence[str], l: int, d: int, letters: str) -> List[str]:
    """Every M in Sigma^l that has an l-mer at Hamming distance exactly d in
    every sequence (the (l,d) planted-motif definition, Sec. 2)."""
    out = []
    lm = [[S[a:a + l] for a in range(len(S) - l + 1)] for S in seqs]
    for tup in itertools.product(letters, repeat=l):
        M = "".join(tup)
        if all(any(hamming(M, x) == d for x in xs) for xs in lm):
            out.append(M)
    return out


def oops_loglik_ratio(seqs: Sequence[str], l: int, theta: Dict[str, List[float]],
                      bg: Dict[str, float]) -> float:
    """ln of the OOPS likelihood of the sequences under theta divided by the
    all-background likelihood, computed by explicit products over every start
    position with a uniform start prior (no log-odds, no log-sum-exp)."""
    total = 0.0
    for S in seqs:
        L = len(S) - l + 1
        back = math.prod(bg[ch] for ch in S)
        acc = 0.0
        for a in range(L):
            pr = 1.0
            for j, ch in enumerate(S):
                pr *= theta[ch][j - a] if a <= j < a + l else bg[ch]
            acc += pr / L
        total += math.log(acc / back)
    return total


def oops_posterior(S: str, l: int, theta: Dict[str, List[float]], bg: Dict[str, float]) -> List[float]:
    """P(start = a | S, theta) by Bayes' rule over explicit products."""
    L = len(S) - l + 1
    w = []
    for a in range(L):
        pr = 1.0
        for j, ch in enumerate(S):
            pr *= theta[ch][j - a] if a <= j < a + l else bg[ch]
        w.append(pr)
    z = sum(w)
    return [v / z for v in w]


def expected_complete_loglik(seqs: Sequence[str], l: int, post: Sequence[Sequence[float]],
                             theta: Dict[str, List[float]]) -> float:
    """Q(theta) = sum_i sum_a P(a | S_i) * sum_p ln theta[S_i[a+p]][p]: the part of
    the expected complete-data log likelihood that depends on the motif model."""
    q = 0.0
    for S, ps in zip(seqs, post):
        for a, w in enumerate(ps):
            if w == 0.0:
                continue
            q += w * sum(math.log(theta[S[a + p]][p]) for p in range(l))
    return q


def oops_mstep(seqs: Sequence[str], l: int, post: Sequence[Sequence[float]], bg: Dict[str, float],
               beta: float) -> Dict[str, List[float]]:
    """One M-step on letters: the expected count of each letter in each column
    (every start weighted by its posterior), smoothed by beta * bg and divided
    by the column's total mass t + beta (Sec. 5.1 names EM; the update is the
    textbook one for a multinomial column under a Dirichlet prior)."""
    out = {c: [beta * bg[c]] * l for c in bg}
    for S, ps in zip(seqs, post):
        for a, w in enumerate(ps):
            for p in range(l):
                out[S[a + p]][p] += w
    tot = len(seqs) + beta
    return {c: [v / tot for v in col] for c, col in out.items()}


def oops_objective(seqs: Sequence[str], l: int, theta: Dict[str, List[float]], bg: Dict[str, float],
                   beta: float) -> float:
    """The objective EM climbs: the OOPS log-likelihood ratio (explicit
    products) plus the log prior beta * sum_c bg_c sum_p ln theta_c[p]."""
    pri = sum(bg[c] * math.log(theta[c][p]) for c in bg for p in range(l))
    return oops_loglik_ratio(seqs, l, theta, bg) + beta * pri


def _site_product(S: str, l: int, a: int, theta: Dict[str, List[float]], bg: Dict[str, float]) -> float:
    """P(S | the motif starts at a) by an explicit product over every letter."""
    pr = 1.0
    for j, ch in enumerate(S):
        pr *= theta[ch][j - a] if a <= j < a + l else bg[ch]
    return pr


def zoops_loglik_ratio(seqs: Sequence[str], l: int, theta: Dict[str, List[float]], bg: Dict[str, float],
                       gamma: float) -> float:
    """ln P(S | ZOOPS) / P(S | background) by explicit products: each sequence
    holds no site with probability 1 - gamma, else one site at a uniform start
    (Sec. 2: at most one occurrence per sequence)."""
    total = 0.0
    for S in seqs:
        L = len(S) - l + 1
        back = math.prod(bg[ch] for ch in S)
        acc = (1.0 - gamma) * back + sum(gamma / L * _site_product(S, l, a, theta, bg) for a in range(L))
        total += math.log(acc / back)
    return total


def zoops_posterior(S: str, l: int, theta: Dict[str, List[float]], bg: Dict[str, float],
                    gamma: float) -> List[float]:
    """P(site at a | S) under ZOOPS by Bayes' rule over explicit products (the
    remaining mass is the no-site case)."""
    L = len(S) - l + 1
    back = math.prod(bg[ch] for ch in S)
    w = [gamma / L * _site_product(S, l, a, theta, bg) for a in range(L)]
    z = (1.0 - gamma) * back + sum(w)
    return [v / z for v in w]


def tcm_loglik_ratio(seqs: Sequence[str], l: int, theta: Dict[str, List[float]], bg: Dict[str, float],
                     lam: float) -> float:
    """ln of the TCM likelihood ratio: every window independently an
    occurrence with probability lam (Sec. 2: zero or more occurrences),
    explicit products per window."""
    total = 0.0
    for S in seqs:
        for a in range(len(S) - l + 1):
            w = S[a:a + l]
            motif = math.prod(theta[ch][p] for p, ch in enumerate(w))
            back = math.prod(bg[ch] for ch in w)
            total += math.log(((1.0 - lam) * back + lam * motif) / back)
    return total


def tcm_posterior(S: str, l: int, theta: Dict[str, List[float]], bg: Dict[str, float], lam: float) -> List[float]:
    out = []
    for a in range(len(S) - l + 1):
        w = S[a:a + l]
        motif = lam * math.prod(theta[ch][p] for p, ch in enumerate(w))
        back = (1.0 - lam) * math.prod(bg[ch] for ch in w)
        out.append(motif / (motif + back))
    return out


def mixture_expected_loglik(seqs: Sequence[str], l: int, post: Sequence[Sequence[float]],
                            theta: Dict[str, List[float]], mix: float, model: str) -> float:
    """The part of the expected complete-data log-likelihood that depends on
    (theta, mix): sum Z ln theta over the site columns, plus the mixing terms
    (ZOOPS: per sequence q ln gamma + (1 - q) ln(1 - gamma), q = sum_a Z;
    TCM: per window Z ln lam + (1 - Z) ln(1 - lam))."""
    v = expected_complete_loglik(seqs, l, post, theta)
    for ps in post:
        if model == "zoops":
            q = sum(ps)
            v += q * math.log(mix) + (1.0 - q) * math.log(1.0 - mix)
        else:
            v += sum(z * math.log(mix) + (1.0 - z) * math.log(1.0 - mix) for z in ps)
    return v


def gibbs_conditional(seqs: Sequence[str], l: int, sites: Sequence[int], i: int, bg: Dict[str, float],
                      beta: float) -> List[float]:
    """P(a_i = a | the other sites) for the site sampler: the model is the
    profile of the other t-1 aligned l-mers with pseudocounts beta * bg, and
    the start is drawn by Bayes' rule over explicit products (uniform prior)."""
    others = [seqs[j][sites[j]:sites[j] + l] for j in range(len(seqs)) if j != i]
    theta = {c: [(sum(1 for w in others if w[p] == c) + beta * bg[c]) / (len(others) + beta) for p in range(l)]
             for c in bg}
    S = seqs[i]
    w = [_site_product(S, l, a, theta, bg) for a in range(len(S) - l + 1)]
    z = sum(w)
    return [v / z for v in w]


def alignment_log_odds(seqs: Sequence[str], l: int, sites: Sequence[int], bg: Dict[str, float],
                       beta: float) -> float:
    """F = sum over columns and letters of count * ln(theta / bg), theta the
    smoothed profile of the aligned l-mers."""
    words = [S[a:a + l] for S, a in zip(seqs, sites)]
    t = len(words)
    F = 0.0
    for c in bg:
        for p in range(l):
            n = sum(1 for w in words if w[p] == c)
            if n:
                F += n * math.log((n + beta * bg[c]) / (t + beta) / bg[c])
    return F
