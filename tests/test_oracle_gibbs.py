"""Pins of the oracle's Gibbs site sampler (the local optimiser Sec. 1 and
Sec. 3 name beside EM): its random numbers against numpy's Philox4x64-10, its
conditional distribution against Bayes' rule over explicit products, the
alignment score on letters, the sampling loop replayed step by step, and a
planted instance.  Nothing here touches the GPU."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import planted_instance, random_sequences

DNA, PROT = 4, 20


def test_philox_matches_numpy():
    """Philox4x64-10 (Salmon et al., SC'11): numpy's generator increments its
    256-bit counter before each block, so its first block is the oracle's
    block at counter + 1."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        ctr = rng.integers(1, 2 ** 63, size=4, dtype=np.uint64)
        g = np.random.Philox(key=key, counter=ctr - np.array([1, 0, 0, 0], dtype=np.uint64))
        assert np.array_equal(g.random_raw(4).astype(np.uint64), oracle.philox4x64(ctr, key))
    g = np.random.Philox(key=np.zeros(2, dtype=np.uint64), counter=np.zeros(4, dtype=np.uint64))
    assert np.array_equal(g.random_raw(4).astype(np.uint64), oracle.philox4x64([1, 0, 0, 0], [0, 0]))


def test_uniforms_are_53_bit_and_spread():
    u = np.array([oracle.gibbs_uniform(9, r, i, b) for r in range(10) for i in range(20) for b in range(10)])
    assert np.all((u >= 0) & (u < 1)) and len(set(u)) == len(u)
    assert abs(u.mean() - 0.5) < 0.03
    assert np.all(u * 2 ** 53 == np.floor(u * 2 ** 53))


@pytest.mark.parametrize("A,alpha", [(DNA, "dna"), (PROT, "protein")])
def test_conditional_is_bayes_over_explicit_products(A, alpha):
    rng = np.random.default_rng(2)
    seqs = random_sequences(rng, 5, [14, 11, 17, 12, 15], alpha)
    l = 5
    S = oracle.Seqs(A, seqs)
    bg = rng.dirichlet(np.ones(A))
    bgd = dict(zip(oracle.letters(A), bg))
    sites = [int(rng.integers(0, len(q) - l + 1)) for q in seqs]
    for beta in (0.3, 1.0):
        for i in range(len(seqs)):
            w = oracle.gibbs_weights(S, l, bg, beta, sites, i)
            ref = brute.gibbs_conditional(seqs, l, sites, i, bgd, beta)
            np.testing.assert_allclose(w, ref, rtol=1e-11, atol=1e-15)


def test_alignment_score_on_letters():
    rng = np.random.default_rng(3)
    seqs = random_sequences(rng, 6, 30, "dna")
    S = oracle.Seqs(DNA, seqs)
    bg = rng.dirichlet(np.ones(4))
    bgd = dict(zip(oracle.letters(DNA), bg))
    for _ in range(5):
        sites = [int(rng.integers(0, 30 - 8 + 1)) for _ in seqs]
        F, th = oracle.alignment_score(S, 8, bg, 0.7, sites)
        assert math.isclose(F, brute.alignment_log_odds(seqs, 8, sites, bgd, 0.7), rel_tol=1e-12)
        np.testing.assert_allclose(th.sum(axis=0), 1.0, rtol=1e-13)


def test_sampler_replayed_step_by_step():
    """The chain from theta0's best starts, sequences visited in order, each
    start drawn as the first whose running weight exceeds u times the total,
    F after every sweep, and the best alignment kept (earliest on ties)."""
    rng = np.random.default_rng(4)
    inst = planted_instance(rng, 7, [40, 55, 38, 61, 47, 50, 44], 9, 2)
    S = oracle.Seqs(DNA, inst.seqs)
    bg = np.full(4, 0.25)
    th0 = np.stack([rng.dirichlet(np.ones(4), size=9).T for _ in range(3)])
    sweeps, beta, seed = 6, 0.8, 12345
    th, F, sites = oracle.gibbs(S, 9, th0, bg, sweeps, beta, seed)
    for b in range(3):
        _, s, _, _ = oracle.estep(S, 9, th0[b], bg)
        cur, w0 = [], 0
        for q in inst.seqs:
            L = len(q) - 8
            cur.append(int(np.argmax(s[w0:w0 + L])))
            w0 += L
        hist = [oracle.alignment_score(S, 9, bg, beta, cur)[0]]
        best, bF = list(cur), hist[0]
        for r in range(sweeps):
            for i in range(len(cur)):
                w = oracle.gibbs_weights(S, 9, bg, beta, cur, i)
                u = oracle.gibbs_uniform(seed, r, i, b)
                cur[i] = min(int(np.searchsorted(np.cumsum(w), u, side="right")), len(w) - 1)
            hist.append(oracle.alignment_score(S, 9, bg, beta, cur)[0])
            if hist[-1] > bF:
                best, bF = list(cur), hist[-1]
        np.testing.assert_allclose(F[b], hist, rtol=1e-12)
        assert list(sites[b]) == best
        np.testing.assert_allclose(th[b], oracle.alignment_score(S, 9, bg, beta, best)[1], rtol=1e-13)


def test_planted_motif_is_sampled():
    """A (12,1) motif in 12 sequences of 120.  From weak models of the motif
    (0.4 on each consensus letter, as a bucket's profile gives) the best
    alignment is the planted one; from random models the sampler still
    improves on its start (it can lock onto a shifted copy of the motif, the
    phase trap of site samplers)."""
    rng = np.random.default_rng(5)
    inst = planted_instance(rng, 12, 120, 12, 1)
    S = oracle.Seqs(DNA, inst.seqs)
    bg = np.full(4, 0.25)
    L = oracle.letters(DNA)
    weak = np.full((4, 12), 0.2)
    for p, ch in enumerate(inst.motif):
        weak[L.index(ch), p] = 0.4
    th, F, sites = oracle.gibbs(S, 12, np.stack([weak] * 4), bg, 10, 1.0, 99)
    for b in range(4):
        assert np.array_equal(sites[b], inst.starts)
    rnd = np.stack([rng.dirichlet(np.ones(4), size=12).T for _ in range(8)])
    th, F, sites = oracle.gibbs(S, 12, rnd, bg, 30, 1.0, 99)
    assert np.all(F.max(axis=1) > F[:, 0])


def test_gibbs_needs_positive_beta():
    S = oracle.Seqs(DNA, ["ACGTACGTAC", "ACGTTTGTAC"])
    with pytest.raises(ValueError):
        oracle.gibbs(S, 4, np.full((1, 4, 4), 0.25), np.full(4, 0.25), 2, 0.0, 1)
