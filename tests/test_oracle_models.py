"""Pins of the oracle's ZOOPS and TCM EM (the two sequence models Sec. 2
names beside OOPS) against explicit products, Bayes' rule, the M-step's
optimality, the EM guarantee and the special cases where the models meet.
Nothing here touches the GPU; the brute-force side works on letters."""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import planted_instance, random_sequences

DNA, PROT = 4, 20


def _rand_theta(rng, A, l):
    return np.ascontiguousarray(rng.dirichlet(np.ones(A), size=l).T)


def _as_dict(th, A):
    return {c: list(th[i]) for i, c in enumerate(oracle.letters(A))}


@pytest.mark.parametrize("A,alpha", [(DNA, "dna"), (PROT, "protein")])
@pytest.mark.parametrize("mix", [0.05, 0.5, 0.93])
def test_zoops_estep_equals_explicit_products(A, alpha, mix):
    rng = np.random.default_rng(int(mix * 100) + A)
    seqs = random_sequences(rng, 3, [9, 12, 10], alpha)
    l = 4
    S = oracle.Seqs(A, seqs)
    th = _rand_theta(rng, A, l)
    bg = rng.dirichlet(np.ones(A))
    bgd = dict(zip(oracle.letters(A), bg))
    llr, s, Z, q = oracle.estep_model(S, l, oracle.ZOOPS, mix, th, bg)
    ref = brute.zoops_loglik_ratio(seqs, l, _as_dict(th, A), bgd, mix)
    assert math.isclose(llr, ref, rel_tol=1e-11, abs_tol=1e-12)
    w0 = 0
    for i, seq in enumerate(seqs):
        post = brute.zoops_posterior(seq, l, _as_dict(th, A), bgd, mix)
        np.testing.assert_allclose(Z[w0:w0 + len(post)], post, rtol=1e-11, atol=1e-15)
        assert math.isclose(q[i], sum(post), rel_tol=1e-11)
        w0 += len(post)


@pytest.mark.parametrize("A,alpha", [(DNA, "dna"), (PROT, "protein")])
@pytest.mark.parametrize("mix", [0.01, 0.3, 0.9])
def test_tcm_estep_equals_explicit_products(A, alpha, mix):
    rng = np.random.default_rng(int(mix * 100) + 7 * A)
    seqs = random_sequences(rng, 3, [9, 12, 10], alpha)
    l = 5
    S = oracle.Seqs(A, seqs)
    th = _rand_theta(rng, A, l)
    bg = rng.dirichlet(np.ones(A))
    bgd = dict(zip(oracle.letters(A), bg))
    llr, s, Z, q = oracle.estep_model(S, l, oracle.TCM, mix, th, bg)
    ref = brute.tcm_loglik_ratio(seqs, l, _as_dict(th, A), bgd, mix)
    assert math.isclose(llr, ref, rel_tol=1e-11, abs_tol=1e-12)
    post = np.concatenate([brute.tcm_posterior(x, l, _as_dict(th, A), bgd, mix) for x in seqs])
    np.testing.assert_allclose(Z, post, rtol=1e-11, atol=1e-15)


def test_zoops_with_gamma_one_is_oops():
    rng = np.random.default_rng(3)
    inst = planted_instance(rng, 6, 70, 9, 2)
    S = oracle.Seqs(DNA, inst.seqs)
    bg = np.full(4, 0.25)
    th0 = np.stack([_rand_theta(rng, DNA, 9) for _ in range(5)])
    th, mix, J, LL, sites = oracle.em_model(S, 9, oracle.ZOOPS, 1.0, th0, bg, 4, 1.0)
    th_o, J_o, LL_o, sites_o = oracle.em(S, 9, th0, bg, 4, 1.0)
    np.testing.assert_allclose(J, J_o, rtol=1e-12)
    np.testing.assert_allclose(LL, LL_o, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(th, th_o, rtol=1e-12)
    np.testing.assert_allclose(mix, 1.0, rtol=1e-12)
    assert np.array_equal(sites, sites_o)


def test_models_meet_on_one_window_per_sequence():
    """With n_i = l every sequence has one window: at most one occurrence and
    any number of occurrences are the same model, so ZOOPS and TCM agree on
    every iteration (the gamma and lambda updates divide by t = x)."""
    rng = np.random.default_rng(4)
    l = 7
    seqs = random_sequences(rng, 12, l, "dna")
    S = oracle.Seqs(DNA, seqs)
    bg = rng.dirichlet(np.ones(4))
    th0 = np.stack([_rand_theta(rng, DNA, l) for _ in range(3)])
    z = oracle.em_model(S, l, oracle.ZOOPS, 0.4, th0, bg, 5, 0.7)
    t = oracle.em_model(S, l, oracle.TCM, 0.4, th0, bg, 5, 0.7)
    for a, b in zip(z[:4], t[:4]):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)
    assert np.array_equal(z[4], t[4])


@pytest.mark.parametrize("model", [oracle.ZOOPS, oracle.TCM])
def test_background_model_is_a_fixed_point(model):
    """theta = bg: every score is 0, LLR = 0, the posteriors are the prior
    (gamma / L_i, or lambda), the mixing parameter does not move, and the new
    theta is the windows' letter composition weighted by that prior."""
    rng = np.random.default_rng(5)
    seqs = random_sequences(rng, 4, [30, 25, 40, 33], "dna")
    S = oracle.Seqs(DNA, seqs)
    bg = np.array([0.1, 0.2, 0.3, 0.4])
    l = 6
    th = np.repeat(bg[:, None], l, axis=1)
    llr, s, Z, q = oracle.estep_model(S, l, model, 0.35, th, bg)
    assert abs(llr) < 1e-13 and np.all(s == 0.0)
    if model == oracle.ZOOPS:
        Ls = [len(x) - l + 1 for x in seqs]
        np.testing.assert_allclose(Z, np.concatenate([np.full(L, 0.35 / L) for L in Ls]), rtol=1e-13)
    else:
        np.testing.assert_allclose(Z, 0.35, rtol=1e-13)
    new, mix = oracle.mstep_model(S, l, model, Z, bg, 1.0, 0.35)
    assert math.isclose(mix, 0.35, rel_tol=1e-13)
    L = oracle.letters(DNA)
    cnt = np.zeros((4, l))
    for x, zs in zip(seqs, np.split(Z, np.cumsum([len(q) - l + 1 for q in seqs])[:-1])):
        for a, z in enumerate(zs):
            for p in range(l):
                cnt[L.index(x[a + p]), p] += z
    np.testing.assert_allclose(new, (cnt + bg[:, None]) / (Z.sum() + 1.0), rtol=1e-12)


@pytest.mark.parametrize("model,name", [(oracle.ZOOPS, "zoops"), (oracle.TCM, "tcm")])
def test_mstep_maximises_expected_loglik(model, name):
    """The M-step maximises the expected complete log-likelihood plus the
    Dirichlet prior over theta on the simplex and the mixing parameter on
    (0, 1): random feasible moves of (theta, mix) never increase it."""
    rng = np.random.default_rng(6)
    seqs = random_sequences(rng, 3, [14, 11, 16], "dna")
    l, A = 4, DNA
    S = oracle.Seqs(A, seqs)
    bg = rng.dirichlet(np.ones(A))
    bgd = dict(zip(oracle.letters(A), bg))
    th = _rand_theta(rng, A, l)
    mix = 0.4
    if model == oracle.ZOOPS:
        post = [brute.zoops_posterior(x, l, _as_dict(th, A), bgd, mix) for x in seqs]
    else:
        post = [brute.tcm_posterior(x, l, _as_dict(th, A), bgd, mix) for x in seqs]
    Z = np.concatenate(post)
    for beta in (0.0, 0.5, 2.0):
        new, mix2 = oracle.mstep_model(S, l, model, Z, bg, beta, mix)
        np.testing.assert_allclose(new.sum(axis=0), 1.0, rtol=1e-13)

        def obj(t_, m_):
            q = brute.mixture_expected_loglik(seqs, l, post, _as_dict(t_, A), m_, name)
            return q + beta * float(np.sum(bg[:, None] * np.log(t_)))

        base = obj(new, mix2)
        for _ in range(40):
            d = rng.normal(size=(A, l))
            d -= d.mean(axis=0)
            eps = 1e-3 * float(rng.uniform(0.1, 1.0))
            cand = new + eps * d
            cm = mix2 + 1e-3 * float(rng.normal())
            if np.all(cand > 0) and 0 < cm < 1:
                assert obj(cand, cm) <= base + 1e-12


@pytest.mark.parametrize("model", [oracle.ZOOPS, oracle.TCM])
@pytest.mark.parametrize("beta", [0.1, 1.0])
def test_em_objective_never_decreases(model, beta):
    rng = np.random.default_rng(9)
    inst = planted_instance(rng, 10, 90, 10, 2)
    S = oracle.Seqs(DNA, inst.seqs)
    bg = np.full(4, 0.25)
    th0 = np.stack([_rand_theta(rng, DNA, 10) for _ in range(6)])
    mix0 = 0.5 if model == oracle.ZOOPS else 0.01
    th, mix, J, LL, sites = oracle.em_model(S, 10, model, mix0, th0, bg, 8, beta)
    assert np.all(np.diff(J, axis=1) >= -1e-9 * np.abs(J[:, 1:]))
    assert np.all((mix > 0) & (mix <= 1))


def test_zoops_finds_the_planted_sites_and_the_empty_sequences():
    """Half of the sequences carry a planted (16,1) site, the other half none:
    ZOOPS started from the motif itself keeps the planted starts and reports
    no site (-1) in (nearly) every sequence without one -- a random 16-mer can
    still look enough like the motif -- and gamma ends near one half, where
    OOPS reports a site in every sequence."""
    rng = np.random.default_rng(10)
    inst = planted_instance(rng, 12, 150, 16, 1)
    empty = random_sequences(rng, 12, 150, "dna")
    seqs = inst.seqs + empty
    S = oracle.Seqs(DNA, seqs)
    bg = np.full(4, 0.25)
    L = oracle.letters(DNA)
    th0 = np.full((4, 16), 0.05)
    for p, ch in enumerate(inst.motif):
        th0[L.index(ch), p] = 0.85
    th, mix, J, LL, sites = oracle.em_model(S, 16, oracle.ZOOPS, 0.5, th0[None], bg, 10, 1.0)
    assert np.array_equal(sites[0, :12], inst.starts)
    assert np.sum(sites[0, 12:] == -1) >= 10
    assert 0.4 < mix[0] < 0.65
    assert np.all(oracle.em(S, 16, th0[None], bg, 10, 1.0)[3] >= 0)
