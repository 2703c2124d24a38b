"""Pins of the triage oracle: closed forms of the features, the network and
Adam, finite differences for the gradients, brute force for the selection."""
import math

import numpy as np

from oracle import triage as T


def test_features_closed_forms():
    bg = np.full(4, 0.25)
    l = 3
    prof = np.zeros((3, 4, l))
    prof[0] = 2                          # uniform columns: no information
    prof[1, 1, :] = 5                    # one letter per column: 2 bits each
    prof[2, :, 0] = [2, 1, 1, 0]         # 0.5 log2 2 + 2 * 0.25 log2 1 = 0.5 bits
    prof[2, 0, 1:] = 4
    F = T.features(prof, bg)
    assert F.shape == (3, 87)
    assert np.all(F[:, 4 * l:84] == 0)   # padding columns
    for b in range(3):
        cols = F[b, :4 * l].reshape(l, 4)
        assert np.allclose(cols.sum(axis=1), 1.0)
        assert math.isclose(F[b, 85], 2.0)
    assert np.allclose(F[1, :4 * l].reshape(l, 4), [[1, 0, 0, 0]] * l)
    # bucket 2: two pure columns first, then (2,1,1,0)/4
    assert np.allclose(F[2, :4 * l].reshape(l, 4), [[1, 0, 0, 0], [1, 0, 0, 0], [0.5, 0.25, 0.25, 0]])
    assert math.isclose(F[0, 84], math.log(8)) and math.isclose(F[1, 84], math.log(5))
    assert math.isclose(F[0, 86], 0.0, abs_tol=1e-15)
    assert math.isclose(F[1, 86], 2.0)
    assert math.isclose(F[2, 86], 2.0)   # columns 1, 2 are pure
    prof[2, 0, 1:] = 0
    prof[2, :, 1:] = 1
    assert math.isclose(T.features(prof[2:], bg)[0, 86], 0.5)


def test_features_canonical_order():
    """Sorted letters within a column, columns in decreasing order of their
    sorted counts; permuting positions or renaming letters changes nothing."""
    rng = np.random.default_rng(5)
    bg = np.full(4, 0.25)
    prof = rng.integers(0, 6, size=(4, 4, 9)).astype(float)
    prof[:, 0, :] += 1
    # every column must total the bucket size
    tot = prof.sum(axis=1, keepdims=True)
    prof[:, 0:1, :] += tot.max() - tot
    F = T.features(prof, bg)
    for b in range(4):
        cols = F[b, :36].reshape(9, 4)
        assert np.all(np.diff(cols, axis=1) <= 0)          # letters sorted
        keys = [tuple(c) for c in cols]
        assert keys == sorted(keys, reverse=True)          # columns sorted
    perm = rng.permutation(9)
    lett = rng.permutation(4)
    G = T.features(prof[:, lett][:, :, perm], bg)
    assert np.array_equal(F[:, :84], G[:, :84]) and np.allclose(F[:, 84:86], G[:, 84:86])
    assert np.allclose(F[:, 86], G[:, 86])


def test_features_nonuniform_background_entropy():
    bg = np.array([0.5, 0.25, 0.125, 0.125])
    prof = np.zeros((1, 4, 2))
    prof[0, 3] = 1                       # letter of probability 1/8: 3 bits
    F = T.features(prof, bg)
    assert math.isclose(F[0, 85], 1.75)
    assert math.isclose(F[0, 86], 3.0)


def test_forward_hand_network():
    sizes = (3, 2, 2, 1)
    W1 = np.array([[1.0, -1.0], [2.0, 0.0], [0.0, 1.0]])
    b1 = np.array([0.5, -4.0])
    W2 = np.array([[1.0, 2.0], [3.0, -1.0]])
    b2 = np.array([0.0, -1.0])
    W3 = np.array([[2.0], [-0.5]])
    b3 = np.array([0.25])
    X = np.array([[1.0, 1.0, 1.0], [-1.0, 0.0, 10.0]])
    # row 0: z1 = (3.5, -4) -> (3.5, 0); z2 = (3.5, 6) -> y = 7 - 3 + 0.25
    # row 1: z1 = (-0.5, 7) -> (0, 7);   z2 = (21, -8) -> (21, 0) -> y = 42.25
    y, _ = T.forward([W1, b1, W2, b2, W3, b3], X)
    assert np.allclose(y, [4.25, 42.25])
    assert sizes[0] == W1.shape[0]


def _fd_check(params, X, t, idx_sets, h=1e-6):
    y, cache = T.forward(params, X)
    grads = T.backward(params, cache, y, t)
    for k, idxs in idx_sets:
        for idx in idxs:
            P = [p.copy() for p in params]
            P[k][idx] += h
            lp = T.loss(T.forward(P, X)[0], t)
            P[k][idx] -= 2 * h
            lm = T.loss(T.forward(P, X)[0], t)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grads[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, grads[k][idx])


def test_backward_matches_finite_differences_small():
    rng = np.random.default_rng(0)
    sizes = (5, 7, 6, 1)
    params = T.init_params(rng, sizes)
    params = [p + 0.1 * rng.normal(size=p.shape) for p in params]  # non-zero biases too
    X = rng.normal(size=(9, 5))
    t = rng.normal(size=9)
    sets = [(k, list(np.ndindex(p.shape))) for k, p in enumerate(params)]
    _fd_check(params, X, t, sets)


def test_backward_matches_finite_differences_full_size_sample():
    rng = np.random.default_rng(1)
    params = T.init_params(rng)
    params = [p + 0.05 * rng.normal(size=p.shape) for p in params]
    X = rng.normal(size=(6, T.N_IN))
    t = rng.normal(size=6)
    sets = []
    for k, p in enumerate(params):
        flat_idx = rng.choice(p.size, size=min(12, p.size), replace=False)
        sets.append((k, [np.unravel_index(i, p.shape) for i in flat_idx]))
    _fd_check(params, X, t, sets)


def test_adam_first_step_closed_form():
    g = [np.array([0.5, -2.0, 1e-3]), np.array([[3.0]])]
    p = [np.zeros(3), np.ones((1, 1))]
    m = [np.zeros_like(x) for x in p]
    v = [np.zeros_like(x) for x in p]
    T.adam_step(p, g, m, v, 1, lr=0.01, eps=1e-8)
    # bias-corrected moments are g and g^2: the step is lr * sign(g) (up to eps)
    assert np.allclose(p[0], -0.01 * np.sign(g[0]) * np.abs(g[0]) / (np.abs(g[0]) + 1e-8))
    assert np.allclose(p[1], 1.0 - 0.01 * 3.0 / (3.0 + 1e-8))


def test_adam_minimises_a_quadratic():
    x = [np.array([5.0, -3.0])]
    m, v = [np.zeros(2)], [np.zeros(2)]
    for step in range(1, 3001):
        T.adam_step(x, [2 * x[0]], m, v, step, lr=0.05)
    assert np.all(np.abs(x[0]) < 1e-2)


def test_top_fraction_brute_force():
    rng = np.random.default_rng(3)
    scores = np.round(rng.normal(size=200), 1)     # many ties
    group = np.sort(rng.integers(0, 5, size=200))
    for frac in (0.01, 0.05, 0.3, 1.0):
        keep = T.top_fraction(scores, group, frac)
        for gval in np.unique(group):
            idx = np.nonzero(group == gval)[0]
            c = max(1, math.ceil(frac * len(idx)))
            # kept = everything at least as large as the c-th largest
            ranked = sorted(scores[idx], reverse=True)
            assert set(idx[keep[idx]]) == {i for i in idx if scores[i] >= ranked[c - 1]}
            assert keep[idx].sum() >= c


def test_bf16_rounding_values():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 3.0e-3, 65504.0, 0.0])
    r = T.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1 + 2 ** -6 and r[3] == -2.5 and r[6] == 0.0
    assert abs(r[4] - 3.0e-3) <= 2 ** -8 * 3.0e-3  # half a unit in the 8th bit
    # 65504 = 1.99902... * 2^15 rounds to 2^16 with 8 significant bits
    assert r[5] == 65536.0


def test_flat_roundtrip_and_count():
    rng = np.random.default_rng(4)
    params = T.init_params(rng)
    v = T.flat(params)
    assert v.size == 88577
    back = T.unflat(v)
    assert all(np.array_equal(a, b) for a, b in zip(params, back))


def test_winner_z_closed_form():
    J = np.array([1.0, 2.0, 3.0, 10.0, 10.0, 4.0])
    group = np.array([0, 0, 0, 1, 1, 2])
    z = T.winner_z(J, group, {0: 2, 1: 3})
    # group 0: mean 2, population sd sqrt(2/3) -> z = 1 / sqrt(2/3)
    assert math.isclose(z[0], 1 / math.sqrt(2 / 3))
    assert z[1] == 0.0                 # equal objectives: sd = 0
    assert z[2] == -math.inf           # no winner
