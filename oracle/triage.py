"""CPU oracle of the learned bucket triage -- TEST INFRASTRUCTURE ONLY.

Plain FP64 numpy, written from the description of the triage network (bucket
features -> 87 -> 256 -> 256 -> 1 multilayer perceptron with ReLU, trained by
mean-squared error against the post-EM score of the bucket, Adam updates) and
from the textbook definitions it rests on: the information content of a
profile column in bits relative to the background, the Shannon entropy of the
background, the chain rule for the gradients, and Adam (Kingma and Ba, 2015).
Only tests/ may import it.  It shares no code with the GPU path.

Feature vector of a DNA bucket (87 values).  The PWM block is the profile's
frequencies in a canonical order: within a column the four letter frequencies
in decreasing order, and the columns in decreasing lexicographic order of
those sorted counts; padded to l_max = 21 columns with zeros.  Which letters
and which motif positions carry the agreement says nothing about whether the
bucket holds motif copies (the projection picks the positions at random), so
the network sees the agreement pattern only.
    [r * 4 + j] for r < 21, j < 4 : j-th largest frequency of the r-th column
    [84]  ln(size)
    [85]  background entropy  -sum_c bg_c log2 bg_c        (bits)
    [86]  max over columns of sum_c f_cp log2(f_cp / bg_c) (bits; 0 log 0 = 0)
"""
from __future__ import annotations

import math

import numpy as np

L_MAX = 21
N_IN = 4 * L_MAX + 3
HIDDEN = 256


def features(profile: np.ndarray, bg: np.ndarray) -> np.ndarray:
    """profile [B][4][l] letter counts per column -> [B][87] features."""
    profile = np.asarray(profile, dtype=np.float64)
    B, A, l = profile.shape
    assert A == 4 and 1 <= l <= L_MAX
    bg = np.asarray(bg, dtype=np.float64)
    out = np.zeros((B, N_IN))
    for b in range(B):
        size = profile[b, :, 0].sum()
        f = profile[b] / size
        cols = sorted((tuple(sorted((int(profile[b, c, p]) for c in range(4)), reverse=True))
                       for p in range(l)), reverse=True)
        for r, col in enumerate(cols):
            for j in range(4):
                out[b, 4 * r + j] = col[j] / size
        out[b, 84] = math.log(size)
        out[b, 85] = -sum(v * math.log2(v) for v in bg if v > 0)
        ic = []
        for p in range(l):
            ic.append(sum(f[c, p] * math.log2(f[c, p] / bg[c]) for c in range(4) if f[c, p] > 0))
        out[b, 86] = max(ic)
    return out


def init_params(rng: np.random.Generator, sizes=(N_IN, HIDDEN, HIDDEN, 1)) -> list:
    """He-normal weights, zero biases: [W1, b1, W2, b2, W3, b3], W_i [in][out]."""
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        params.append(rng.normal(0.0, math.sqrt(2.0 / a), size=(a, b)))
        params.append(np.zeros(b))
    return params


def forward(params: list, X: np.ndarray):
    """Scores y [N] and the activations the backward pass needs."""
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1 + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2 + b2
    H2 = np.maximum(Z2, 0.0)
    y = (H2 @ W3 + b3)[:, 0]
    return y, (X, Z1, H1, Z2, H2)


def loss(y: np.ndarray, target: np.ndarray) -> float:
    """Mean squared error."""
    return float(np.mean((y - target) ** 2))


def backward(params: list, cache, y: np.ndarray, target: np.ndarray) -> list:
    """Gradients of the mean squared error by the chain rule, in the order of
    params."""
    W1, b1, W2, b2, W3, b3 = params
    X, Z1, H1, Z2, H2 = cache
    N = len(y)
    dy = 2.0 * (y - target) / N            # dL/dy
    gW3 = H2.T @ dy[:, None]
    gb3 = np.array([dy.sum()])
    dZ2 = (dy[:, None] @ W3.T) * (Z2 > 0)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * (Z1 > 0)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(axis=0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments) of every tensor, in place.
    step counts from 1."""
    for P, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1 - beta1) * g
        vv *= beta2
        vv += (1 - beta2) * g * g
        mh = mm / (1 - beta1 ** step)
        vh = vv / (1 - beta2 ** step)
        P -= lr * mh / (np.sqrt(vh) + eps)


def top_fraction(scores: np.ndarray, group: np.ndarray, frac: float) -> np.ndarray:
    """Per group (instance): keep every bucket whose score is at least the
    c-th largest of the group, c = ceil(frac * n_group) (at least 1).  Returns
    a boolean mask."""
    keep = np.zeros(len(scores), dtype=bool)
    for gval in np.unique(group):
        idx = np.nonzero(group == gval)[0]
        c = max(1, math.ceil(frac * len(idx)))
        cut = np.sort(scores[idx])[::-1][c - 1]
        keep[idx[scores[idx] >= cut]] = True
    return keep


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits), ties to even, via
    the bit pattern of the float32 value; returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(params: list, X: np.ndarray) -> np.ndarray:
    """The serving arithmetic: inputs, W1, W2 and the first hidden layer
    rounded to bfloat16, everything else exact."""
    W1, b1, W2, b2, W3, b3 = params
    H1 = bf16_round(np.maximum(bf16_round(X) @ bf16_round(W1) + b1, 0.0))
    H2 = np.maximum(H1 @ bf16_round(W2) + b2, 0.0)
    return (H2 @ W3 + b3)[:, 0]


def flat(params: list) -> np.ndarray:
    """The parameters as one vector: W1, b1, W2, b2, W3, b3 (row-major)."""
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in params])


def unflat(v: np.ndarray, sizes=(N_IN, HIDDEN, HIDDEN, 1)) -> list:
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append(np.asarray(v[o:o + a * b], dtype=np.float64).reshape(a, b))
        o += a * b
        out.append(np.asarray(v[o:o + b], dtype=np.float64).copy())
        o += b
    return out


def winner_z(J: np.ndarray, group: np.ndarray, winner: dict) -> dict:
    """Fallback statistic per group (instance): the z-score of the winner's
    objective among the objectives of every refined bucket of the group,
    (J_w - mean) / sd with the population deviation; 0 when sd = 0; -inf
    for a group without a winner.  winner maps group -> index into J."""
    out = {}
    for gval in np.unique(group):
        v = J[group == gval]
        w = winner.get(gval, -1)
        if w is None or w < 0:
            out[gval] = -math.inf
            continue
        mu = v.mean()
        sd = math.sqrt(np.mean((v - mu) ** 2))
        out[gval] = (J[w] - mu) / sd if sd > 0 else 0.0
    return out
