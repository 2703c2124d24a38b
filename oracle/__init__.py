"""CPU oracle for the PROJECTION hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 reference written from the paper ("PROJECTION Algorithm
for Motif Finding on GPUs", Clemente, Cabarle, Adorna).  Only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the GPU path: its arithmetic lives in ``oracle.c`` (built by
``oracle/build.py`` with gcc) and in the pure-Python brute-force checks of
``oracle/brute.py``.  This module only marshals numpy arrays into that C code.

Every function of the C side is pinned by ``tests/test_oracle_*.py`` against
values the paper prints, closed forms, invariants and brute force on tiny
inputs.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

_i32, _i64, _u32, _u64, _dbl = C.c_int, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
_P = C.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.or_encode.restype = _i64
        L.or_encode.argtypes = [_i32, C.c_char_p, _i64, _P]
        L.or_num_windows.restype = _i64
        L.or_num_windows.argtypes = [_i32, _P, _i32]
        L.or_hash.restype = _i32
        L.or_hash.argtypes = [_i32, _i32, _P, _P, _i32, _i32, _P, _i32, _P, _P]
        L.or_select.restype = _i32
        L.or_select_sorted.restype = _i32
        L.or_select_sorted.argtypes = [_i32, _P, _i32, _P, _i32, _u32, _P, _i64, _P, _i64, _P]
        L.or_select.argtypes = [_i32, _P, _i32, _i32, _i32, _P, _P, _i32, _u32,
                                _P, _i64, _P, _i64, _P]
        L.or_profile.restype = None
        L.or_profile.argtypes = [_i32, _P, _P, _i32, _i32, _P, _i64, _P, _P]
        L.or_theta0.restype = None
        L.or_theta0.argtypes = [_i32, _i32, _P, _i64, _P, _dbl, _P]
        L.or_estep.restype = _dbl
        L.or_estep.argtypes = [_i32, _P, _P, _i32, _i32, _P, _P, _P, _P, _P]
        L.or_mstep.restype = None
        L.or_mstep.argtypes = [_i32, _P, _P, _i32, _i32, _P, _P, _dbl, _P]
        L.or_em.restype = None
        L.or_em.argtypes = [_i32, _P, _P, _i32, _i32, _P, _P, _i64, _i32, _dbl, _P, _P, _P, _P]
        L.or_estep_model.restype = _dbl
        L.or_estep_model.argtypes = [_i32, _dbl, _i32, _P, _P, _i32, _i32, _P, _P, _P, _P, _P]
        L.or_mstep_model.restype = None
        L.or_mstep_model.argtypes = [_i32, _i32, _P, _P, _i32, _i32, _P, _P, _dbl, _dbl, _P, _P]
        L.or_philox4x64.restype = None
        L.or_philox4x64.argtypes = [_P, _P, _P]
        L.or_gibbs_uniform.restype = _dbl
        L.or_gibbs_uniform.argtypes = [_u64, _i32, _i32, _i64]
        L.or_gibbs_weights.restype = None
        L.or_gibbs_weights.argtypes = [_i32, _P, _P, _i32, _i32, _P, _dbl, _P, _i32, _P]
        L.or_alignment_score.restype = _dbl
        L.or_alignment_score.argtypes = [_i32, _P, _P, _i32, _i32, _P, _dbl, _P, _P]
        L.or_gibbs.restype = _i32
        L.or_gibbs.argtypes = [_i32, _P, _P, _i32, _i32, _P, _P, _i64, _i32, _dbl, _u64, _P, _P, _P]
        L.or_em_model.restype = None
        L.or_em_model.argtypes = [_i32, _dbl, _i32, _P, _P, _i32, _i32, _P, _P, _i64, _i32, _dbl, _P, _P, _P,
                                  _P, _P]
        L.or_best.restype = _i64
        L.or_best.argtypes = [_P, _i64, _i32, _P, _i32, _i32, C.c_char_p]
        L.or_parkmiller.restype = _u32
        L.or_parkmiller.argtypes = [_u64, _i32]
        L.or_masks.restype = None
        L.or_masks.argtypes = [_u64, _i32, _i32, _i32, _P]
        L.or_letter.restype = C.c_char
        L.or_letter.argtypes = [_i32, _i32]
        L.or_set_threads.restype = _i32
        L.or_set_threads.argtypes = [_i32]
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops (n <= 0: unchanged); returns the
    number in use."""
    return int(lib().or_set_threads(n))


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def alphabet_size(alphabet) -> int:
    if alphabet in (4, "dna", "DNA"):
        return 4
    if alphabet in (20, "protein", "PROTEIN"):
        return 20
    raise ValueError(alphabet)


def letters(A: int) -> str:
    """Letters in code order (code c is letters(A)[c])."""
    return "".join(lib().or_letter(A, c).decode() for c in range(A))


# --------------------------------------------------------------------------
class Seqs:
    """Encoded sequences: codes (uint8, concatenated) and offsets (int64, t+1)."""

    def __init__(self, A: int, seqs: Sequence[str]):
        self.A = A
        self.t = len(seqs)
        self.lens = np.array([len(s) for s in seqs], dtype=np.int64)
        self.off = np.zeros(self.t + 1, dtype=np.int64)
        self.off[1:] = np.cumsum(self.lens)
        raw = "".join(seqs).encode("ascii")
        self.codes = np.zeros(max(len(raw), 1), dtype=np.uint8)
        bad = lib().or_encode(A, raw, len(raw), _p(self.codes))
        if bad >= 0:
            raise ValueError(f"symbol {raw[bad:bad+1]!r} at {bad} is not in the alphabet")

    def nwin(self, l: int) -> int:
        return int(lib().or_num_windows(self.t, _p(self.off), l))

    def window_site(self, l: int, w: int):
        L = self.lens - l + 1
        cum = np.concatenate([[0], np.cumsum(L)])
        i = int(np.searchsorted(cum, w, side="right") - 1)
        return i, int(w - cum[i])


def hash_trials(S: Seqs, l: int, k: int, masks: np.ndarray, keys: bool = True,
                counts: bool = True):
    masks = np.ascontiguousarray(masks, dtype=np.uint32)
    m = len(masks)
    x = S.nwin(l)
    nb = S.A ** k
    K = np.zeros((m, x), dtype=np.uint32) if keys else None
    N = np.zeros((m, nb), dtype=np.uint32) if counts else None
    if lib().or_hash(S.A, S.t, _p(S.off), _p(S.codes), l, k, _p(masks), m, _p(K), _p(N)) != 0:
        raise ValueError("every mask must keep exactly k of the l positions")
    return K, N


def select(S: Seqs, l: int, k: int, keys: np.ndarray, counts: np.ndarray, s: int,
           cap_b: int | None = None, cap_m: int | None = None):
    m = keys.shape[0]
    if cap_b is None or cap_m is None:
        n = np.zeros(2, dtype=np.int64)
        lib().or_select(S.t, _p(S.off), l, S.A, k, _p(keys), _p(counts), m, s,
                        None, 0, None, 0, _p(n))
        cap_b = int(n[0]) if cap_b is None else cap_b
        cap_m = int(n[1]) if cap_m is None else cap_m
    bk = np.zeros((max(cap_b, 1), 4), dtype=np.uint32)
    mem = np.zeros(max(cap_m, 1), dtype=np.uint32)
    n = np.zeros(2, dtype=np.int64)
    rc = lib().or_select(S.t, _p(S.off), l, S.A, k, _p(keys), _p(counts), m, s,
                         _p(bk), cap_b, _p(mem), cap_m, _p(n))
    nb_, nm_ = int(n[0]), int(n[1])
    return bk[:min(nb_, cap_b)], mem[:min(nm_, cap_m)], (nb_, nm_), rc


def select_sorted(S: Seqs, l: int, keys: np.ndarray, s: int):
    """Enriched buckets of every trial from its keys alone (no count table):
    (key, window) pairs sorted per trial, runs of at least s equal keys.
    Same output as select()."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    m = keys.shape[0]
    n = np.zeros(2, dtype=np.int64)
    rc = lib().or_select_sorted(S.t, _p(S.off), l, _p(keys), m, s, None, 0, None, 0, _p(n))
    if rc == -2:
        raise MemoryError("or_select_sorted")
    cap_b, cap_m = int(n[0]), int(n[1])
    bk = np.zeros((max(cap_b, 1), 4), dtype=np.uint32)
    mem = np.zeros(max(cap_m, 1), dtype=np.uint32)
    rc = lib().or_select_sorted(S.t, _p(S.off), l, _p(keys), m, s, _p(bk), cap_b, _p(mem), cap_m, _p(n))
    return bk[:cap_b], mem[:cap_m], (int(n[0]), int(n[1])), rc


def profile(S: Seqs, l: int, bk: np.ndarray, members: np.ndarray) -> np.ndarray:
    bk = np.ascontiguousarray(bk, dtype=np.uint32)
    out = np.zeros((len(bk), S.A, l), dtype=np.uint32)
    lib().or_profile(S.t, _p(S.off), _p(S.codes), l, S.A, _p(bk), len(bk),
                     _p(np.ascontiguousarray(members, dtype=np.uint32)), _p(out))
    return out


def theta0(prof: np.ndarray, bg: np.ndarray, beta: float) -> np.ndarray:
    prof = np.ascontiguousarray(prof, dtype=np.uint32)
    B, A, l = prof.shape
    out = np.zeros((B, A, l), dtype=np.float64)
    lib().or_theta0(A, l, _p(prof), B, _p(np.ascontiguousarray(bg, dtype=np.float64)),
                    float(beta), _p(out))
    return out


def estep(S: Seqs, l: int, theta: np.ndarray, bg: np.ndarray):
    """One E-step for one model: returns (llr, s[x], Z[x], lse[t])."""
    x = S.nwin(l)
    s = np.zeros(x, dtype=np.float64)
    Z = np.zeros(x, dtype=np.float64)
    lse = np.zeros(S.t, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    v = lib().or_estep(S.t, _p(S.off), _p(S.codes), l, S.A, _p(th),
                       _p(np.ascontiguousarray(bg, dtype=np.float64)), _p(s), _p(Z), _p(lse))
    return v, s, Z, lse


def mstep(S: Seqs, l: int, Z: np.ndarray, bg: np.ndarray, beta: float) -> np.ndarray:
    out = np.zeros((S.A, l), dtype=np.float64)
    lib().or_mstep(S.t, _p(S.off), _p(S.codes), l, S.A,
                   _p(np.ascontiguousarray(Z, dtype=np.float64)),
                   _p(np.ascontiguousarray(bg, dtype=np.float64)), float(beta), _p(out))
    return out


def em(S: Seqs, l: int, theta0_: np.ndarray, bg: np.ndarray, iters: int, beta: float):
    th0 = np.ascontiguousarray(theta0_, dtype=np.float64)
    B = th0.shape[0]
    th = np.zeros_like(th0)
    J = np.zeros((B, iters + 1))
    LL = np.zeros((B, iters + 1))
    sites = np.zeros((B, S.t), dtype=np.int32)
    lib().or_em(S.t, _p(S.off), _p(S.codes), l, S.A, _p(th0),
                _p(np.ascontiguousarray(bg, dtype=np.float64)), B, iters, float(beta),
                _p(th), _p(J), _p(LL), _p(sites))
    return th, J, LL, sites


OOPS, ZOOPS, TCM = 0, 1, 2


def estep_model(S: Seqs, l: int, model: int, mix: float, theta: np.ndarray, bg: np.ndarray):
    """One E-step of the OOPS, ZOOPS or TCM model: (LLR, s[x], Z[x], q[t])."""
    x = S.nwin(l)
    s = np.zeros(max(x, 1))
    Z = np.zeros(max(x, 1))
    q = np.zeros(max(S.t, 1))
    v = lib().or_estep_model(model, float(mix), S.t, _p(S.off), _p(S.codes), l, S.A,
                             _p(np.ascontiguousarray(theta, dtype=np.float64)),
                             _p(np.ascontiguousarray(bg, dtype=np.float64)), _p(s), _p(Z), _p(q))
    return float(v), s[:x], Z[:x], q[:S.t]


def mstep_model(S: Seqs, l: int, model: int, Z: np.ndarray, bg: np.ndarray, beta: float, mix: float):
    """The M-step of the model given posteriors Z: (theta', mix')."""
    th = np.zeros((S.A, l))
    mx = np.zeros(1)
    lib().or_mstep_model(model, S.t, _p(S.off), _p(S.codes), l, S.A, _p(np.ascontiguousarray(Z, dtype=np.float64)),
                         _p(np.ascontiguousarray(bg, dtype=np.float64)), float(beta), float(mix), _p(th), _p(mx))
    return th, float(mx[0])


def em_model(S: Seqs, l: int, model: int, mix0: float, theta0_: np.ndarray, bg: np.ndarray, iters: int,
             beta: float):
    """EM of the OOPS, ZOOPS or TCM model: (theta, mix, J, LLR, sites)."""
    th0 = np.ascontiguousarray(theta0_, dtype=np.float64)
    B = th0.shape[0]
    th = np.zeros_like(th0)
    mix = np.zeros(B)
    J = np.zeros((B, iters + 1))
    LL = np.zeros((B, iters + 1))
    sites = np.zeros((B, S.t), dtype=np.int32)
    lib().or_em_model(model, float(mix0), S.t, _p(S.off), _p(S.codes), l, S.A, _p(th0),
                      _p(np.ascontiguousarray(bg, dtype=np.float64)), B, iters, float(beta), _p(th), _p(mix),
                      _p(J), _p(LL), _p(sites))
    return th, mix, J, LL, sites


def best(J: np.ndarray, theta: np.ndarray):
    B, it1 = J.shape
    _, A, l = theta.shape
    buf = C.create_string_buffer(l + 1)
    b = lib().or_best(_p(np.ascontiguousarray(J)), B, it1 - 1,
                      _p(np.ascontiguousarray(theta)), A, l, buf)
    return int(b), buf.value.decode()


def parkmiller(seed: int, n: int) -> int:
    return int(lib().or_parkmiller(seed, n))


def masks_from_seed(seed: int, l: int, k: int, m: int) -> np.ndarray:
    out = np.zeros(m, dtype=np.uint32)
    lib().or_masks(seed, l, k, m, _p(out))
    return out


def bg_vector(A: int, bg: dict | None, S: Seqs | None = None) -> np.ndarray:
    """Background in code order: from a letter->frequency dict, else the
    composition of the input (reading: bg is fixed, never re-estimated)."""
    L = letters(A)
    if bg is not None:
        v = np.array([bg[c] for c in L], dtype=np.float64)
    else:
        v = np.bincount(S.codes[: int(S.off[-1])], minlength=A).astype(np.float64)
    return v / v.sum()


# --------------------------------------------------------------------------
# Sec. 5, choice of k, s and m when they are not given.
def p_hat(l: int, d: int, k: int) -> float:
    """Probability that a planted occurrence with d mutations is projected
    onto the planted bucket: C(l-d, k) / C(l, k)."""
    return math.comb(l - d, k) / math.comb(l, k)


def b_below(t_hat: int, p: float, s: int) -> float:
    """B_{t,p}(s): probability that fewer than s of t_hat occurrences land in
    the planted bucket in one trial (binomial lower tail)."""
    return sum(math.comb(t_hat, i) * p ** i * (1 - p) ** (t_hat - i) for i in range(s))


def auto_params(l: int, d: int, t: int, n_total_windows: int, A: int, q: float = 0.95):
    """k = l - d - 1; s = twice the mean bucket size t(n-l+1)/|Sigma|^k, but
    at least 3 (the paper: that mean is far below 1 for the challenge
    instances, where 3-4 is used); m = ceil(log(1-q) / log B(s))."""
    k = l - d - 1
    s = max(3, math.ceil(2.0 * n_total_windows / float(A) ** k))
    if s > t:
        raise ValueError("the threshold exceeds t: the planted bucket cannot pass")
    p = p_hat(l, d, k)
    # 1 - B(s) summed directly, so log B = log1p(-tail) stays accurate near 1
    tail = sum(math.comb(t, i) * p ** i * (1 - p) ** (t - i) for i in range(s, t + 1))
    m = 1 if tail >= 1 else max(1, math.ceil(math.log(1 - q) / math.log1p(-tail)))
    return k, s, m


# --------------------------------------------------------------------------
def run(seqs: Sequence[str], A: int, l: int, k: int, s: int, masks: np.ndarray, iters: int,
        beta: float = 1.0, beta0: float | None = None, bg: np.ndarray | None = None):
    """The whole path on one instance: hash, select, profile, theta0, EM, best."""
    S = Seqs(A, seqs)
    bgv = bg if bg is not None else bg_vector(A, None, S)
    keys, counts = hash_trials(S, l, k, masks)
    bk, mem, (nb_, nm_), _ = select(S, l, k, keys, counts, s)
    prof = profile(S, l, bk, mem)
    th0 = theta0(prof, bgv, beta if beta0 is None else beta0)
    th, J, LL, sites = em(S, l, th0, bgv, iters, beta)
    b, cons = best(J, th) if len(bk) else (-1, "")
    return dict(S=S, keys=keys, counts=counts, buckets=bk, members=mem, profile=prof,
                theta0=th0, theta=th, J=J, llr=LL, sites=sites, best=b, consensus=cons,
                bg=bgv)


def run_range(seqs: Sequence[str], A: int, l_minus: int, l_plus: int, d: int, seed: int, iters: int,
              beta: float = 1.0, bg: np.ndarray | None = None, k: int = 0, s: int = 0, m: int = 0):
    """A motif-length range (l-, l+) (Sec. 2): the whole path at every length,
    k, s, m from auto_params (Sec. 5) unless given, masks from the seeded
    Park-Miller tables (Sec. 6); the chosen length has the largest
    log-likelihood ratio per motif column, the longer on ties (the paper does
    not say how lengths compete).  Returns (per-length dicts, chosen l or -1)."""
    out = []
    S = Seqs(A, seqs)
    bgv = bg if bg is not None else bg_vector(A, None, S)
    for l in range(l_minus, l_plus + 1):
        x = S.nwin(l)
        ak, as_, am = auto_params(l, d, S.t, x, A) if (k <= 0 or s <= 0 or m <= 0) else (k, s, m)
        kk, ss, mm = (k if k > 0 else ak), (s if s > 0 else as_), (m if m > 0 else am)
        masks = masks_from_seed(seed, l, kk, mm)
        keys, counts = hash_trials(S, l, kk, masks, counts=float(A) ** kk <= 2 ** 22)
        if counts is not None:
            bk, mem, _, _ = select(S, l, kk, keys, counts, ss)
        else:
            bk, mem, _, _ = select_sorted(S, l, keys, ss)
        r = dict(l=l, k=kk, s=ss, m=mm, n_enriched=len(bk), consensus="", llr=-math.inf, J=-math.inf, best=-1)
        if len(bk):
            prof = profile(S, l, bk, mem)
            th0 = theta0(prof, bgv, beta)
            th, J, LL, sites = em(S, l, th0, bgv, iters, beta)
            b, cons = best(J, th)
            r.update(best=b, consensus=cons, llr=float(LL[b, -1]), J=float(J[b, -1]), theta=th[b],
                     sites=sites[b], bucket=bk[b])
        out.append(r)
    chosen, bv = -1, -math.inf
    for r in out:
        if r["best"] < 0:
            continue
        v = r["llr"] / r["l"]
        if chosen < 0 or v >= bv:
            chosen, bv = r["l"], v
    return out, chosen


# ------------------------------------------------------------ Gibbs sampling
def philox4x64(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64(_p(c), _p(k), _p(out))
    return out


def gibbs_uniform(seed: int, sweep: int, i: int, model: int) -> float:
    return float(lib().or_gibbs_uniform(seed, sweep, i, model))


def gibbs_weights(S: Seqs, l: int, bg: np.ndarray, beta: float, sites: np.ndarray, i: int) -> np.ndarray:
    """The sampler's conditional distribution of the start of sequence i."""
    L = int(S.off[i + 1] - S.off[i]) - l + 1
    w = np.zeros(L)
    lib().or_gibbs_weights(S.t, _p(S.off), _p(S.codes), l, S.A, _p(np.ascontiguousarray(bg, dtype=np.float64)),
                           float(beta), _p(np.ascontiguousarray(sites, dtype=np.int32)), i, _p(w))
    return w


def alignment_score(S: Seqs, l: int, bg: np.ndarray, beta: float, sites: np.ndarray):
    th = np.zeros((S.A, l))
    F = lib().or_alignment_score(S.t, _p(S.off), _p(S.codes), l, S.A,
                                 _p(np.ascontiguousarray(bg, dtype=np.float64)), float(beta),
                                 _p(np.ascontiguousarray(sites, dtype=np.int32)), _p(th))
    return float(F), th


def gibbs(S: Seqs, l: int, theta0_: np.ndarray, bg: np.ndarray, sweeps: int, beta: float, seed: int):
    """Gibbs refinement of every model: (theta, F [B][sweeps+1], sites)."""
    th0 = np.ascontiguousarray(theta0_, dtype=np.float64)
    B = th0.shape[0]
    th = np.zeros_like(th0)
    F = np.zeros((B, sweeps + 1))
    sites = np.zeros((B, S.t), dtype=np.int32)
    rc = lib().or_gibbs(S.t, _p(S.off), _p(S.codes), l, S.A, _p(th0), _p(np.ascontiguousarray(bg, dtype=np.float64)),
                        B, sweeps, float(beta), seed, _p(th), _p(F), _p(sites))
    if rc != 0:
        raise ValueError("Gibbs sampling needs beta > 0")
    return th, F, sites
