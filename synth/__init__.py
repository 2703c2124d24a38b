"""Seeded synthetic inputs for planted (l,d)-motif finding.

This module only draws random strings and random position subsets.  It holds
none of the motif-finding arithmetic (no symbol codes, keys, counts, profiles or
likelihoods), so both the CPU oracle and the GPU path can take their inputs from
it without sharing any part of the method.

Workload recipe (paper Sec. 2, the (l,d) variant; Sec. 5, challenge instances
with t = 20, n = 600):

* background symbols are drawn i.i.d. from ``bg`` (uniform for DNA; a
  Dirichlet(2 * 1_20) draw for protein);
* the consensus M is drawn uniformly from Sigma^l;
* every sequence receives one copy of M at a uniform start in [0, n - l],
  with exactly d distinct positions, chosen uniformly, each replaced by a
  uniformly chosen *different* letter (Hamming distance exactly d);
* projection tables are uniform k-subsets of the l window positions, drawn
  from their own stream (bit p of a mask set means position p is kept).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence

import numpy as np

DNA_LETTERS = "ACGT"
# The twenty standard amino acids.  Only used to draw letters; the code order
# each side uses for keys lives on that side.
PROTEIN_LETTERS = "ARNDCQEGHILKMFPSTWYV"


@dataclass
class Instance:
    seqs: List[str]
    motif: str
    starts: List[int]          # 0-based start of the planted copy in each sequence
    l: int
    d: int
    letters: str               # alphabet letters (draw order, not code order)
    bg: Dict[str, float]       # background frequency per letter
    meta: dict = field(default_factory=dict)

    @property
    def t(self) -> int:
        return len(self.seqs)


def _letters(alphabet: str) -> str:
    if alphabet in ("dna", "DNA", 4):
        return DNA_LETTERS
    if alphabet in ("protein", "PROTEIN", 20):
        return PROTEIN_LETTERS
    raise ValueError(f"unknown alphabet {alphabet!r}")


def planted_instance(rng: np.random.Generator, t: int, n, l: int, d: int,
                     alphabet: str = "dna", bg: Dict[str, float] | None = None,
                     dirichlet_alpha: float | None = None) -> Instance:
    """Draw one planted (l,d) instance.

    ``n`` is an int (all sequences that long) or a sequence of t lengths.
    ``bg``: explicit background; else uniform, or Dirichlet(alpha * 1) when
    ``dirichlet_alpha`` is given.
    """
    letters = _letters(alphabet)
    A = len(letters)
    if isinstance(n, (int, np.integer)):
        lens = [int(n)] * t
    else:
        lens = [int(v) for v in n]
        assert len(lens) == t
    if bg is None:
        if dirichlet_alpha is not None:
            p = rng.dirichlet(np.full(A, float(dirichlet_alpha)))
        else:
            p = np.full(A, 1.0 / A)
    else:
        p = np.array([bg[c] for c in letters], dtype=np.float64)
        p = p / p.sum()
    if not 0 <= d <= l:
        raise ValueError("need 0 <= d <= l")
    motif_idx = rng.integers(0, A, size=l)
    motif = "".join(letters[i] for i in motif_idx)
    seqs, starts = [], []
    for i in range(t):
        ni = lens[i]
        if ni < l:
            raise ValueError("sequence shorter than the motif")
        s = rng.choice(A, size=ni, p=p)
        a = int(rng.integers(0, ni - l + 1))
        copy = motif_idx.copy()
        pos = rng.choice(l, size=d, replace=False)
        for q in pos:
            shift = int(rng.integers(1, A))          # a different letter
            copy[q] = (copy[q] + shift) % A
        s[a:a + l] = copy
        seqs.append("".join(letters[j] for j in s))
        starts.append(a)
    return Instance(seqs=seqs, motif=motif, starts=starts, l=l, d=d,
                    letters=letters, bg={c: float(v) for c, v in zip(letters, p)})


def projection_masks(rng: np.random.Generator, l: int, k: int, m: int) -> np.ndarray:
    """m uniform k-subsets of {0..l-1} as uint32 bit masks (bit p = kept).

    The l-k excluded positions are drawn without replacement, as in the
    paper's host-side generation of the positions not to project (Sec. 6).
    """
    if not (1 <= k <= l <= 32):
        raise ValueError("need 1 <= k <= l <= 32")
    full = (1 << l) - 1
    out = np.empty(m, dtype=np.uint32)
    for j in range(m):
        excl = rng.choice(l, size=l - k, replace=False)
        mask = full
        for p in excl:
            mask &= ~(1 << int(p))
        out[j] = mask
    return out


# ---------------------------------------------------------------------------
# The five workloads.  Each returns (instances, per-instance parameters).
# ---------------------------------------------------------------------------

CONFIGS = {
    # plain (15,4) DNA, t=20, n=600, k=7, s=4, m=200, 5 EM iterations, FP64
    "c1": dict(alphabet="dna", t=20, n=600, l=15, d=4, k=7, s=4, m=200, iters=5),
    # plain at scale (18,6) DNA, t=20, n=1000, k=8, s=4, m=5000, 10 EM iterations
    "c2": dict(alphabet="dna", t=20, n=1000, l=18, d=6, k=8, s=4, m=5000, iters=10),
    # protein (20,6), Dirichlet(2) background, t=30, n=1000, k=4, s=3, m=2000
    "c4": dict(alphabet="protein", t=30, n=1000, l=20, d=6, k=4, s=3, m=2000, iters=5,
               dirichlet_alpha=2.0),
    # (21,7) DNA, t=50, n=2000, k=9, s=3, m=10000
    "c5": dict(alphabet="dna", t=50, n=2000, l=21, d=7, k=9, s=3, m=10000, iters=5),
}


def make_config(name: str, seed: int, m: int | None = None, **override):
    """One instance of a fixed-shape workload plus its mask table."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    if m is not None:
        cfg["m"] = m
    ss = np.random.SeedSequence([seed, sum(map(ord, name))])
    inst_ss, mask_ss = ss.spawn(2)
    inst = planted_instance(np.random.default_rng(inst_ss), cfg["t"], cfg["n"], cfg["l"],
                            cfg["d"], cfg["alphabet"],
                            dirichlet_alpha=cfg.get("dirichlet_alpha"))
    masks = projection_masks(np.random.default_rng(mask_ss), cfg["l"], cfg["k"], cfg["m"])
    inst.meta.update(cfg)
    return inst, masks


def batch_config(seed: int, count: int = 512, m: int = 1000):
    """Uneven DNA batch: t~U[10,40], n~U[300,2000], l~U[11,21],
    d = floor(l/4)+1, k = clamp(l-d-4, 6, 9), s = 3."""
    ss = np.random.SeedSequence([seed, 3])
    out = []
    for child in ss.spawn(count):
        shape_ss, inst_ss, mask_ss = child.spawn(3)
        r = np.random.default_rng(shape_ss)
        t = int(r.integers(10, 41))
        n = int(r.integers(300, 2001))
        l = int(r.integers(11, 22))
        d = l // 4 + 1
        k = min(max(l - d - 4, 6), 9)
        inst = planted_instance(np.random.default_rng(inst_ss), t, n, l, d, "dna")
        masks = projection_masks(np.random.default_rng(mask_ss), l, k, m)
        inst.meta.update(dict(alphabet="dna", t=t, n=n, l=l, d=d, k=k, s=3, m=m, iters=5))
        out.append((inst, masks))
    return out


def random_sequences(rng: np.random.Generator, t: int, lens: Sequence[int] | int,
                     alphabet: str = "dna") -> List[str]:
    """Plain i.i.d. uniform sequences (no motif), for edge-case tests."""
    letters = _letters(alphabet)
    if isinstance(lens, (int, np.integer)):
        lens = [int(lens)] * t
    return ["".join(letters[j] for j in rng.integers(0, len(letters), size=ni)) for ni in lens]
