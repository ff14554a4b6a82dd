"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws strings and job descriptions; it holds none of the
alignment-plot arithmetic, so both the oracle's tests and the HIP path can use
it.  Every draw goes through ``numpy.random.Generator(PCG64(seed))``.

The paper measures on biological sequences (DNA/protein pairs of a few thousand
to 97k residues, Section 4) that are not available here; the paper notes that
the sequence content does not change the running time of the seaweed method.
The configurations below stand in for them:

* ``config(1)``  DNA pair, iid uniform ACGT, m = n = 1000, w = 16.
* ``config(2)``  DNA pair, m = n = 50,000, w = 64, iid ACGT background with 20
  planted homologous segments of length 2,000 copied from x into y (10%
  substitutions, 5% single-character indels); dot-plot threshold 48.
* ``config(3)``  protein pair (20 letters, background frequencies from a seeded
  Dirichlet(1) draw), m = n = 30,000, w = 128, 10 planted segments of length
  1,000 at 20% substitution.
* ``batch_config()``  256 iid DNA pairs, m, n uniform in [1000, 20000], w drawn
  from {16, 32, 64, 128}.
* ``serving_jobs()``  a Poisson stream of DNA/protein jobs, m and n
  log-uniform in [500, 50000], w in {16, 32, 64, 128}, threshold ceil(3w/4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DNA = b"ACGT"
PROTEIN = b"ACDEFGHIKLMNPQRSTVWY"
WS = (16, 32, 64, 128)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def iid(g: np.random.Generator, length: int, alphabet: bytes, p=None) -> np.ndarray:
    """length letters drawn independently from alphabet (uniform unless p)."""
    letters = np.frombuffer(alphabet, dtype=np.uint8)
    return letters[g.choice(len(letters), size=length, p=p)].astype(np.uint8)


def protein_background(seed: int = 3) -> np.ndarray:
    """Non-uniform amino-acid frequencies: one seeded Dirichlet(1) draw."""
    return rng(seed).dirichlet(np.ones(len(PROTEIN)))


def _mutate(g, seg: np.ndarray, alphabet: bytes, p, sub: float, ins: float, dele: float,
            length: int, background) -> np.ndarray:
    """Copy seg letter by letter: delete with prob dele, insert a random letter
    before it with prob ins, otherwise substitute a different letter with prob
    sub.  The result is cut or padded (with background letters) to length."""
    letters = np.frombuffer(alphabet, dtype=np.uint8)
    out = []
    for c in seg:
        u = g.random()
        if u < dele:
            continue
        if u < dele + ins:
            out.append(letters[g.choice(len(letters), p=p)])
            out.append(c)
            continue
        if g.random() < sub:
            others = [k for k in range(len(letters)) if letters[k] != c]
            q = None
            if p is not None:
                q = np.asarray([p[k] for k in others])
                q = q / q.sum()
            out.append(letters[others[g.choice(len(others), p=q)]])
        else:
            out.append(c)
    out = np.asarray(out[:length], dtype=np.uint8)
    if out.size < length:
        out = np.concatenate([out, background(length - out.size)])
    return out


def plant(g, x: np.ndarray, y: np.ndarray, nseg: int, seglen: int, alphabet: bytes, p,
          sub: float, ins: float, dele: float) -> list:
    """Copy nseg segments of length seglen from x into y, mutated.

    x and y are cut into nseg equal slots; segment s comes from slot s of x and
    lands in slot perm[s] of y, with perm a random derangement (so no segment
    sits on the main diagonal), each at a random offset inside its slot.
    Returns the (x_start, y_start) pairs."""
    slot_x, slot_y = x.size // nseg, y.size // nseg
    assert slot_x >= seglen and slot_y >= seglen
    while True:
        perm = g.permutation(nseg)
        if nseg == 1 or not np.any(perm == np.arange(nseg)):
            break
    placed = []
    for s in range(nseg):
        xs = s * slot_x + int(g.integers(0, slot_x - seglen + 1))
        ys = int(perm[s]) * slot_y + int(g.integers(0, slot_y - seglen + 1))
        seg = _mutate(g, x[xs:xs + seglen], alphabet, p, sub, ins, dele, seglen,
                      lambda k: iid(g, k, alphabet, p))
        y[ys:ys + seglen] = seg
        placed.append((xs, ys))
    return placed


@dataclass
class Pair:
    name: str
    x: np.ndarray
    y: np.ndarray
    w: int
    alphabet: bytes
    threshold: int | None = None
    planted: list = field(default_factory=list)

    @property
    def m(self) -> int:
        return int(self.x.size)

    @property
    def n(self) -> int:
        return int(self.y.size)


def config(k: int, seed: int | None = None, scale: float = 1.0) -> Pair:
    """Single-pair configurations 1-3 (see module docstring).  scale < 1 shrinks
    the string lengths (and planted segments) proportionally for quick tests."""
    seed = k if seed is None else seed
    g = rng(seed)
    if k == 1:
        m = n = max(int(1000 * scale), 17)
        return Pair("dna-1k-w16", iid(g, m, DNA), iid(g, n, DNA), 16, DNA)
    if k == 2:
        m = n = max(int(50_000 * scale), 4000)
        x, y = iid(g, m, DNA), iid(g, n, DNA)
        seglen = max(int(2000 * scale), 100)
        placed = plant(g, x, y, 20 if m >= 20 * seglen else max(m // (seglen + 500), 1), seglen,
                       DNA, None, 0.10, 0.025, 0.025)
        return Pair("dna-50k-w64-planted", x, y, 64, DNA, 48, placed)
    if k == 3:
        p = protein_background(3 if seed == 3 else seed)
        m = n = max(int(30_000 * scale), 3000)
        x, y = iid(g, m, PROTEIN, p), iid(g, n, PROTEIN, p)
        seglen = max(int(1000 * scale), 200)
        placed = plant(g, x, y, 10 if m >= 10 * (seglen + 500) else max(m // (seglen + 500), 1),
                       seglen, PROTEIN, p, 0.20, 0.0, 0.0)
        return Pair("protein-30k-w128-planted", x, y, 128, PROTEIN, None, placed)
    raise ValueError(f"no single-pair configuration {k}")


def batch_config(seed: int = 4, npairs: int = 256, lo: int = 1000, hi: int = 20000,
                 ws=WS) -> list:
    """256 independent iid DNA pairs of uneven sizes and windows."""
    g = rng(seed)
    pairs = []
    for q in range(npairs):
        m, n = int(g.integers(lo, hi + 1)), int(g.integers(lo, hi + 1))
        w = int(ws[int(g.integers(0, len(ws)))])
        pairs.append(Pair(f"batch-{q}", iid(g, m, DNA), iid(g, n, DNA), w, DNA))
    return pairs


@dataclass
class Job:
    jid: int
    arrival: float          # seconds after the stream starts
    pair: Pair
    threshold: int


def serving_jobs(rate: float, njobs: int = 2000, seed: int = 5, lo: int = 500,
                 hi: int = 50_000, ws=WS) -> list:
    """Poisson arrivals at `rate` jobs/s; half DNA, half protein (the protein
    background of configuration 3); m, n log-uniform in [lo, hi]; w uniform
    over ws; threshold ceil(3w/4)."""
    g = rng(seed)
    p = protein_background(3)
    t = 0.0
    jobs = []
    for q in range(njobs):
        t += float(g.exponential(1.0 / rate))
        protein = bool(g.random() < 0.5)
        m = int(math.floor(math.exp(g.uniform(math.log(lo), math.log(hi + 1)))))
        n = int(math.floor(math.exp(g.uniform(math.log(lo), math.log(hi + 1)))))
        w = int(ws[int(g.integers(0, len(ws)))])
        alpha, pp = (PROTEIN, p) if protein else (DNA, None)
        pair = Pair(f"job-{q}", iid(g, m, alpha, pp), iid(g, n, alpha, pp), w, alpha)
        jobs.append(Job(q, t, pair, int(math.ceil(3 * w / 4))))
    return jobs


def random_pair(seed: int, m: int, n: int, w: int, alphabet: bytes = DNA) -> Pair:
    g = rng(seed)
    return Pair(f"rand-{seed}", iid(g, m, alphabet), iid(g, n, alphabet), w, alphabet)
