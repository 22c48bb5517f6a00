"""Seeded synthetic inputs for the symmetric tridiagonal eigenvalue problem.

This module is shared by the CPU oracle, the tests and the benchmark. It only
draws and lays out numbers; it holds none of the eigenvalue method's arithmetic.

Every array comes from ``numpy.random.Generator(PCG64(SeedSequence(key)))`` with
``key = [2605, 26599, cfg, fam, n, inst]`` so that each (configuration, family,
size, instance) has one reproducible input.

Families (a tridiagonal T is given by its diagonal d[0..n) and off-diagonal
e[0..n-1), e[i] coupling rows i and i+1):

* ``uniform``   d, e ~ U(-1, 1)
* ``normal``    d, e ~ N(0, 1)
* ``toeplitz``  d = 2, e = -1 (closed-form spectrum 2 - 2 cos(k pi/(n+1)))
* ``wilkinson`` W+: d_i = |i - (n-1)/2| (0-based i), e = 1
* ``clustered`` d_i = 10**(-8 + 8 i/(n-1)) (geometric in [1e-8, 1]),
                e = 1e-6 * U(0, 1); deflates heavily
* ``paper_uniform`` / ``paper_normal`` / ``paper_toeplitz`` / ``paper_clustered``:
  the families of the paper's experimental setup (Section 5.1), kept as
  optional presets: d ~ U[-1,1] or N(0,1) with e ~ U[0.1, 0.3]; Toeplitz d=2,
  e=0.25; clustered d_i = 1 + 1e-12 (i - (n+1)/2), e_i = 1e-4 (1 + 0.1 cos(0.33 i)).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_ROOT = (2605, 26599)

FAMILIES = (
    "uniform",
    "normal",
    "toeplitz",
    "wilkinson",
    "clustered",
    "paper_uniform",
    "paper_normal",
    "paper_toeplitz",
    "paper_clustered",
)
_FAM_ID = {name: i for i, name in enumerate(FAMILIES)}

# Configuration ids used in the seed key.
CFG_SMALL = 0      # n = 1024, uniform, leaf 32, 20 instances
CFG_FAMILIES = 1   # n in {16384, 32768, 65536} x 4 families
CFG_LARGE = 2      # n in {131072, 262144}, normal
CFG_BATCHED = 3    # 4096 problems, log-uniform sizes in [32, 4096]
CFG_GRAD = 4       # loss weights and inputs for differentiation
CFG_TEST = 9       # ad-hoc test inputs


def rng(cfg: int, fam: str | int, n: int, inst: int = 0) -> np.random.Generator:
    fam_id = _FAM_ID[fam] if isinstance(fam, str) else int(fam)
    ss = np.random.SeedSequence([SEED_ROOT[0], SEED_ROOT[1], int(cfg), fam_id, int(n), int(inst)])
    return np.random.Generator(np.random.PCG64(ss))


def tridiag(family: str, n: int, cfg: int = CFG_TEST, inst: int = 0):
    """Return (d, e) float64 arrays of lengths n and max(n-1, 0)."""
    n = int(n)
    m = max(n - 1, 0)
    g = rng(cfg, family, n, inst)
    i = np.arange(n, dtype=np.float64)
    if family == "uniform":
        d = g.uniform(-1.0, 1.0, n)
        e = g.uniform(-1.0, 1.0, m)
    elif family == "normal":
        d = g.standard_normal(n)
        e = g.standard_normal(m)
    elif family == "toeplitz":
        d = np.full(n, 2.0)
        e = np.full(m, -1.0)
    elif family == "wilkinson":
        d = np.abs(i - (n - 1) / 2.0)
        e = np.ones(m)
    elif family == "clustered":
        if n > 1:
            d = 10.0 ** (-8.0 + 8.0 * i / (n - 1))
        else:
            d = np.ones(n)
        e = 1e-6 * g.uniform(0.0, 1.0, m)
    elif family == "paper_uniform":
        d = g.uniform(-1.0, 1.0, n)
        e = g.uniform(0.1, 0.3, m)
    elif family == "paper_normal":
        d = g.standard_normal(n)
        e = g.uniform(0.1, 0.3, m)
    elif family == "paper_toeplitz":
        d = np.full(n, 2.0)
        e = np.full(m, 0.25)
    elif family == "paper_clustered":
        i1 = i + 1.0
        d = 1.0 + 1e-12 * (i1 - (n + 1) / 2.0)
        e = 1e-4 * (1.0 + 0.1 * np.cos(0.33 * i1[:m]))
    else:
        raise ValueError(f"unknown family {family!r}")
    return np.ascontiguousarray(d, dtype=np.float64), np.ascontiguousarray(e, dtype=np.float64)


def loss_weights(n: int, cfg: int = CFG_GRAD, inst: int = 0) -> np.ndarray:
    """w ~ N(0, 1) for the loss L = sum_k w_k lambda_k."""
    g = rng(cfg, 0, n, 1000 + inst)
    return g.standard_normal(int(n))


def batched_sizes(count: int = 4096, lo: int = 32, hi: int = 4096, cfg: int = CFG_BATCHED,
                  inst: int = 0) -> np.ndarray:
    """Sizes floor(exp(U[ln lo, ln(hi+1)))), i.e. log-uniform integers in [lo, hi]."""
    g = rng(cfg, 0, count, inst)
    u = g.uniform(math.log(lo), math.log(hi + 1), int(count))
    s = np.floor(np.exp(u)).astype(np.int64)
    return np.clip(s, lo, hi)


@dataclass
class Batch:
    """Packed batch: problem b owns d[off[b]:off[b+1]]; e uses the same offsets
    (slot off[b+1]-1 of e is unused padding, set to 0)."""

    d: np.ndarray
    e: np.ndarray
    offsets: np.ndarray

    @property
    def count(self) -> int:
        return len(self.offsets) - 1

    def problem(self, b: int):
        lo, hi = int(self.offsets[b]), int(self.offsets[b + 1])
        return self.d[lo:hi], self.e[lo:max(hi - 1, lo)]


def pack(problems) -> Batch:
    sizes = [len(d) for d, _ in problems]
    off = np.zeros(len(sizes) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    total = int(off[-1])
    d = np.zeros(total, dtype=np.float64)
    e = np.zeros(total, dtype=np.float64)
    for b, (db, eb) in enumerate(problems):
        lo = int(off[b])
        d[lo:lo + len(db)] = db
        e[lo:lo + len(eb)] = eb
    return Batch(d=d, e=e, offsets=off)


def batched(family: str = "uniform", count: int = 4096, lo: int = 32, hi: int = 4096,
            cfg: int = CFG_BATCHED, inst: int = 0) -> Batch:
    sizes = batched_sizes(count, lo, hi, cfg, inst)
    probs = [tridiag(family, int(s), cfg=cfg, inst=inst * 100000 + b) for b, s in enumerate(sizes)]
    return pack(probs)


def tnorm1(d: np.ndarray, e: np.ndarray) -> float:
    """max_i (|e_{i-1}| + |d_i| + |e_i|): the 1-norm (= inf-norm) of symmetric T."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    if d.size == 0:
        return 0.0
    s = np.abs(d).copy()
    if e.size:
        s[:-1] += np.abs(e)
        s[1:] += np.abs(e)
    return float(s.max())
