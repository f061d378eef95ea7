"""Seeded synthetic inputs for the EBIC population evaluator.

This module builds the *inputs* that both the CPU oracle and the HIP path are
run on: expression-shaped FP32 matrices with planted order-preserving
biclusters, populations of candidate column series, their CBF packing, and a
few adversarial matrices (ties, NaN, signed zeros, infinities, denormals).

It holds none of the method's arithmetic: no trend test, no row counting and
no fitness.  Both sides import it; neither side is imported here.

Planting follows the paper's synthetic setting (Section 2.3: biclusters of a
given size implanted in a background matrix, with trend-preserving patterns)
and the shapes of its expression datasets (Table 1).  The concrete recipe
(draw order, noise-then-sort, overlap construction) is this project's reading
and is written out in the docstrings below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

__all__ = [
    "Planted",
    "Workload",
    "WORKLOADS",
    "make_matrix",
    "random_population",
    "planted_population",
    "mixed_population",
    "pack_cbf",
    "unpack_cbf",
    "adversarial_matrix",
    "tiny_tie_matrix",
    "batched_workload",
    "rows_to_masks",
]


@dataclass(frozen=True)
class Planted:
    """One planted bicluster: row set, ordered column series, direction."""

    rows: np.ndarray          # int64, sorted row indices
    cols: np.ndarray          # int64, the planted column order
    descending: bool          # True: values decrease along ``cols``


@dataclass(frozen=True)
class Workload:
    """A named synthetic workload: matrix recipe, trend and run parameters."""

    name: str
    n_rows: int
    n_cols: int
    seed: int
    background: str                      # "normal" or "lognormal"
    n_planted: int
    planted_rows: Tuple[int, int]        # inclusive range of planted row counts
    planted_cols: Tuple[int, int]        # inclusive range of planted series lengths
    noise_sd: float
    noise_then_sort: bool                # True: planted rows match exactly
    overlap_max: float                   # max pairwise row/col overlap fraction
    descending_every_other: bool
    # trend / fitness parameters
    sigma: int
    max_violations: int
    negative_trends: bool
    # evolution parameters
    population: int
    len_min: int
    len_max: int
    generations: int
    overlap: float = 0.5
    toplist: int = 100
    tournament: int = 3
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # 200x50 N(0,1), 3 planted 30x8 increasing, noise N(0,0.01) then sort,
    # positive exact trends, P=200, L in [3,8], 50 generations.
    "tiny": Workload(
        name="tiny", n_rows=200, n_cols=50, seed=0, background="normal",
        n_planted=3, planted_rows=(30, 30), planted_cols=(8, 8),
        noise_sd=0.01, noise_then_sort=True, overlap_max=0.0,
        descending_every_other=False,
        sigma=15, max_violations=0, negative_trends=False,
        population=200, len_min=3, len_max=8, generations=50),
    # 20000x200 log-normal(0,1), 10 planted, positive+negative, k=1,
    # P=2048, L in [3,20], 200 generations.
    "expression": Workload(
        name="expression", n_rows=20000, n_cols=200, seed=1,
        background="lognormal", n_planted=10, planted_rows=(100, 500),
        planted_cols=(5, 15), noise_sd=0.01, noise_then_sort=True,
        overlap_max=0.0, descending_every_other=True,
        sigma=50, max_violations=1, negative_trends=True,
        population=2048, len_min=3, len_max=20, generations=200),
    # 5000x1000 N(0,1), 20 planted with 0-50% pairwise overlap, half
    # descending, sorted then N(0,0.1) noise (approximate), P=4096,
    # L in [3,30], 300 generations.
    "wide": Workload(
        name="wide", n_rows=5000, n_cols=1000, seed=3, background="normal",
        n_planted=20, planted_rows=(50, 300), planted_cols=(4, 30),
        noise_sd=0.1, noise_then_sort=False, overlap_max=0.5,
        descending_every_other=True,
        sigma=25, max_violations=0, negative_trends=True,
        population=4096, len_min=3, len_max=30, generations=300),
    # 20000x500 log-normal, planted as "expression" (surrogate workload).
    "surrogate": Workload(
        name="surrogate", n_rows=20000, n_cols=500, seed=2,
        background="lognormal", n_planted=10, planted_rows=(100, 500),
        planted_cols=(5, 15), noise_sd=0.01, noise_then_sort=True,
        overlap_max=0.0, descending_every_other=True,
        sigma=50, max_violations=1, negative_trends=True,
        population=2048, len_min=3, len_max=20, generations=300),
}


def batched_workload(r: int, rows=(500, 50000), cols=(20, 1000), population: int = 1024,
                     generations: int = 100) -> Workload:
    """Run r of the batched setting: N log-uniform in ``rows``, M uniform in
    ``cols``, N(0,1) background, 1-10 exact rising biclusters of
    U{50..min(500, N/(2k))} rows x U{4..min(15, M/2)} columns, matrix seed r
    (shapes drawn from an independent stream keyed by r)."""
    import math
    rng = np.random.default_rng([4, int(r)])
    n = int(round(math.exp(rng.uniform(math.log(rows[0]), math.log(rows[1])))))
    m = int(rng.integers(cols[0], cols[1] + 1))
    k = int(rng.integers(1, 11))
    r_hi = max(2, min(500, n // (2 * k)))
    c_hi = max(2, min(15, m // 2))
    return Workload(
        name=f"batched-{r}", n_rows=n, n_cols=m, seed=int(r), background="normal",
        n_planted=k, planted_rows=(min(50, r_hi), r_hi), planted_cols=(min(4, c_hi), c_hi),
        noise_sd=0.01, noise_then_sort=True, overlap_max=0.0, descending_every_other=False,
        sigma=25, max_violations=0, negative_trends=False,
        population=population, len_min=3, len_max=min(20, m), generations=generations)


def _background(rng: np.random.Generator, kind: str, n: int, m: int) -> np.ndarray:
    if kind == "normal":
        return rng.standard_normal((n, m))
    if kind == "lognormal":
        return rng.lognormal(mean=0.0, sigma=1.0, size=(n, m))
    raise ValueError(f"unknown background {kind!r}")


def _has_adjacent_tie(v32: np.ndarray) -> bool:
    # Equal neighbours after the cast to float32 (the planted order would be
    # broken by a tie).  Pure data hygiene for the generator.
    return bool(np.any(v32[1:] == v32[:-1]))


def _choose_overlapping(rng, pool_size, size, partner, frac, exclude=None):
    """Pick ``size`` distinct indices from ``range(pool_size)``.

    ``round(frac * min(size, len(partner)))`` of them are taken from
    ``partner`` (overlap); the rest are fresh indices outside ``partner``
    (and outside ``exclude`` when given).
    """
    take = int(round(frac * min(size, len(partner)))) if partner is not None else 0
    chosen = []
    if take:
        chosen.extend(rng.choice(partner, size=take, replace=False).tolist())
    banned = set(chosen)
    if partner is not None:
        banned.update(np.asarray(partner).tolist())
    if exclude is not None:
        banned.update(exclude)
    free = np.setdiff1d(np.arange(pool_size), np.fromiter(banned, dtype=np.int64, count=len(banned)))
    need = size - len(chosen)
    chosen.extend(rng.choice(free, size=need, replace=False).tolist())
    return np.asarray(chosen, dtype=np.int64)


def make_matrix(w: Workload) -> Tuple[np.ndarray, List[Planted]]:
    """Build the FP32 row-major matrix of workload ``w`` and its planted truth.

    Draw order (all from ``numpy.random.default_rng(w.seed)``):
    background N x M; then per planted bicluster b: row count, series length,
    (if overlapping) partner and overlap fractions, rows, columns (in planted
    order), then per row the noise vector (redrawn until the FP32 values of
    the row along the series hold no tie, for noise-then-sort recipes).

    * noise-then-sort (exact): the row's background values on the series'
      columns plus N(0, sd) noise are sorted (ascending, or descending for a
      negative-trend bicluster) and written along the planted order.
    * sort-then-noise (approximate): the background values are sorted along
      the planted order first, then N(0, sd) noise is added.
    Rows of non-overlapping workloads are disjoint across biclusters;
    overlapping workloads take up to ``overlap_max`` of a random earlier
    bicluster's rows and columns, later biclusters overwriting shared cells.
    """
    rng = np.random.default_rng(w.seed)
    a = _background(rng, w.background, w.n_rows, w.n_cols)
    planted: List[Planted] = []
    used_rows: set = set()
    for b in range(w.n_planted):
        nr = int(rng.integers(w.planted_rows[0], w.planted_rows[1] + 1))
        nc = int(rng.integers(w.planted_cols[0], w.planted_cols[1] + 1))
        nc = min(nc, w.n_cols)
        nr = min(nr, w.n_rows)
        if w.overlap_max > 0.0 and b > 0:
            p = planted[int(rng.integers(0, b))]
            fr = float(rng.uniform(0.0, w.overlap_max))
            fc = float(rng.uniform(0.0, w.overlap_max))
            rows = _choose_overlapping(rng, w.n_rows, nr, p.rows, fr)
            cols = _choose_overlapping(rng, w.n_cols, nc, p.cols, fc)
            cols = rng.permutation(cols)
        else:
            free = np.setdiff1d(np.arange(w.n_rows), np.fromiter(used_rows, dtype=np.int64, count=len(used_rows)))
            rows = rng.choice(free, size=nr, replace=False).astype(np.int64)
            cols = rng.choice(w.n_cols, size=nc, replace=False).astype(np.int64)
        used_rows.update(rows.tolist())
        desc = bool(w.descending_every_other and (b % 2 == 1))
        for r in rows:
            base = a[r, cols]
            if w.noise_then_sort:
                while True:
                    v = np.sort(base + rng.normal(0.0, w.noise_sd, size=nc))
                    if desc:
                        v = v[::-1]
                    v32 = v.astype(np.float32)
                    if not _has_adjacent_tie(v32):
                        break
                a[r, cols] = v32
            else:
                v = np.sort(base)
                if desc:
                    v = v[::-1]
                a[r, cols] = v + rng.normal(0.0, w.noise_sd, size=nc)
        planted.append(Planted(rows=np.sort(rows), cols=cols, descending=desc))
    return np.ascontiguousarray(a.astype(np.float32)), planted


def random_population(rng: np.random.Generator, n_cols: int, p: int,
                      len_min: int, len_max: int) -> List[np.ndarray]:
    """``p`` series, each of U{len_min..len_max} distinct random columns."""
    out = []
    for _ in range(p):
        L = int(rng.integers(len_min, len_max + 1))
        out.append(rng.choice(n_cols, size=min(L, n_cols), replace=False).astype(np.int32))
    return out


def planted_population(rng: np.random.Generator, planted: Sequence[Planted], p: int,
                       len_min: int) -> List[np.ndarray]:
    """``p`` order-preserving subsequences of planted series.

    Each draw picks a planted bicluster, a length in [min(len_min, L), L], a
    sorted random subset of positions, and with probability 1/2 reverses the
    result (so it follows the opposite direction).  These candidates keep
    many rows matching to the end of the series, the slow case for any
    evaluator that exits early.
    """
    out = []
    for _ in range(p):
        pb = planted[int(rng.integers(0, len(planted)))]
        L = len(pb.cols)
        lo = min(len_min, L)
        n = int(rng.integers(lo, L + 1))
        pos = np.sort(rng.choice(L, size=n, replace=False))
        s = pb.cols[pos].astype(np.int32)
        if rng.random() < 0.5:
            s = s[::-1].copy()
        out.append(s)
    return out


def mixed_population(rng: np.random.Generator, w: Workload, planted: Sequence[Planted],
                     p: int, planted_frac: float = 0.25) -> List[np.ndarray]:
    """Random series with a ``planted_frac`` share of planted subsequences,
    interleaved in a seeded random order."""
    n_pl = int(round(planted_frac * p)) if planted else 0
    pop = random_population(rng, w.n_cols, p - n_pl, w.len_min, w.len_max)
    if n_pl:
        pop += planted_population(rng, planted, n_pl, w.len_min)
    order = rng.permutation(len(pop))
    return [pop[i] for i in order]


def pack_cbf(series: Sequence[Sequence[int]]) -> Tuple[np.ndarray, np.ndarray]:
    """Pack series into the Compressed Bicluster Format (Fig. 2): an offsets
    array of P+1 start positions (with the total as sentinel) and the
    concatenated 0-based column indices."""
    offsets = np.zeros(len(series) + 1, dtype=np.int32)
    lens = np.fromiter((len(s) for s in series), dtype=np.int64, count=len(series))
    if len(series):
        offsets[1:] = np.cumsum(lens)
    cols = (np.concatenate([np.asarray(s, dtype=np.int32) for s in series])
            if len(series) else np.zeros(0, dtype=np.int32))
    return offsets, np.ascontiguousarray(cols, dtype=np.int32)


def unpack_cbf(offsets: np.ndarray, cols: np.ndarray) -> List[np.ndarray]:
    return [np.asarray(cols[offsets[i]:offsets[i + 1]]) for i in range(len(offsets) - 1)]


def adversarial_matrix(rng: np.random.Generator, n_rows: int, n_cols: int) -> np.ndarray:
    """A matrix full of the values that make strict comparisons subtle.

    Values come from a small pool: small integers (many ties), +0 and -0,
    +-inf, NaN, the smallest denormals of both signs, the largest finite
    values, and ordinary normals.
    """
    f32 = np.float32
    pool = np.array([
        0.0, -0.0, 1.0, -1.0, 2.0, np.inf, -np.inf, np.nan,
        np.float32(1e-45), -np.float32(1e-45), np.float32(3e-45),
        np.finfo(f32).max, -np.finfo(f32).max, np.finfo(f32).tiny,
        0.5, 3.0,
    ], dtype=f32)
    kind = rng.integers(0, 3, size=(n_rows, n_cols))
    pool_vals = pool[rng.integers(0, len(pool), size=(n_rows, n_cols))]
    ints = rng.integers(0, 3, size=(n_rows, n_cols)).astype(f32)
    normals = rng.standard_normal((n_rows, n_cols)).astype(f32)
    out = np.where(kind == 0, pool_vals, np.where(kind == 1, ints, normals))
    return np.ascontiguousarray(out.astype(f32))


def tiny_tie_matrix(rng: np.random.Generator, n_rows: int, n_cols: int,
                    special_rows: bool = True) -> np.ndarray:
    """Integer-valued FP32 matrix with values in {0,1,2} (tie-heavy), with
    optional extra rows holding NaN, signed zeros and infinities."""
    a = rng.integers(0, 3, size=(n_rows, n_cols)).astype(np.float32)
    if special_rows and n_rows >= 4:
        specials = np.array([np.nan, -0.0, 0.0, np.inf, -np.inf, 1.0], dtype=np.float32)
        for r in range(min(4, n_rows)):
            a[r] = specials[rng.integers(0, len(specials), size=n_cols)]
    return np.ascontiguousarray(a)


def rows_to_masks(rows_list: Sequence[Sequence[int]], n_rows: int) -> np.ndarray:
    """Pack row sets into 64-row words: uint64 [K][W], bit r % 64 of word
    r // 64 (the layout of the evaluator's row masks)."""
    W = (n_rows + 63) // 64
    out = np.zeros((len(rows_list), W), dtype=np.uint64)
    for k, rows in enumerate(rows_list):
        r = np.asarray(rows, dtype=np.int64)
        if r.size:
            np.bitwise_or.at(out[k], r // 64, np.left_shift(np.uint64(1), (r % 64).astype(np.uint64)))
    return out
