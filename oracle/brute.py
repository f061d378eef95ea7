"""Independent NumPy formulation of the trend test, for tiny inputs.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

It does not count violating pairs the way ``ebic_oracle.c`` does.  For the
exact case it uses the rank formulation of the Motivation's rule: a row
follows a series (p, q, r, ...) rising iff every successive difference of its
values along the series is positive, i.e. ``np.all(np.diff(v) > 0)``, and
falling iff every difference is negative.  For the approximate case it counts
the non-positive (resp. non-negative) differences -- the descents of v --
and compares with k.  NaN differences are neither positive nor negative, so
they break both directions, as a NaN comparison does.

Differences are taken in float64, where the sign of the difference of two
float32 values is always the sign of their exact difference (the difference
is 0 only when the values are equal).
"""
from __future__ import annotations

import itertools
import math
from typing import Iterable, List, Sequence

import numpy as np


def row_matches(v: np.ndarray, k: int):
    """(rising, falling) acceptance for one row's values along a series."""
    with np.errstate(invalid="ignore"):
        d = np.diff(np.asarray(v, dtype=np.float64))
        up_desc = int(np.count_nonzero(~(d > 0)))
        dn_desc = int(np.count_nonzero(~(d < 0)))
    return up_desc <= k, dn_desc <= k


def evaluate_series(a: np.ndarray, series: Sequence[int], k: int, negative: bool):
    """Per-row (rising, falling) boolean masks and the union count."""
    sub = np.asarray(a, dtype=np.float64)[:, list(series)]
    with np.errstate(invalid="ignore"):
        d = np.diff(sub, axis=1)
        up = np.count_nonzero(~(d > 0), axis=1) <= k
        dn = np.count_nonzero(~(d < 0), axis=1) <= k
    if not negative:
        dn = np.zeros_like(dn)
    return up, dn, int(np.count_nonzero(up | dn))


def evaluate_exact_rank(a: np.ndarray, series: Sequence[int]):
    """Exact (k = 0) rising/falling masks by the rank formulation only."""
    sub = np.asarray(a, dtype=np.float64)[:, list(series)]
    with np.errstate(invalid="ignore"):
        up = np.all(np.diff(sub, axis=1) > 0, axis=1)
        dn = np.all(np.diff(sub, axis=1) < 0, axis=1)
    return up, dn


def all_series(n_cols: int, max_len: int) -> Iterable[tuple]:
    """Every ordered series of distinct columns of length 1..max_len."""
    for L in range(1, max_len + 1):
        yield from itertools.permutations(range(n_cols), L)


def eulerian(n: int, k: int) -> int:
    """Eulerian number A(n, k): permutations of n with exactly k descents."""
    return sum((-1) ** j * math.comb(n + 1, j) * (k + 1 - j) ** n for j in range(k + 2))


def match_probability(L: int, k: int) -> float:
    """Chance that i.i.d. continuous values along an L-series rise with at
    most k descents: sum_{d <= k} A(L, d) / L!."""
    return sum(eulerian(L, d) for d in range(0, min(k, L - 1) + 1)) / math.factorial(L)


def masks_to_words(mask: np.ndarray) -> np.ndarray:
    """Pack a boolean row mask into uint64 words, bit r % 64 of word r // 64."""
    n = len(mask)
    w = (n + 63) // 64
    out = np.zeros(w, dtype=np.uint64)
    idx = np.nonzero(mask)[0]
    for r in idx:
        out[r // 64] |= np.uint64(1) << np.uint64(r % 64)
    return out


def series_list(offsets, cols) -> List[np.ndarray]:
    return [np.asarray(cols[offsets[i]:offsets[i + 1]]) for i in range(len(offsets) - 1)]
