"""EBIC's evolutionary run (Steps 1-7), written out plainly in Python.

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

The paper gives the structure of the run (Section 2.2, Steps 1-7; the
crowding penalty 1.2^theta and the five genetic operations of Fig. 1 in
Section 2.1) but no constants or operator details.  Every choice below is a
reading, fixed so that two independent implementations can agree draw for
draw:

* Random numbers: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014).  ``uint(n)``
  is ``next() % n``.
* Step 1: each initial series has length Lmin + uint(Lmax - Lmin + 1) and
  distinct columns drawn by rejection, in draw order; a series already seen
  is redrawn whole (not a tabu hit).  The population is evaluated and the
  top-rank list is seeded by the Step 5 update.
* Step 2: the per-column penalty starts at zero each generation; the first
  min(|top|, floor(P * elite_num / elite_den)) top-rank entries are copied
  (with their scores) into the new population, each adding 1 to the penalty
  of each of its columns.
* Step 3: until the population is full: tournament selection of T draws
  with replacement from the previous population, the adjusted quality of a
  draw being fitness / 1.2^(sum of its columns' penalties / its length),
  the first best draw winning ties; one genetic operation chosen by weight
  (insert, delete, swap, substitute, crossover); a child already in the tabu
  list is a hit, and more than ``tabu_limit`` hits in one generation end the
  run (go to Step 6); a new child joins the population and the tabu list
  and adds 1 to its columns' penalties.
* Step 4: the new members are evaluated; elites keep their stored scores.
* Step 5: members in order of decreasing fitness (ties by position) with
  fitness > 0 and not already listed are admitted unless a listed entry of
  at least equal fitness overlaps them by more than theta; an admitted member
  evicts weaker entries it overlaps by more than theta.  Overlap is
  |x & e| / min(|x|, |e|) over column sets.  The list is then sorted by
  decreasing fitness (stable) and cut to K entries.
* Steps 6-7: the listed series are evaluated with the expansion parameters
  and their matching rows reported.

Mutations (Fig. 1a-d) are no-ops when not applicable (and then consume no
random numbers): insert needs L < Lmax (position uint(L+1), then a new column
by rejection), delete needs L > Lmin (position uint(L)), swap needs L >= 2
(i = uint(L), j = uint(L-1), j += 1 if j >= i), substitute needs L < M
(position uint(L), then a new column by rejection).  Crossover (Fig. 1e) is
one-point: i = 1 + uint(|a|), j = uint(|b|), child = a[:i] followed by the
columns of b[j:] not in a[:i], cut to Lmax; a child shorter than Lmin is a.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import evaluate as _oracle_evaluate

MASK64 = (1 << 64) - 1

OP_INSERT, OP_DELETE, OP_SWAP, OP_SUBSTITUTE, OP_CROSSOVER = range(5)


class SplitMix64:
    """SplitMix64 generator: a Weyl sequence with step 0x9E3779B97F4A7C15
    passed through a 64-bit finalizer (Steele, Lea & Flood 2014)."""

    GAMMA = 0x9E3779B97F4A7C15

    def __init__(self, seed: int):
        self.state = int(seed) & MASK64

    def next(self) -> int:
        self.state = (self.state + self.GAMMA) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uint(self, n: int) -> int:
        return self.next() % n


@dataclass
class TrendParams:
    sigma: int
    max_violations: int = 0
    negative_trends: bool = False


@dataclass
class EvolveParams:
    population: int
    len_min: int
    len_max: int
    tournament: int = 3
    op_weight: Tuple[int, int, int, int, int] = (1, 1, 1, 1, 1)
    elite_num: int = 1
    elite_den: int = 4
    penalty_base: float = 1.2
    overlap: float = 0.5
    toplist_size: int = 100
    tabu_limit: int = -1            # -1: the population size
    eval: TrendParams = field(default_factory=lambda: TrendParams(sigma=0))
    expand: TrendParams = field(default_factory=lambda: TrendParams(sigma=0))


@dataclass
class TopEntry:
    series: tuple
    count: int
    fitness: float


@dataclass
class Generation:
    gen: int
    population: List[tuple]
    counts: np.ndarray
    fitness: np.ndarray


@dataclass
class Result:
    biclusters: List[dict]          # cols, count, fitness, rows (bool mask)
    generations_run: int
    stopped_by_tabu: bool
    history: List[Generation]
    top: List[TopEntry]


def _evaluate(a, series: Sequence[tuple], tp: TrendParams, want_masks=False):
    offsets = np.zeros(len(series) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([len(s) for s in series])
    cols = np.array([c for s in series for c in s], dtype=np.int32)
    return _oracle_evaluate(a, offsets, cols, sigma=tp.sigma, max_violations=tp.max_violations,
                            negative_trends=tp.negative_trends, want_masks=want_masks)


def search_space(n_cols: int, len_min: int, len_max: int) -> int:
    """Number of distinct ordered series of distinct columns."""
    total = 0
    for L in range(len_min, len_max + 1):
        t = 1
        for i in range(L):
            t *= n_cols - i
        total += t
    return total


def check_params(p: EvolveParams, n_cols: int) -> None:
    if p.population < 1 or p.len_min < 1 or p.len_min > p.len_max or p.len_max > n_cols:
        raise ValueError("bad population or length bounds")
    if p.tournament < 1 or min(p.op_weight) < 0 or sum(p.op_weight) <= 0:
        raise ValueError("bad tournament or operation weights")
    if p.elite_den < 1 or not (0 <= p.elite_num <= p.elite_den) or p.toplist_size < 1:
        raise ValueError("bad elitism or top-list size")
    if not (p.penalty_base > 0.0) or not (0.0 <= p.overlap <= 1.0):
        raise ValueError("bad penalty base or overlap")
    if p.population > search_space(n_cols, p.len_min, p.len_max):
        raise ValueError("population larger than the number of distinct series")


def _overlap(sx: set, x: tuple, e: tuple) -> float:
    return len(sx.intersection(e)) / min(len(x), len(e))


def update_top(top: List[TopEntry], pop: Sequence[tuple], counts, fitness, theta: float,
               k_size: int) -> List[TopEntry]:
    """Step 5: top-rank list update."""
    order = sorted(range(len(pop)), key=lambda i: -float(fitness[i]))
    top = list(top)
    for i in order:
        x, fx = pop[i], float(fitness[i])
        if not fx > 0.0:
            continue
        if any(e.series == x for e in top):
            continue
        sx = set(x)
        if any(e.fitness >= fx and _overlap(sx, x, e.series) > theta for e in top):
            continue
        top = [e for e in top if not (e.fitness < fx and _overlap(sx, x, e.series) > theta)]
        top.append(TopEntry(series=x, count=int(counts[i]), fitness=fx))
    top.sort(key=lambda e: -e.fitness)
    return top[:k_size]


def _new_column(rng: SplitMix64, series: list, n_cols: int) -> int:
    while True:
        c = rng.uint(n_cols)
        if c not in series:
            return c


def mutate(rng: SplitMix64, s: list, op: int, p: EvolveParams, n_cols: int) -> list:
    L = len(s)
    if op == OP_INSERT:
        if L < p.len_max:
            pos = rng.uint(L + 1)
            s.insert(pos, _new_column(rng, s, n_cols))
    elif op == OP_DELETE:
        if L > p.len_min:
            del s[rng.uint(L)]
    elif op == OP_SWAP:
        if L >= 2:
            i = rng.uint(L)
            j = rng.uint(L - 1)
            if j >= i:
                j += 1
            s[i], s[j] = s[j], s[i]
    elif op == OP_SUBSTITUTE:
        if L < n_cols:
            pos = rng.uint(L)
            s[pos] = _new_column(rng, s, n_cols)
    return s


def crossover(rng: SplitMix64, a: tuple, b: tuple, p: EvolveParams) -> tuple:
    i = 1 + rng.uint(len(a))
    j = rng.uint(len(b))
    head = list(a[:i])
    child = head + [x for x in b[j:] if x not in head]
    child = child[:p.len_max]
    if len(child) < p.len_min:
        return tuple(a)
    return tuple(child)


def tournament(rng, prev: Sequence[tuple], prev_fit: Sequence[float], penalty: Sequence[int],
               size: int, base: float) -> int:
    """Step 3 selection with the crowding penalty of Section 2.1: ``size``
    draws i = uint(|prev|) with replacement; each draw's quality is its
    fitness divided by base^theta, theta being the mean penalty of its
    columns (their penalty sum over the series length); the first draw with
    the strictly highest quality wins."""
    best, best_adj = -1, float("-inf")
    for _ in range(size):
        i = rng.uint(len(prev))
        si = prev[i]
        vartheta = sum(penalty[c] for c in si) / len(si)
        adj = prev_fit[i] / (base ** vartheta)
        if adj > best_adj:
            best, best_adj = i, adj
    return best


def evolve(a: np.ndarray, seed: int, generations: int, p: EvolveParams,
           on_generation: Optional[Callable[[Generation], None]] = None,
           keep_history: bool = True) -> Result:
    """Run EBIC for ``generations`` iterations (generation 0 is Step 1)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    n_cols = a.shape[1]
    check_params(p, n_cols)

    def ev(series, tp):
        r = _evaluate(a, series, tp)
        return [int(x) for x in r["counts"]], [float(x) for x in r["fitness"]]

    P = p.population
    tabu_limit = P if p.tabu_limit < 0 else p.tabu_limit
    rng = SplitMix64(seed)
    tabu = set()
    history: List[Generation] = []

    def emit(g, pop, counts, fit):
        rec = Generation(g, list(pop), np.array(counts, dtype=np.int32), np.array(fit, dtype=np.float64))
        if keep_history:
            history.append(rec)
        if on_generation:
            on_generation(rec)

    # Step 1: initial population.
    pop: List[tuple] = []
    while len(pop) < P:
        L = p.len_min + rng.uint(p.len_max - p.len_min + 1)
        s: list = []
        while len(s) < L:
            c = rng.uint(n_cols)
            if c not in s:
                s.append(c)
        t = tuple(s)
        if t in tabu:
            continue
        pop.append(t)
        tabu.add(t)
    counts, fit = ev(pop, p.eval)
    emit(0, pop, counts, fit)
    top = update_top([], pop, counts, fit, p.overlap, p.toplist_size)
    prev, prev_fit = pop, fit

    wsum = sum(p.op_weight)
    gens_run = 0
    stopped = False
    for g in range(1, generations + 1):
        # Step 2: elitism and penalties.
        penalty = [0] * n_cols
        n_e = min(len(top), (P * p.elite_num) // p.elite_den)
        new = [e.series for e in top[:n_e]]
        new_counts = [e.count for e in top[:n_e]]
        new_fit = [e.fitness for e in top[:n_e]]
        for s in new:
            for c in s:
                penalty[c] += 1

        def select() -> int:
            return tournament(rng, prev, prev_fit, penalty, p.tournament, p.penalty_base)

        # Step 3: fill the population with novel children.
        hits = 0
        while len(new) < P:
            ia = select()
            u = rng.uint(wsum)
            op, acc = 0, 0
            for op in range(5):
                acc += p.op_weight[op]
                if u < acc:
                    break
            if op == OP_CROSSOVER:
                ib = select()
                child = crossover(rng, prev[ia], prev[ib], p)
            else:
                child = tuple(mutate(rng, list(prev[ia]), op, p, n_cols))
            if child in tabu:
                hits += 1
                if hits > tabu_limit:
                    stopped = True
                    break
                continue
            new.append(child)
            tabu.add(child)
            for c in child:
                penalty[c] += 1
        if stopped:
            break

        # Step 4: evaluate the new members.
        cnt, fit = ev(new[n_e:], p.eval)
        new_counts += cnt
        new_fit += fit
        emit(g, new, new_counts, new_fit)
        gens_run = g

        # Step 5: top-rank list.
        top = update_top(top, new, new_counts, new_fit, p.overlap, p.toplist_size)
        prev, prev_fit = new, new_fit

    # Steps 6-7: matching rows of the listed series, with expansion params.
    bic = []
    if top:
        series = [e.series for e in top]
        offsets = np.zeros(len(series) + 1, dtype=np.int32)
        offsets[1:] = np.cumsum([len(s) for s in series])
        cols = np.array([c for s in series for c in s], dtype=np.int32)
        res = _oracle_evaluate(a, offsets, cols, sigma=p.expand.sigma,
                               max_violations=p.expand.max_violations,
                               negative_trends=p.expand.negative_trends, want_masks=True)
        for i, s in enumerate(series):
            words = res["masks"][i, 0] | res["masks"][i, 1]
            bic.append({"cols": s, "count": int(res["counts"][i]),
                        "fitness": float(res["fitness"][i]), "mask_words": words})
    return Result(biclusters=bic, generations_run=gens_run, stopped_by_tabu=stopped,
                  history=history, top=top)
