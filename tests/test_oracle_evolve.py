"""Pins for the oracle's evolutionary run (no GPU).

The paper fixes the structure of the run (Steps 1-7) but prints no worked
example, so draw-for-draw behaviour is unpinned by the paper.  These tests
pin what the paper and the written readings do fix: the published SplitMix64
outputs, the properties of each genetic operation (Fig. 1), the tabu rule
and its stop criterion (Step 3), elitism (Step 2), and the top-rank list
invariants (Step 5).
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import evolve as ev


def test_splitmix64_published_outputs(golden_dir):
    with open(os.path.join(golden_dir, "splitmix64.json")) as f:
        g = json.load(f)
    for st in g["streams"]:
        r = ev.SplitMix64(st["seed"])
        if "outputs_hex" in st:
            want = [int(x, 16) for x in st["outputs_hex"]]
        else:
            want = [int(x) for x in st["outputs_dec"]]
        assert [r.next() for _ in want] == want


def _params(**kw):
    base = dict(population=60, len_min=3, len_max=7,
                eval=ev.TrendParams(sigma=10), expand=ev.TrendParams(sigma=10, negative_trends=True))
    base.update(kw)
    return ev.EvolveParams(**base)


@pytest.fixture(scope="module")
def tiny_run():
    w = synth.WORKLOADS["tiny"]
    a, planted = synth.make_matrix(w)
    p = _params(population=w.population, len_min=w.len_min, len_max=w.len_max,
                eval=ev.TrendParams(sigma=w.sigma),
                expand=ev.TrendParams(sigma=w.sigma, max_violations=0, negative_trends=True))
    return a, p, ev.evolve(a, 0, 12, p)


def test_run_is_deterministic(tiny_run):
    a, p, res = tiny_run
    again = ev.evolve(a, 0, 12, p)
    assert len(again.history) == len(res.history)
    for g1, g2 in zip(res.history, again.history):
        assert g1.population == g2.population
        assert np.array_equal(g1.fitness, g2.fitness)
    other = ev.evolve(a, 1, 2, p)
    assert other.history[0].population != res.history[0].population


def test_generation_invariants(tiny_run):
    a, p, res = tiny_run
    seen = set()
    top_prev = None
    for g in res.history:
        assert len(g.population) == p.population
        assert len(set(g.population)) == p.population
        for s in g.population:
            assert p.len_min <= len(s) <= p.len_max
            assert len(set(s)) == len(s)
            assert all(0 <= c < a.shape[1] for c in s)
        # Scores are the oracle's evaluation of each member (elites keep
        # their stored scores, which are the same values).
        off, cols = synth.pack_cbf([list(s) for s in g.population])
        chk = oracle.evaluate(a, off, cols, sigma=p.eval.sigma)
        assert np.array_equal(chk["counts"], g.counts)
        assert np.array_equal(chk["fitness"], g.fitness)
        # Tabu: apart from the elites carried over, no series is seen twice.
        n_e = 0 if g.gen == 0 else min(len(top_prev), p.population // 4)
        if g.gen > 0:
            assert g.population[:n_e] == [e.series for e in top_prev[:n_e]]
        for s in g.population[n_e:]:
            assert s not in seen
            seen.add(s)
        top_prev = ev.update_top(top_prev or [], g.population, g.counts, g.fitness,
                                 p.overlap, p.toplist_size)


def test_top_list_invariants(tiny_run):
    a, p, res = tiny_run
    top = res.top
    assert 0 < len(top) <= p.toplist_size
    fits = [e.fitness for e in top]
    assert fits == sorted(fits, reverse=True)
    assert all(f > 0 for f in fits)
    for i in range(len(top)):
        for j in range(i + 1, len(top)):
            x, e = top[i].series, top[j].series
            assert x != e
            assert len(set(x) & set(e)) / min(len(x), len(e)) <= p.overlap
    # Step 6/7 output: one bicluster per listed series, rows from both
    # directions with the expansion parameters.
    assert [b["cols"] for b in res.biclusters] == [e.series for e in top]
    off, cols = synth.pack_cbf([list(e.series) for e in top])
    chk = oracle.evaluate(a, off, cols, sigma=p.expand.sigma, negative_trends=True, want_masks=True)
    for i, b in enumerate(res.biclusters):
        assert b["count"] == chk["counts"][i]
        assert np.array_equal(b["mask_words"], chk["masks"][i, 0] | chk["masks"][i, 1])


def test_top_update_rules():
    # Hand-built cases of Step 5: admission, rejection by a fitter
    # overlapping entry, eviction of weaker overlapping entries, truncation.
    top = [ev.TopEntry((0, 1, 2, 3), 10, 5.0), ev.TopEntry((10, 11, 12), 9, 4.0)]
    pop = [(0, 1, 2, 9), (10, 11, 20, 21), (30, 31, 32), (40, 41), (0, 1, 2, 3)]
    fit = [4.5, 6.0, 1.0, 0.0, 7.0]
    cnt = [8, 12, 4, 3, 10]
    out = ev.update_top(top, pop, cnt, fit, 0.5, 3)
    # (10,11,20,21) overlaps (10,11,12) by 2/3 > 0.5 and is fitter: evicts it.
    # (0,1,2,3) is already listed: skipped.  (0,1,2,9) overlaps (0,1,2,3) by
    # 3/4 and is weaker: rejected.  (30,31,32) is new: admitted.  (40,41) has
    # zero fitness: skipped.
    assert [e.series for e in out] == [(10, 11, 20, 21), (0, 1, 2, 3), (30, 31, 32)]
    out2 = ev.update_top(top, pop, cnt, fit, 0.5, 2)
    assert [e.series for e in out2] == [(10, 11, 20, 21), (0, 1, 2, 3)]
    # Equal fitness and overlap: the incumbent wins.
    out3 = ev.update_top([ev.TopEntry((1, 2), 5, 3.0)], [(2, 1)], [5], [3.0], 0.5, 5)
    assert [e.series for e in out3] == [(1, 2)]


def test_mutation_properties():
    rng = ev.SplitMix64(7)
    p = _params(len_min=2, len_max=6)
    m = 12
    for _ in range(500):
        L = 2 + rng.uint(5)
        s = []
        while len(s) < L:
            c = rng.uint(m)
            if c not in s:
                s.append(c)
        for op in range(4):
            before = list(s)
            after = ev.mutate(rng, list(s), op, p, m)
            assert len(set(after)) == len(after)
            if op == ev.OP_INSERT:
                if L < p.len_max:
                    assert len(after) == L + 1
                    rest = [c for c in after if c in before]
                    assert rest == before
                else:
                    assert after == before
            elif op == ev.OP_DELETE:
                if L > p.len_min:
                    assert len(after) == L - 1
                    assert all(c in before for c in after)
                    assert [c for c in before if c in after] == after
                else:
                    assert after == before
            elif op == ev.OP_SWAP:
                assert sorted(after) == sorted(before)
                diff = [i for i in range(L) if after[i] != before[i]]
                assert len(diff) == 2
            else:
                assert len(after) == L
                diff = [i for i in range(L) if after[i] != before[i]]
                assert len(diff) == 1 and after[diff[0]] not in before


def test_crossover_properties():
    rng = ev.SplitMix64(11)
    p = _params(len_min=3, len_max=6)
    for _ in range(500):
        a = tuple(int(x) for x in np.random.default_rng(rng.next() % 1000).permutation(15)[:3 + rng.uint(4)])
        b = tuple(int(x) for x in np.random.default_rng(rng.next() % 1000).permutation(15)[:3 + rng.uint(4)])
        child = ev.crossover(rng, a, b, p)
        assert len(set(child)) == len(child)
        assert p.len_min <= len(child) <= p.len_max
        if child != a:
            # a prefix of a, then columns of b in b's order
            i = 0
            while i < len(child) and i < len(a) and child[i] == a[i]:
                i += 1
            tail = child[i:]
            assert all(c in b for c in tail)
            pos = [b.index(c) for c in tail]
            assert pos == sorted(pos)


def test_tabu_stop_on_exhausted_search_space():
    # 4 columns, series of length 2: only 12 distinct series exist, so the
    # tabu list fills and the run must stop on the hit counter (Step 3).
    rng = np.random.default_rng(3)
    a = rng.standard_normal((100, 4)).astype(np.float32)
    p = _params(population=6, len_min=2, len_max=2)
    res = ev.evolve(a, 5, 50, p)
    assert res.stopped_by_tabu
    assert res.generations_run < 50
    all_series = [s for g in res.history for s in g.population]
    assert len(set(all_series)) <= 12


def test_population_larger_than_search_space_is_rejected():
    a = np.zeros((10, 3), dtype=np.float32)
    with pytest.raises(ValueError):
        ev.evolve(a, 0, 1, _params(population=7, len_min=2, len_max=2))


class _Draws:
    """A stand-in for the random stream that returns scripted uint draws."""

    def __init__(self, draws):
        self.draws = list(draws)

    def uint(self, n):
        x = self.draws.pop(0)
        assert 0 <= x < n
        return x


# Hand-worked tournaments (Step 3 selection; the crowding penalty of
# Section 2.1: quality divided by base^theta, theta the mean penalty of the
# series' columns).  Base 2 keeps every quality exact:
#   member  series          fitness  penalties        theta  quality
#   0       (0, 1)          8        1, 1             1      8 / 2  = 4
#   1       (2, 3)          5        0, 0             0      5 / 1  = 5
#   2       (4, 5)          12       2, 2             2      12 / 4 = 3
#   3       (6, 7)          10       1, 1             1      10 / 2 = 5   (ties member 1)
#   4       (8, 9, 10, 11)  20       1, 1, 1, 1       1      20 / 2 = 10  (theta = 4 / 4)
_PREV = [(0, 1), (2, 3), (4, 5), (6, 7), (8, 9, 10, 11)]
_FIT = [8.0, 5.0, 12.0, 10.0, 20.0]
_PEN = [1, 1, 0, 0, 2, 2, 1, 1, 1, 1, 1, 1]


@pytest.mark.parametrize("draws,winner", [
    ([0, 1, 2], 1),    # 4, 5, 3: the penalty decides (raw fitness would pick 2;
                       # multiplying by 2^theta would pick 2 with 48)
    ([2, 0, 2], 0),    # 3, 4, 3: the largest quality, not the smallest (3)
    ([1, 3, 0], 1),    # 5, 5, 4: equal qualities, the first draw wins
    ([3, 1, 0], 3),    # 5, 5, 4: ... whichever is drawn first
    ([4, 1, 2], 4),    # 10, 5, 3: theta is the mean penalty (a sum of 4 would give 1.25)
    ([2, 2, 2], 2),    # repeated draws of one member
])
def test_tournament_hand_worked(draws, winner):
    rng = _Draws(draws)
    assert ev.tournament(rng, _PREV, _FIT, _PEN, 3, 2.0) == winner
    assert rng.draws == []                    # exactly `size` draws


def test_tournament_with_the_paper_base():
    # base 1.2: member 0 has fitness 12 and theta 1 -> 12 / 1.2 = 10 (to
    # within one rounding); member 1 has fitness 10.5 and theta 0 -> 10.5.
    prev, fit, pen = [(0, 1), (2, 3)], [12.0, 10.5], [1, 1, 0, 0]
    assert ev.tournament(_Draws([0, 1]), prev, fit, pen, 2, 1.2) == 1
    assert ev.tournament(_Draws([1, 0]), prev, fit, pen, 2, 1.2) == 1
    # with fitness 10.6 for member 0 (10.6 / 1.2 = 8.83) member 1 still wins,
    # with 12.7 (10.58) member 0 does
    assert ev.tournament(_Draws([0, 1]), prev, [10.6, 10.5], pen, 2, 1.2) == 1
    assert ev.tournament(_Draws([1, 0]), prev, [12.7, 10.5], pen, 2, 1.2) == 0
    # a single draw always wins, whatever its quality
    assert ev.tournament(_Draws([0]), prev, [0.0, 10.5], pen, 1, 1.2) == 0


def _recovery_top(res, planted, n_rows, k):
    from oracle import scores as osc
    found = []
    for b in res.biclusters[:k]:
        rows = osc.mask_rows(np.asarray(b["mask_words"], dtype=np.uint64)[None, :], n_rows)[0]
        found.append((rows, list(b["cols"])))
    expected = [(p.rows, list(p.cols)) for p in planted]
    _, rec, rel = osc.match_scores(found, expected)
    return rec, rel


@pytest.mark.parametrize("seed", [0, 1])
def test_search_recovers_planted_biclusters(seed):
    # Behavioural pin of the whole run (Section 3, synthetic data: the
    # trend-preserving patterns are recovered): on the 200x50 matrix with
    # three planted 30x8 rising biclusters, 1000 generations find them; the
    # best three biclusters of the top-rank list score recovery and relevance
    # (Eqs. 2-3) of at least 0.85 against the planted truth.  A tournament
    # that picks the weakest draw, or a penalty that rewards crowding, leaves
    # both far lower (the configured 50 generations reach 0.15-0.37).
    w = synth.WORKLOADS["tiny"]
    a, planted = synth.make_matrix(w)
    p = _params(population=w.population, len_min=w.len_min, len_max=w.len_max,
                eval=ev.TrendParams(sigma=w.sigma), expand=ev.TrendParams(sigma=w.sigma))
    res = ev.evolve(a, seed, 1000, p, keep_history=False)
    assert res.generations_run == 1000 and not res.stopped_by_tabu
    rec, rel = _recovery_top(res, planted, w.n_rows, len(planted))
    assert rec >= 0.85 and rel >= 0.85, (rec, rel)
