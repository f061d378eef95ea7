"""The library's host steps of the evolutionary run (Steps 1-3, 5-7) against
the oracle's independent implementation, generation by generation, with the
oracle's CPU evaluation plugged in as the evaluator (ebic_evolve_with).  No
GPU: this isolates the host logic; tests/test_evolve_parity.py runs the whole
product path on the GPU."""
import numpy as np
import pytest

import oracle
import synth
from oracle import evolve as oev

import paper_1801_03039_amd as E


def _oracle_eval(a):
    def ev(o, c, sigma, k, neg, want_masks):
        r = oracle.evaluate(a, o, c, sigma=sigma, max_violations=k, negative_trends=neg,
                            want_masks=want_masks)
        return r["counts"], r["fitness"], r.get("masks")
    return ev


def _configs(pop, lmin, lmax, ev, ex, **kw):
    cfg = E.EvolveConfig(population=pop, len_min=lmin, len_max=lmax,
                         eval=E.Trend(*ev), expand=E.Trend(*ex), **kw)
    okw = dict(kw)
    op = oev.EvolveParams(population=pop, len_min=lmin, len_max=lmax,
                          eval=oev.TrendParams(*ev), expand=oev.TrendParams(*ex), **okw)
    return cfg, op


def _compare(a, seed, gens, cfg, op):
    got = []
    res = E.evolve_with(_oracle_eval(a), a.shape[0], a.shape[1], seed, gens, cfg,
                        on_generation=got.append)
    ref = oev.evolve(a, seed, gens, op)
    assert len(got) == len(ref.history)
    for g, r in zip(got, ref.history):
        assert g.gen == r.gen
        assert g.population == r.population, f"generation {g.gen}"
        assert np.array_equal(g.counts, r.counts)
        assert np.array_equal(g.fitness.view(np.int64), r.fitness.view(np.int64))
    assert res.stats["generations_run"] == ref.generations_run
    assert bool(res.stats["stopped_by_tabu"]) == ref.stopped_by_tabu
    assert len(res.biclusters) == len(ref.biclusters)
    for b, r in zip(res.biclusters, ref.biclusters):
        assert b["cols"] == r["cols"]
        assert b["count"] == r["count"]
        assert b["fitness"] == r["fitness"]
        assert np.array_equal(b["mask_words"], r["mask_words"])
    return res, ref


def test_tiny_workload_full_run():
    w = synth.WORKLOADS["tiny"]
    a, _ = synth.make_matrix(w)
    cfg, op = _configs(w.population, w.len_min, w.len_max, (w.sigma, 0, False), (w.sigma, 0, True))
    res, ref = _compare(a, 0, w.generations, cfg, op)
    assert res.stats["candidates_evaluated"] > 0


@pytest.mark.parametrize("seed", [1, 2])
def test_other_parameters(seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((300, 30)).astype(np.float32)
    cfg, op = _configs(80, 2, 9, (10, 1, True), (10, 2, True), tournament=5,
                       op_weight=(3, 1, 2, 0, 4), elite_num=1, elite_den=3, overlap=0.75,
                       toplist_size=20, penalty_base=1.5)
    _compare(a, seed, 15, cfg, op)


def test_tabu_stop_matches():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((100, 5)).astype(np.float32)
    cfg, op = _configs(10, 2, 2, (3, 0, False), (3, 0, True))
    res, ref = _compare(a, 5, 60, cfg, op)
    assert ref.stopped_by_tabu and res.stats["stopped_by_tabu"]


def test_tabu_limit_zero_and_length_bounds_equal_m():
    # L = M: substitution is never applicable (every column already used).
    rng = np.random.default_rng(4)
    a = rng.standard_normal((120, 6)).astype(np.float32)
    cfg, op = _configs(30, 4, 6, (3, 0, False), (3, 0, True), tabu_limit=0)
    _compare(a, 9, 10, cfg, op)


def test_expression_shaped_first_generations():
    w = synth.WORKLOADS["expression"]
    a, _ = synth.make_matrix(w)
    a = a[:2000]                           # rows cut for CPU time
    cfg, op = _configs(256, w.len_min, w.len_max, (w.sigma, 1, True), (w.sigma, 1, True))
    _compare(a, 1, 3, cfg, op)


def test_argument_errors():
    a = np.zeros((10, 4), dtype=np.float32)
    ev = _oracle_eval(a)
    bad = [
        dict(population=0, len_min=1, len_max=2),
        dict(population=5, len_min=3, len_max=2),
        dict(population=5, len_min=1, len_max=5),          # len_max > n_cols
        dict(population=5, len_min=1, len_max=2, tournament=0),
        dict(population=5, len_min=1, len_max=2, op_weight=(0, 0, 0, 0, 0)),
        dict(population=5, len_min=1, len_max=2, elite_num=3, elite_den=2),
        dict(population=5, len_min=1, len_max=2, toplist_size=0),
        dict(population=5, len_min=1, len_max=2, overlap=1.5),
        dict(population=17, len_min=2, len_max=2),          # 4*3 = 12 distinct series
    ]
    for kw in bad:
        cfg = E.EvolveConfig(eval=E.Trend(1), expand=E.Trend(1), **kw)
        with pytest.raises(E.EbicError) as ex:
            E.evolve_with(ev, 10, 4, 0, 1, cfg)
        assert ex.value.status == 1, kw
    cfg = E.EvolveConfig(population=5, len_min=1, len_max=2, eval=E.Trend(-1), expand=E.Trend(1))
    with pytest.raises(E.EbicError) as ex:
        E.evolve_with(ev, 10, 4, 0, 1, cfg)
    assert ex.value.status == 2


@pytest.mark.parametrize("theta,K", [(0.0, 5), (0.3, 3), (0.5, 1), (1.0, 4)])
def test_top_rank_ties_and_small_lists(theta, K):
    # Tie-heavy integer data: many members share counts and fitness, so the
    # stable tie rules and the list cut are exercised every generation.
    rng = np.random.default_rng(int(theta * 10) + K)
    a = rng.integers(0, 3, size=(150, 12)).astype(np.float32)
    cfg, op = _configs(60, 2, 5, (4, 0, True), (4, 1, True), overlap=theta, toplist_size=K)
    _compare(a, 3, 12, cfg, op)
