"""The screened host steps (offspring pool drawn by parallel breeders, kept
by a caller's ranking) on the CPU, with the oracle as evaluator: results do
not depend on the host thread count, every admitted child is scored by the
evaluator, the kept children are the pool's highest ranked, and the pool
rules hold (novel, distinct, elites first)."""
import numpy as np

import oracle
import synth

import paper_1801_03039_amd as E


def _setup():
    w = synth.WORKLOADS["tiny"]
    a, _ = synth.make_matrix(w)
    cfg = E.EvolveConfig(population=w.population, len_min=w.len_min, len_max=w.len_max,
                         eval=E.Trend(w.sigma, 0, False), expand=E.Trend(w.sigma, 0, True))

    def ev(o, c, sigma, k, neg, want_masks):
        r = oracle.evaluate(a, o, c, sigma=sigma, max_violations=k, negative_trends=neg,
                            want_masks=want_masks)
        return r["counts"], r["fitness"], r.get("masks")

    def exact_score(o, c):
        return oracle.evaluate(a, o, c, sigma=w.sigma)["fitness"]

    return w, a, cfg, ev, exact_score


def _run(threads, score, gens=8, seed=4, oversample=4, warmup=2, pools=None):
    w, a, cfg, ev, _ = _setup()
    got = []

    def sc(o, c):
        if pools is not None:
            pools.append((o, c))
        return score(o, c)
    res = E.evolve_screened_with(ev, sc, a.shape[0], a.shape[1], seed, gens, cfg,
                                 oversample=oversample, warmup_generations=warmup,
                                 host_threads=threads, on_generation=got.append)
    return res, got


def _hash_score(o, c):
    # a fixed pseudo-random ranking of series
    out = np.empty(len(o) - 1, dtype=np.float32)
    for i in range(len(o) - 1):
        out[i] = (hash(tuple(int(x) for x in c[o[i]:o[i + 1]])) % 100003) / 100003.0
    return out


def test_results_do_not_depend_on_thread_count():
    r1, g1 = _run(1, _hash_score)
    r4, g4 = _run(4, _hash_score)
    r0, g0 = _run(0, _hash_score)
    for a, b, c in zip(g1, g4, g0):
        assert a.population == b.population == c.population
        assert np.array_equal(a.fitness, b.fitness) and np.array_equal(a.fitness, c.fitness)
    assert [x["cols"] for x in r1.biclusters] == [x["cols"] for x in r4.biclusters]


def test_admitted_children_are_scored_exactly_and_novel():
    w, a, cfg, ev, exact = _setup()
    res, gens = _run(2, exact)
    seen = set()
    for g in gens:
        ref = oracle.evaluate(a, g.offsets, g.cols, sigma=w.sigma)
        assert np.array_equal(g.counts, ref["counts"])
        assert np.array_equal(g.fitness.view(np.int64), ref["fitness"].view(np.int64))
        pop = g.population
        assert len(set(pop)) == len(pop) == w.population
        # every child is new to the run; only the elites (<= P/4) were seen
        fresh = [s for s in pop if s not in seen]
        assert len(fresh) >= w.population - w.population // 4
        seen.update(pop)


def test_kept_children_are_the_pools_best():
    w, a, cfg, ev, exact = _setup()
    pools = []
    res, gens = _run(3, exact, pools=pools)
    screened = [g for g in gens if g.gen > 2]
    assert len(pools) == len(screened) > 0
    for (o, c), g in zip(pools, screened):
        pool = [tuple(int(x) for x in c[o[i]:o[i + 1]]) for i in range(len(o) - 1)]
        assert len(set(pool)) == len(pool)
        f = exact(o, c)
        kept = set(g.population)
        in_pool = [i for i, s in enumerate(pool) if s in kept]
        need = len(in_pool)
        assert need > 0
        # the kept children hold the `need` highest scores of the pool (ties
        # broken by pool order)
        order = sorted(range(len(pool)), key=lambda i: (-f[i], i))[:need]
        assert sorted(order) == in_pool
