"""GPU: the whole product path of the evolutionary run (host steps in the
library, Step 4/6 evaluations on the GPU) reproduces the oracle's run
generation by generation: identical populations, counts and bit-identical
fitness, then identical Step 6/7 output."""
import sys

import numpy as np
import pytest

import synth
from oracle import evolve as oev

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[evolve] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_03039_amd as e
    return e


def _run_both(E, a, w, seed, gens, path, pop=None):
    P = pop or w.population
    ev = (w.sigma, w.max_violations, w.negative_trends)
    ex = (w.sigma, w.max_violations, True)
    cfg = E.EvolveConfig(population=P, len_min=w.len_min, len_max=w.len_max,
                         eval=E.Trend(*ev), expand=E.Trend(*ex), overlap=w.overlap,
                         toplist_size=w.toplist, tournament=w.tournament)
    op = oev.EvolveParams(population=P, len_min=w.len_min, len_max=w.len_max,
                          eval=oev.TrendParams(*ev), expand=oev.TrendParams(*ex),
                          overlap=w.overlap, toplist_size=w.toplist, tournament=w.tournament)
    got = []
    with E.Context(a, path=path) as ctx:
        res = E.evolve(ctx, seed, gens, cfg, on_generation=got.append)
    ref = oev.evolve(a, seed, gens, op)
    assert len(got) == len(ref.history)
    for g, r in zip(got, ref.history):
        assert g.population == r.population, f"generation {g.gen}"
        assert np.array_equal(g.counts, r.counts), f"generation {g.gen}"
        assert np.array_equal(g.fitness.view(np.int64), r.fitness.view(np.int64))
    assert len(res.biclusters) == len(ref.biclusters)
    for b, r in zip(res.biclusters, ref.biclusters):
        assert b["cols"] == r["cols"] and b["count"] == r["count"]
        assert b["fitness"] == r["fitness"]
        assert np.array_equal(b["mask_words"], r["mask_words"])
    return res


@pytest.mark.parametrize("path", ["direct", "index"])
def test_tiny_full_run(E, path):
    w = synth.WORKLOADS["tiny"]
    a, _ = synth.make_matrix(w)
    _note(f"tiny full run path={path}")
    res = _run_both(E, a, w, w.seed, w.generations, path)
    assert res.stats["generations_run"] == w.generations


@pytest.mark.parametrize("seed,path", [(0, "index"), (1, "direct")])
def test_tiny_long_run_recovers_planted(E, seed, path):
    # 1000 generations on the 200x50 matrix with three planted 30x8 rising
    # biclusters: the GPU run equals the oracle's generation by generation,
    # and its best three biclusters recover the planted ones (Eqs. 2-3,
    # recovery and relevance >= 0.85; the oracle run reaches 0.908)
    from oracle import scores as osc
    w = synth.WORKLOADS["tiny"]
    a, planted = synth.make_matrix(w)
    _note(f"tiny 1000 generations seed={seed} path={path}")
    res = _run_both(E, a, w, seed, 1000, path)
    assert res.stats["generations_run"] == 1000
    found = [(osc.mask_rows(b["mask_words"][None, :], w.n_rows)[0], list(b["cols"]))
             for b in res.biclusters[:len(planted)]]
    _, rec, rel = osc.match_scores(found, [(p.rows, list(p.cols)) for p in planted])
    _note(f"recovery {rec:.4f} relevance {rel:.4f}")
    assert rec >= 0.85 and rel >= 0.85


@pytest.mark.parametrize("name,gens", [("expression", 50), ("wide", 2)])
def test_workload_first_generations(E, name, gens):
    w = synth.WORKLOADS[name]
    a, _ = synth.make_matrix(w)
    _note(f"{name} first {gens} generations")
    _run_both(E, a, w, w.seed, gens, "auto")


def test_checkpointed_gpu_run_equals_evolve(E):
    # a GPU run saved after a few generations and resumed on a fresh
    # context equals the uninterrupted ebic_evolve run
    w = synth.WORKLOADS["expression"]
    a, _ = synth.make_matrix(w)
    cfg = E.EvolveConfig(population=512, len_min=w.len_min, len_max=w.len_max,
                            eval=E.Trend(w.sigma, w.max_violations, w.negative_trends),
                            expand=E.Trend(w.sigma, w.max_violations, True))
    ref_gens, gens = [], []
    with E.Context(a) as ctx:
        _note("checkpoint: uninterrupted run")
        ref = E.evolve(ctx, 21, 10, cfg, on_generation=ref_gens.append)
        with E.Run(cfg, 21, 10, ctx=ctx, on_generation=gens.append) as run:
            run.advance(4)
            data = run.save()
    with E.Context(a) as ctx2:
        _note("checkpoint: resumed run")
        with E.Run.load(cfg, data, ctx=ctx2, on_generation=gens.append) as run:
            assert run.advance(100)
            res = run.result()
    assert [g.population for g in gens] == [g.population for g in ref_gens]
    for g, h in zip(gens, ref_gens):
        assert np.array_equal(g.fitness.view(np.int64), h.fitness.view(np.int64))
    assert [b["cols"] for b in res.biclusters] == [b["cols"] for b in ref.biclusters]
    for b, c in zip(res.biclusters, ref.biclusters):
        assert np.array_equal(b["mask_words"], c["mask_words"])


def test_reported_generations_subset(E):
    # on_generation restricted to some generations sees exactly those, equal
    # to the same generations of a fully reported run with the same seed
    w = synth.WORKLOADS["tiny"]
    a, _ = synth.make_matrix(w)
    cfg = E.EvolveConfig(population=w.population, len_min=w.len_min, len_max=w.len_max,
                         eval=E.Trend(w.sigma, w.max_violations, w.negative_trends),
                         expand=E.Trend(w.sigma, w.max_violations, True))
    full, part = [], []
    with E.Context(a) as ctx:
        _note("reported generations subset")
        r1 = E.evolve(ctx, 5, 12, cfg, on_generation=full.append)
        r2 = E.evolve(ctx, 5, 12, cfg, on_generation=part.append, report_generations={0, 4, 12})
    assert [g.gen for g in part] == [0, 4, 12]
    by_gen = {g.gen: g for g in full}
    for g in part:
        h = by_gen[g.gen]
        assert g.population == h.population
        assert np.array_equal(g.fitness.view(np.int64), h.fitness.view(np.int64))
    assert [b["cols"] for b in r1.biclusters] == [b["cols"] for b in r2.biclusters]


def test_best_fitness_callback(E):
    # on_best reports each generation's best fitness, as the full callback sees it
    w = synth.WORKLOADS["tiny"]
    a, _ = synth.make_matrix(w)
    cfg = E.EvolveConfig(population=w.population, len_min=w.len_min, len_max=w.len_max,
                         eval=E.Trend(w.sigma, w.max_violations, w.negative_trends),
                         expand=E.Trend(w.sigma, w.max_violations, True))
    full, best = [], []
    with E.Context(a) as ctx:
        _note("best-fitness callback")
        E.evolve(ctx, 9, 8, cfg, on_generation=full.append)
        E.evolve(ctx, 9, 8, cfg, on_best=lambda g, f: best.append((g, f)))
        with pytest.raises(ValueError):
            E.evolve(ctx, 9, 2, cfg, on_generation=full.append, on_best=print)
    assert [g for g, _ in best] == [g.gen for g in full]
    assert [f for _, f in best] == [float(g.fitness.max(initial=0.0)) for g in full]
