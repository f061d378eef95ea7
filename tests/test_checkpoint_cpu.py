"""Stateful runs and checkpoints on the CPU (oracle as evaluator): a run
advanced in pieces equals ebic_evolve_with, a run saved and resumed equals
the uninterrupted run generation by generation, and bad checkpoints are
refused."""
import numpy as np
import pytest

import oracle
import synth

import paper_1801_03039_amd as E


def _setup(name="tiny", **kw):
    w = synth.WORKLOADS[name]
    a, _ = synth.make_matrix(w)
    cfg = E.EvolveConfig(population=w.population, len_min=w.len_min, len_max=w.len_max,
                         eval=E.Trend(w.sigma, 0, False), expand=E.Trend(w.sigma, 0, True), **kw)

    def ev(o, c, sigma, k, neg, want_masks):
        r = oracle.evaluate(a, o, c, sigma=sigma, max_violations=k, negative_trends=neg,
                            want_masks=want_masks)
        return r["counts"], r["fitness"], r.get("masks")
    return w, a, cfg, ev


def _same_result(x, y):
    assert len(x.biclusters) == len(y.biclusters)
    for b, c in zip(x.biclusters, y.biclusters):
        assert b["cols"] == c["cols"] and b["count"] == c["count"]
        assert b["fitness"] == c["fitness"]
        assert np.array_equal(b["mask_words"], c["mask_words"])
    assert x.stats["generations_run"] == y.stats["generations_run"]
    assert x.stats["stopped_by_tabu"] == y.stats["stopped_by_tabu"]


def test_run_in_pieces_equals_evolve():
    w, a, cfg, ev = _setup()
    ref_gens = []
    ref = E.evolve_with(ev, a.shape[0], a.shape[1], 3, 12, cfg, on_generation=ref_gens.append)
    gens = []
    with E.Run(cfg, 3, 12, evaluate=ev, n_rows=a.shape[0], n_cols=a.shape[1],
               on_generation=gens.append) as run:
        done, steps = False, 0
        while not done:
            done = run.advance(5)
            steps += 1
        res = run.result()
        prog = run.progress()
    assert steps == 3 and prog["generations_run"] == 12 and prog["next_generation"] == 13
    assert [g.population for g in gens] == [g.population for g in ref_gens]
    _same_result(res, ref)


@pytest.mark.parametrize("cut", [0, 1, 4, 9])
def test_resume_equals_uninterrupted(cut):
    w, a, cfg, ev = _setup()
    kw = dict(evaluate=ev, n_rows=a.shape[0], n_cols=a.shape[1])
    full = []
    with E.Run(cfg, 8, 12, on_generation=full.append, **kw) as run:
        run.advance(100)
        ref = run.result()
    part = []
    with E.Run(cfg, 8, 12, on_generation=part.append, **kw) as run:
        run.advance(cut)
        data = run.save()
    with E.Run.load(cfg, data, on_generation=part.append, **kw) as run:
        assert run.progress()["next_generation"] == cut
        run.advance(100)
        res = run.result()
        # the state saved twice in a row is byte-identical
        assert run.save() == E.Run.load(cfg, run.save(), **kw).save()
    assert [g.population for g in part] == [g.population for g in full]
    for g, h in zip(part, full):
        assert np.array_equal(g.fitness.view(np.int64), h.fitness.view(np.int64))
    _same_result(res, ref)


def test_resume_after_tabu_stop():
    # a tiny column count exhausts the search space: the tabu rule stops the
    # run, and a checkpoint taken after the stop resumes as stopped
    w = synth.WORKLOADS["tiny"]
    rng = np.random.default_rng(2)
    a = rng.standard_normal((64, 4)).astype(np.float32)
    cfg = E.EvolveConfig(population=6, len_min=3, len_max=4, eval=E.Trend(2), expand=E.Trend(2))

    def ev(o, c, sigma, k, neg, want_masks):
        r = oracle.evaluate(a, o, c, sigma=sigma, max_violations=k, negative_trends=neg,
                            want_masks=want_masks)
        return r["counts"], r["fitness"], r.get("masks")
    kw = dict(evaluate=ev, n_rows=64, n_cols=4)
    with E.Run(cfg, 1, 500, **kw) as run:
        assert run.advance(500)
        p = run.progress()
        assert p["stopped_by_tabu"] == 1
        data = run.save()
        ref = run.result()
    with E.Run.load(cfg, data, **kw) as run:
        assert run.advance(10)
        _same_result(run.result(), ref)


def test_bad_checkpoints_are_refused():
    w, a, cfg, ev = _setup()
    kw = dict(evaluate=ev, n_rows=a.shape[0], n_cols=a.shape[1])
    with E.Run(cfg, 4, 6, **kw) as run:
        run.advance(3)
        data = run.save()
    with pytest.raises(E.EbicError):
        E.Run.load(cfg, data[:-5], **kw)                      # truncated
    with pytest.raises(E.EbicError):
        E.Run.load(cfg, b"XXXX" + data[4:], **kw)            # not a checkpoint
    other = E.EvolveConfig(population=cfg.population, len_min=cfg.len_min, len_max=cfg.len_max,
                           eval=cfg.eval, expand=cfg.expand, tournament=4)
    with pytest.raises(E.EbicError):
        E.Run.load(other, data, **kw)                          # other parameters
    with pytest.raises(E.EbicError):
        E.Run.load(cfg, data, evaluate=ev, n_rows=a.shape[0] + 1, n_cols=a.shape[1])
    bad = bytearray(data)
    bad[-20] ^= 0xFF                                           # corrupt the tail
    try:
        with E.Run.load(cfg, bytes(bad), **kw) as r:
            r.advance(10)                                      # parses, but must still run
    except E.EbicError:
        pass
