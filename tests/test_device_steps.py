"""GPU: batched runs with Steps 1-3 and 5 on the device
(ebic_batch_evolve_device) equal the oracle's runs generation by generation
-- populations, counts, fitness bits -- and in their Steps 6-7 output, and
equal the host-stepped batched runs on the batched workload's shapes."""
import sys

import numpy as np
import pytest

import synth
from oracle import evolve as oev

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[device-steps] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_03039_amd as e
    return e


def _configs(E, **kw):
    ev = kw.pop("eval", (8, 0, False))
    ex = kw.pop("expand", (8, 1, True))
    cfg = E.EvolveConfig(eval=E.Trend(*ev), expand=E.Trend(*ex), **kw)
    op = oev.EvolveParams(eval=oev.TrendParams(*ev), expand=oev.TrendParams(*ex), **kw)
    return cfg, op


def _compare_with_oracle(E, mats, seeds, G, cfg, op):
    gens = {r: [] for r in range(len(mats))}
    with E.Batch(mats) as b:
        res = b.evolve(seeds, G, cfg, on_generation=lambda r, g: gens[r].append(g),
                       device_steps=True)
    for r, (a, s) in enumerate(zip(mats, seeds)):
        ref = oev.evolve(a, s, G, op)
        assert len(gens[r]) == len(ref.history), f"run {r}"
        for g, h in zip(gens[r], ref.history):
            assert g.population == h.population, f"run {r} generation {h.gen}"
            assert np.array_equal(g.counts, h.counts), f"run {r} generation {h.gen}"
            assert np.array_equal(g.fitness.view(np.int64), h.fitness.view(np.int64))
        assert res[r].stats["generations_run"] == ref.generations_run
        assert res[r].stats["stopped_by_tabu"] == int(ref.stopped_by_tabu)
        assert [x["cols"] for x in res[r].biclusters] == [x["cols"] for x in ref.biclusters]
        for x, y in zip(res[r].biclusters, ref.biclusters):
            assert x["count"] == y["count"] and x["fitness"] == y["fitness"]
            assert np.array_equal(x["mask_words"], y["mask_words"])
    return res


@pytest.mark.parametrize("weights,K,theta", [
    ((1, 1, 1, 1, 1), 100, 0.5),
    ((0, 0, 0, 0, 1), 5, 0.5),      # crossover only; a short top list (evictions, early stop)
    ((3, 1, 2, 2, 0), 8, 0.25),     # mutations only
    ((1, 2, 0, 0, 3), 12, 1.0),
])
def test_device_steps_match_oracle(E, weights, K, theta):
    rng = np.random.default_rng(40 + K)
    shapes = [(150, 20), (300, 12), (90, 30), (500, 8), (64, 40)]
    mats = [rng.standard_normal(s).astype(np.float32) for s in shapes]
    mats[3] = synth.adversarial_matrix(rng, 500, 8)          # ties, NaN, infinities
    seeds = [11, 12, 13, 14, 15]
    cfg, op = _configs(E, population=60, len_min=2, len_max=7, op_weight=weights,
                       toplist_size=K, overlap=theta, eval=(6, 1, True))
    _note(f"oracle parity weights={weights} K={K} theta={theta}")
    _compare_with_oracle(E, mats, seeds, 8, cfg, op)


def test_device_steps_tabu_stop(E):
    # 5 columns, series of 2-3: 80 distinct series; a population of 24
    # exhausts them within a few generations and the tabu rule ends the run
    rng = np.random.default_rng(3)
    mats = [rng.standard_normal((100, 5)).astype(np.float32) for _ in range(3)]
    cfg, op = _configs(E, population=24, len_min=2, len_max=3, tabu_limit=-1)
    _note("tabu stop")
    res = _compare_with_oracle(E, mats, [1, 2, 3], 30, cfg, op)
    assert any(r.stats["stopped_by_tabu"] for r in res)


def test_device_steps_long_run(E):
    # 200 generations of the 200 x 50 planted matrix with three 30 x 8
    # rising biclusters, one run per seed
    w = synth.WORKLOADS["tiny"]
    a, _ = synth.make_matrix(w)
    cfg, op = _configs(E, population=w.population, len_min=w.len_min, len_max=w.len_max,
                       eval=(w.sigma, w.max_violations, w.negative_trends),
                       expand=(w.sigma, w.max_violations, True), toplist_size=w.toplist)
    _note("tiny workload, 200 generations, 2 seeds")
    _compare_with_oracle(E, [a, a], [0, 1], 200, cfg, op)


def test_device_steps_equal_host_steps_on_batched_shapes(E):
    # eight runs of the batched setting (up to 50000 rows, 20-1000 columns),
    # population 1024, 12 generations: every generation of every run equals
    # the host-stepped batched run
    R, G = 8, 12
    ws = [synth.batched_workload(r) for r in range(R)]
    mats = [synth.make_matrix(w)[0] for w in ws]
    cfg = E.EvolveConfig(population=1024, len_min=3, len_max=20, eval=E.Trend(25),
                         expand=E.Trend(25, 0, True))
    runs = {}
    for dev in (False, True):
        gens = {r: [] for r in range(R)}
        with E.Batch(mats) as b:
            _note(f"batched shapes device_steps={dev}")
            res = b.evolve(list(range(R)), G, cfg, on_generation=lambda r, g: gens[r].append(g),
                           device_steps=dev)
        runs[dev] = (gens, res)
    (gh, rh), (gd, rd) = runs[False], runs[True]
    for r in range(R):
        assert len(gd[r]) == len(gh[r]) == G + 1
        for x, y in zip(gd[r], gh[r]):
            assert x.population == y.population, f"run {r} generation {y.gen}"
            assert np.array_equal(x.counts, y.counts)
            assert np.array_equal(x.fitness.view(np.int64), y.fitness.view(np.int64))
        assert [x["cols"] for x in rd[r].biclusters] == [x["cols"] for x in rh[r].biclusters]
        for x, y in zip(rd[r].biclusters, rh[r].biclusters):
            assert x["count"] == y["count"] and x["fitness"] == y["fitness"]
            assert np.array_equal(x["mask_words"], y["mask_words"])


def test_device_steps_limits(E):
    rng = np.random.default_rng(9)
    mats = [rng.standard_normal((100, 70)).astype(np.float32)]
    cfg = E.EvolveConfig(population=20, len_min=3, len_max=59, eval=E.Trend(5),
                         expand=E.Trend(5))
    with E.Batch(mats) as b:
        with pytest.raises(E.EbicError, match="E_ARG"):
            b.evolve([1], 2, cfg, device_steps=True)
