"""GPU: batched evaluation and batched runs (many matrices, one launch per
generation) against the CPU oracle, run by run, bit for bit."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import evolve as oev

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[batch] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_03039_amd as e
    return e


SHAPES = [(1, 5), (65, 9), (200, 50), (1000, 30), (130, 3), (4096, 12)]


@pytest.fixture(scope="module")
def mats():
    rng = np.random.default_rng(21)
    out = []
    for i, (n, m) in enumerate(SHAPES):
        a = synth.adversarial_matrix(rng, n, m) if i % 2 else rng.standard_normal((n, m)).astype(np.float32)
        out.append(a)
    return out


def _pops(rng, mats, skip=()):
    pops = []
    for i, a in enumerate(mats):
        if i in skip:
            pops.append(None)
            continue
        m = a.shape[1]
        pop = synth.random_population(rng, m, int(rng.integers(1, 300)), 1, min(m, 12))
        pops.append(synth.pack_cbf(pop))
    return pops


def _check_runs(mats, pops, got, sigma, k, neg, masks=True):
    for a, pop, g in zip(mats, pops, got):
        if pop is None:
            assert g is None
            continue
        ref = oracle.evaluate(a, pop[0], pop[1], sigma=sigma, max_violations=k,
                              negative_trends=neg, want_masks=masks)
        assert np.array_equal(g["counts"], ref["counts"])
        assert np.array_equal(g["fitness"].view(np.int64), ref["fitness"].view(np.int64))
        if masks:
            assert np.array_equal(g["masks"], ref["masks"])


def test_batch_evaluate_matches_oracle(E, mats):
    rng = np.random.default_rng(1)
    with E.Batch(mats) as b:
        for k in (0, 1, 3):
            for neg in (False, True):
                pops = _pops(rng, mats, skip=(2,) if k == 1 else ())
                _note(f"evaluate k={k} neg={neg}")
                got = b.evaluate(pops, sigma=6, max_violations=k, negative_trends=neg,
                                 want_masks=True)
                _check_runs(mats, pops, got, 6, k, neg)


def test_full_batched_configuration(E):
    # The batched workload at full size: 64 runs on matrices of uneven shapes
    # (rows log-uniform 500-50000, columns 20-1000), a full mixed population
    # of 1024 per run, tuned launch shape; every run against the oracle.
    ws = [synth.batched_workload(r) for r in range(64)]
    data = [synth.make_matrix(w) for w in ws]
    rng = np.random.default_rng(1000)
    pops = [synth.pack_cbf(synth.mixed_population(rng, w, pl, w.population))
            for w, (a, pl) in zip(ws, data)]
    with E.Batch([a for a, _ in data]) as b:
        _note("full batched configuration, tuned")
        got = b.evaluate(pops, sigma=25, tune=True)
        _note(f"tuning {b.tuning()}")
        got2 = b.evaluate(pops, sigma=25)
    for w, (a, _), pop, g, g2 in zip(ws, data, pops, got, got2):
        ref = oracle.evaluate(a, pop[0], pop[1], sigma=25)
        assert np.array_equal(g["counts"], ref["counts"]), w.name
        assert np.array_equal(g["fitness"].view(np.int64), ref["fitness"].view(np.int64))
        assert np.array_equal(g2["counts"], ref["counts"])


@pytest.mark.parametrize("use_graph", [1, 0])
def test_graph_replays_interleaved_with_eager_work(E, mats, use_graph):
    # The captured graph (or the direct launch) is replayed with a new run
    # table each time, with eager single-context work and host
    # synchronisation in between; every replay must equal the oracle.
    import torch
    rng = np.random.default_rng(2)
    with E.Batch(mats) as b, E.Context(mats[3]) as ctx:
        b.set_tuning(0, 4, 1, 0, use_graph)
        assert b.tuning()["use_graph"] == use_graph
        for rep in range(5):
            pops = _pops(rng, mats)
            _note(f"replay {rep} use_graph={use_graph}")
            got = b.evaluate(pops, sigma=4, max_violations=1, negative_trends=True)
            _check_runs(mats, pops, got, 4, 1, True, masks=False)
            eager = ctx.evaluate(*pops[3], sigma=4, max_violations=1, negative_trends=True)
            assert np.array_equal(eager["counts"], got[3]["counts"])
            x = torch.arange(1000, device="cuda").sum()
            torch.cuda.synchronize()
            assert int(x) == 499500


def test_every_launch_shape_agrees(E, mats):
    rng = np.random.default_rng(3)
    pops = _pops(rng, mats)
    with E.Batch(mats) as b:
        ref = b.evaluate(pops, sigma=5, max_violations=2, negative_trends=True, want_masks=True,
                         tune=True)
        t = b.tuning()
        assert t["unroll"] in (1, 2, 4, 8) and (t["workgroups"] >= 1 or t["workgroups"] == -1)
        assert t["best_ms"] > 0
        assert t["words_per_lane"] in (1, 2, 4, 8) and t["whole_candidates"] in (0, 1)
        assert t["unroll"] * t["words_per_lane"] <= 16
        _check_runs(mats, pops, ref, 5, 2, True)
        for wg in (1, 0, 7, 5000, -1):
            for u in (1, 2, 4, 8):
                for v in (1, 2, 4, 8):
                    if u * v > 16:
                        with pytest.raises(E.EbicError):
                            b.set_tuning(wg, u, v, 0)
                        continue
                    for whole in (0, 1):
                        g = (u + v + whole) % 2
                        _note(f"shape wg={wg} unroll={u} words={v} whole={whole} graph={g}")
                        b.set_tuning(wg, u, v, whole, g)
                        got = b.evaluate(pops, sigma=5, max_violations=2, negative_trends=True,
                                         want_masks=True)
                        for g, r in zip(got, ref):
                            assert np.array_equal(g["counts"], r["counts"])
                            assert np.array_equal(g["fitness"].view(np.int64),
                                                  r["fitness"].view(np.int64))
                            assert np.array_equal(g["masks"], r["masks"])


def test_whole_candidate_tiles_on_tall_and_short_runs(E):
    # Runs on both sides of the whole-candidate limit (256 lanes: 16384 rows
    # at one word per lane, 32768 at two, 65536 at four) in one launch, tied
    # and untied matrices, against the oracle; each tiling mode in turn.
    rng = np.random.default_rng(6)
    shapes = [(16384, 9), (16385, 7), (32768, 6), (32769, 5), (65536, 4), (65537, 5),
              (70, 40), (1, 3)]
    mats_ = [synth.adversarial_matrix(rng, *s) if i % 2 else
             rng.standard_normal(s).astype(np.float32) for i, s in enumerate(shapes)]
    pops = []
    for a in mats_:
        m = a.shape[1]
        pop = synth.random_population(rng, m, int(rng.integers(20, 120)), 1, min(m, 8))
        off, cols = synth.pack_cbf(pop)
        pops.append((off, cols))
    with E.Batch(mats_) as b:
        for v in (1, 2, 4, 8):
            for whole in (0, 1):
                for wg in (0, -1):
                    _note(f"tall/short runs words={v} whole={whole} wg={wg}")
                    b.set_tuning(wg, min(4, 16 // v), v, whole)
                    got = b.evaluate(pops, sigma=4, max_violations=1, negative_trends=True,
                                     want_masks=True)
                    _check_runs(mats_, pops, got, 4, 1, True)


def test_batch_errors(E, mats):
    with E.Batch(mats[:2]) as b:
        with pytest.raises(E.EbicError):
            b.time_replays(3)          # nothing launched yet
        bad = [(np.array([0, 2]), np.array([0, 99])), None]
        with pytest.raises(E.EbicError):
            b.evaluate(bad, sigma=1)
        assert b.evaluate([None, None], sigma=1, max_violations=4) == [None, None]
        assert b.evaluate([None, None], sigma=1) == [None, None]
        with pytest.raises(E.EbicError):
            b.time_replays(3)          # the last request launched nothing


def test_parallel_packing_results_and_errors(E):
    # Enough columns for the host-array call to check and pack the runs on
    # several threads: results equal the oracle, and a malformed run is
    # reported by its index (the first one in run order).
    rng = np.random.default_rng(8)
    mats_ = [rng.standard_normal((int(rng.integers(60, 200)), 30)).astype(np.float32)
             for _ in range(16)]
    pops = [synth.pack_cbf(synth.random_population(rng, 30, 1024, 5, 12)) for _ in mats_]
    assert sum(int(o[-1]) for o, _ in pops) >= 1 << 17
    with E.Batch(mats_) as b:
        _note("parallel packing")
        got = b.evaluate(pops, sigma=3, max_violations=1, negative_trends=True)
        for i in (0, 7, 15):
            ref = oracle.evaluate(mats_[i], pops[i][0], pops[i][1], sigma=3, max_violations=1,
                                  negative_trends=True)
            assert np.array_equal(got[i]["counts"], ref["counts"])
            assert np.array_equal(got[i]["fitness"].view(np.int64), ref["fitness"].view(np.int64))
        bad = list(pops)
        o11, c11 = pops[11][0], pops[11][1].copy()
        c11[o11[500] + 1] = c11[o11[500]]                      # a repeated column in run 11
        o5, c5 = pops[5][0], pops[5][1].copy()
        c5[o5[3]] = 30                                        # a column out of range in run 5
        bad[11] = (o11, c11)
        with pytest.raises(E.EbicError, match="run 11"):
            b.evaluate(bad, sigma=3)
        bad[5] = (o5, c5)
        with pytest.raises(E.EbicError, match="run 5"):
            b.evaluate(bad, sigma=3)
        o2 = pops[2][0].copy()
        o2[10] = o2[9]                                        # an empty series in run 2
        bad[2] = (o2, pops[2][1])
        with pytest.raises(E.EbicError, match="run 2"):
            b.evaluate(bad, sigma=3)
        again = b.evaluate(pops, sigma=3, max_violations=1, negative_trends=True)
        for g, h in zip(got, again):
            assert np.array_equal(g["counts"], h["counts"])


def test_replays_keep_state(E, mats):
    # Back-to-back replays of a launch (queue and accumulators left as
    # found) do not disturb later launches, in every tiling mode.
    rng = np.random.default_rng(7)
    with E.Batch(mats) as b:
        for wg, u, v, whole in ((0, 4, 1, 0), (-1, 2, 2, 0), (-1, 1, 8, 1), (7, 2, 4, 1)):
            b.set_tuning(wg, u, v, whole)
            pops = _pops(rng, mats)
            b.evaluate(pops, sigma=3, max_violations=1, negative_trends=True)
            with pytest.raises(E.EbicError):
                b.time_replays(0)
            _note(f"replays wg={wg} u={u} v={v} whole={whole}")
            assert b.time_replays(5) > 0
            pops2 = _pops(rng, mats)
            got = b.evaluate(pops2, sigma=3, max_violations=1, negative_trends=True,
                             want_masks=True)
            _check_runs(mats, pops2, got, 3, 1, True)


@pytest.mark.parametrize("shape", [None, (-1, 2, 8, 1, 1), (0, 4, 2, 0, 1)])
def test_batch_evolve_matches_oracle_runs(E, shape):
    # tuned on the first generation (None), or a fixed shape replayed as a
    # graph whose queue-free grid grows with the largest generation seen
    rng = np.random.default_rng(4)
    shapes = [(150, 20), (300, 12), (90, 30), (500, 8)]
    mats_ = [rng.standard_normal(s).astype(np.float32) for s in shapes]
    seeds = [11, 12, 13, 14]
    G = 6
    cfg = E.EvolveConfig(population=60, len_min=3, len_max=7, eval=E.Trend(8),
                         expand=E.Trend(8, 1, True))
    gens = {r: [] for r in range(len(mats_))}
    with E.Batch(mats_) as b:
        _note(f"batch evolve shape={shape}")
        if shape is not None:
            b.set_tuning(*shape)
        res = b.evolve(seeds, G, cfg, on_generation=lambda r, g: gens[r].append(g), host_threads=3)
    for r, (a, s) in enumerate(zip(mats_, seeds)):
        op = oev.EvolveParams(population=60, len_min=3, len_max=7, eval=oev.TrendParams(8),
                              expand=oev.TrendParams(8, 1, True))
        ref = oev.evolve(a, s, G, op)
        assert len(gens[r]) == len(ref.history)
        for g, h in zip(gens[r], ref.history):
            assert g.population == h.population
            assert np.array_equal(g.counts, h.counts)
            assert np.array_equal(g.fitness.view(np.int64), h.fitness.view(np.int64))
        assert [x["cols"] for x in res[r].biclusters] == [x["cols"] for x in ref.biclusters]
        for x, y in zip(res[r].biclusters, ref.biclusters):
            assert x["count"] == y["count"] and x["fitness"] == y["fitness"]
            assert np.array_equal(x["mask_words"], y["mask_words"])


def test_batched_workload_shapes_one_generation(E):
    # Four runs of the batched setting at full size (up to 50000 rows and
    # 1000 columns), one population each, against the oracle.
    ws = [synth.batched_workload(r) for r in range(4)]
    data = [synth.make_matrix(w) for w in ws]
    rng = np.random.default_rng(5)
    pops = [synth.pack_cbf(synth.mixed_population(rng, w, pl, 256)) for w, (a, pl) in zip(ws, data)]
    with E.Batch([a for a, _ in data]) as b:
        _note("batched workload shapes")
        got = b.evaluate(pops, sigma=25, tune=True)
    _check_runs([a for a, _ in data], pops, got, 25, 0, False, masks=False)


def test_large_tolerance_batches_use_the_direct_kernel(E, mats):
    # k above the index kernel's limit: every run is evaluated by the direct
    # kernel after the (empty) batched launch, with the same results
    rng = np.random.default_rng(31)
    with E.Batch(mats) as b:
        for k in (4, 7):
            for neg in (False, True):
                pops = _pops(rng, mats, skip=(1,))
                _note(f"evaluate k={k} neg={neg}")
                got = b.evaluate(pops, sigma=5, max_violations=k, negative_trends=neg,
                                 want_masks=True)
                _check_runs(mats, pops, got, 5, k, neg)


def test_run_over_its_index_budget_is_evaluated_directly(E):
    # A 60000 x 1200 matrix needs a 10.9 GB order index, over the default
    # 8 GiB budget of its context: its run has no index and is evaluated by
    # the direct kernel, the other runs by the batched index kernel, in the
    # same call; a batched EBIC run equals the oracle's.  Device-side steps
    # need every run's index and refuse the batch.
    rng = np.random.default_rng(33)
    big = rng.standard_normal((60000, 1200)).astype(np.float32)
    small = [rng.standard_normal((300, 14)).astype(np.float32),
             synth.adversarial_matrix(rng, 500, 10)]
    mats_ = [small[0], big, small[1]]
    with E.Batch(mats_) as b:
        _note("evaluate with a directly evaluated run")
        for k, neg in ((0, False), (1, True), (5, True)):
            pops = [synth.pack_cbf(synth.random_population(rng, a.shape[1], 40, 2, 8))
                    for a in mats_]
            got = b.evaluate(pops, sigma=9, max_violations=k, negative_trends=neg,
                             want_masks=True)
            _check_runs(mats_, pops, got, 9, k, neg)
        cfg = E.EvolveConfig(population=40, len_min=3, len_max=6, eval=E.Trend(9),
                             expand=E.Trend(9, 1, True))
        _note("batched run with a directly evaluated run")
        res = b.evolve([5, 6, 7], 2, cfg, host_threads=2)
        for r, (a, s) in enumerate(zip(mats_, (5, 6, 7))):
            op = oev.EvolveParams(population=40, len_min=3, len_max=6, eval=oev.TrendParams(9),
                                  expand=oev.TrendParams(9, 1, True))
            ref = oev.evolve(a, s, 2, op)
            assert [x["cols"] for x in res[r].biclusters] == [x["cols"] for x in ref.biclusters]
            for x, y in zip(res[r].biclusters, ref.biclusters):
                assert x["count"] == y["count"] and x["fitness"] == y["fitness"]
                assert np.array_equal(x["mask_words"], y["mask_words"])
        with pytest.raises(E.EbicError):
            b.evolve([5, 6, 7], 1, cfg, device_steps=True)
