"""GPU parity: the HIP evaluators against the CPU oracle, element by element.

Masks and counts must be identical and fitness bit-identical (FP64 bit
patterns compared as integers): the kernels make the same IEEE FP32
comparisons and the same one-rounding FP64 fitness as the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

PATHS = ["direct", "index"]


def _note(msg):
    print(f"[parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ebic():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_03039_amd as e
    return e


def _same(gpu, ref, masks=True):
    assert np.array_equal(gpu["counts"], ref["counts"]), \
        np.nonzero(gpu["counts"] != ref["counts"])[0][:10]
    assert np.array_equal(gpu["fitness"].view(np.int64), ref["fitness"].view(np.int64))
    if masks:
        assert np.array_equal(gpu["masks"], ref["masks"])


def _check(ebic, a, series, path, *, sigma, k, neg, masks=True):
    off, cols = synth.pack_cbf(series)
    ref = oracle.evaluate(a, off, cols, sigma=sigma, max_violations=k, negative_trends=neg,
                          want_masks=masks)
    with ebic.Context(a, path=path) as ctx:
        got = ctx.evaluate(off, cols, sigma=sigma, max_violations=k, negative_trends=neg,
                           want_masks=masks)
    _same(got, ref, masks)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n", [1, 63, 64, 65, 130, 257, 1000])
def test_ragged_rows_adversarial_values(ebic, path, n):
    rng = np.random.default_rng(n)
    m = 11
    a = synth.adversarial_matrix(rng, n, m)
    pop = synth.random_population(rng, m, 97, 1, m)    # includes L = 1 and L = M
    for k in (0, 1, 3):
        for neg in (False, True):
            _note(f"ragged path={path} n={n} k={k} neg={neg}")
            _check(ebic, a, pop, path, sigma=7, k=k, neg=neg)


@pytest.mark.parametrize("path", PATHS)
def test_tie_heavy_every_short_series(ebic, path):
    from oracle import brute
    rng = np.random.default_rng(7)
    a = synth.tiny_tie_matrix(rng, 200, 6)
    series = [list(s) for s in brute.all_series(6, 4)]
    for k in (0, 1, 2, 3):
        for neg in (False, True):
            _note(f"ties path={path} k={k} neg={neg}")
            _check(ebic, a, series, path, sigma=3, k=k, neg=neg)


@pytest.mark.parametrize("k", [4, 6, 40])
def test_large_tolerance_uses_direct_and_matches(ebic, k):
    rng = np.random.default_rng(100 + k)
    a = synth.adversarial_matrix(rng, 333, 40)
    pop = synth.random_population(rng, 40, 150, 1, 40)
    _note(f"large k={k}")
    _check(ebic, a, pop, "auto", sigma=9, k=k, neg=True)


@pytest.mark.parametrize("path", PATHS)
def test_long_series_beyond_lds_stage(ebic, path):
    # Series longer than the direct kernel's LDS column stage (512).
    rng = np.random.default_rng(9)
    m = 700
    a = rng.standard_normal((150, m)).astype(np.float32)
    a[:, :] = np.sort(a, axis=1)          # every row rises along 0..m-1
    a[5] = a[5, ::-1]
    pop = [np.arange(m, dtype=np.int32), np.arange(m, dtype=np.int32)[::-1].copy(),
           rng.permutation(m).astype(np.int32)[:600]]
    for k in (0, 1):
        _note(f"long path={path} k={k}")
        _check(ebic, a, pop, path, sigma=10, k=k, neg=True)


@pytest.mark.parametrize("n", [1, 64, 200, 5000, 8192, 8193, 10000, 15000, 20000, 20480, 20481,
                               32768, 32769, 65536, 65537])
def test_tiling_boundary_row_counts(ebic, n):
    # The index evaluator holds whole candidates per workgroup with 1, 2 or
    # 4 words per lane up to 8192, 20480 and 65536 rows, and spreads taller
    # matrices over workgroups; both sides of each switch (and of 32768
    # rows), and heights that pack 1 to 64 candidates per workgroup, with
    # planted rows.
    rng = np.random.default_rng(n)
    m = 24
    a = rng.standard_normal((n, m)).astype(np.float32)
    rows = rng.choice(n, size=min(300, n), replace=False)
    order = rng.permutation(m)[:8]
    a[np.ix_(rows, order)] = np.sort(a[np.ix_(rows, order)], axis=1)
    pop = synth.random_population(rng, m, 150, 2, 10) + [list(order), list(order[:5])]
    for k, neg in ((0, False), (1, True)):
        _note(f"tiling boundary n={n} k={k} neg={neg}")
        _check(ebic, a, pop, "index", sigma=50, k=k, neg=neg)


@pytest.mark.parametrize("name", ["tiny", "expression", "wide"])
@pytest.mark.parametrize("path", PATHS)
def test_workload_populations(ebic, name, path):
    w = synth.WORKLOADS[name]
    a, planted = synth.make_matrix(w)
    rng = np.random.default_rng(1234)
    P = min(w.population, 1024)
    pop = synth.mixed_population(rng, w, planted, P)
    _note(f"workload {name} path={path} P={P}")
    _check(ebic, a, pop, path, sigma=w.sigma, k=w.max_violations, neg=w.negative_trends)


@pytest.mark.parametrize("name", ["expression", "wide", "surrogate"])
def test_full_size_device_entry_point(ebic, name):
    """Full workload size, full population, through the device entry point
    with torch tensors on the current stream, both paths; compared with the
    oracle on every candidate."""
    import torch
    w = synth.WORKLOADS[name]
    a, planted = synth.make_matrix(w)
    rng = np.random.default_rng(77)
    pop = synth.mixed_population(rng, w, planted, w.population)
    off, cols = synth.pack_cbf(pop)
    ref = oracle.evaluate(a, off, cols, sigma=w.sigma, max_violations=w.max_violations,
                          negative_trends=w.negative_trends, want_masks=True)
    dev = torch.device("cuda:0")
    d_off = torch.from_numpy(off).to(dev)
    d_cols = torch.from_numpy(cols).to(dev)
    P = len(pop)
    with ebic.Context(torch.from_numpy(a).to(dev)) as ctx:
        for path in PATHS:
            _note(f"full device {name} path={path}")
            ctx.set_path(path)
            counts = torch.full((P,), -7, dtype=torch.int32, device=dev)
            fit = torch.full((P,), -7.0, dtype=torch.float64, device=dev)
            masks = torch.zeros((P, 2, ctx.W), dtype=torch.int64, device=dev)
            ctx.evaluate_device(d_off, d_cols, counts, fit, masks, sigma=w.sigma,
                                max_violations=w.max_violations,
                                negative_trends=w.negative_trends)
            torch.cuda.synchronize()
            got = {"counts": counts.cpu().numpy(), "fitness": fit.cpu().numpy(),
                   "masks": masks.cpu().numpy().view(np.uint64)}
            _same(got, ref)


def test_paths_agree_and_repeat_bit_identically(ebic):
    w = synth.WORKLOADS["expression"]
    a, planted = synth.make_matrix(w)
    rng = np.random.default_rng(5)
    pop = synth.mixed_population(rng, w, planted, 512)
    off, cols = synth.pack_cbf(pop)
    with ebic.Context(a) as ctx:
        outs = []
        for path in PATHS * 3:
            ctx.set_path(path)
            outs.append(ctx.evaluate(off, cols, sigma=w.sigma, max_violations=1,
                                     negative_trends=True, want_masks=True))
        for o in outs[1:]:
            _same(o, outs[0])


def test_row_sharded_counts_sum(ebic):
    # One GPU's share of a row-sharded matrix: counts over row slices cut at
    # multiples of 64 add up to the whole-matrix counts, and the slices'
    # masks tile the whole mask.
    w = synth.WORKLOADS["expression"]
    a, planted = synth.make_matrix(w)
    rng = np.random.default_rng(6)
    pop = synth.mixed_population(rng, w, planted, 256)
    off, cols = synth.pack_cbf(pop)
    with ebic.Context(a) as ctx:
        whole = ctx.evaluate(off, cols, sigma=w.sigma, max_violations=1, negative_trends=True,
                             want_masks=True)
    cuts = [0, 64 * 40, 64 * 160, a.shape[0]]
    total = np.zeros(len(pop), dtype=np.int64)
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        with ebic.Context(a[lo:hi]) as ctx:
            part = ctx.evaluate(off, cols, sigma=w.sigma, max_violations=1, negative_trends=True,
                                want_masks=True)
        total += part["counts"]
        assert np.array_equal(part["masks"], whole["masks"][:, :, lo // 64:lo // 64 + part["masks"].shape[2]])
    assert np.array_equal(total, whole["counts"])


def test_malformed_candidates_on_device(ebic):
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(8)
    a = rng.standard_normal((300, 9)).astype(np.float32)
    good = [[0, 1, 2], [3, 4], [5, 6, 7, 8]]
    off, cols = synth.pack_cbf(good)
    ref = oracle.evaluate(a, off, cols, sigma=3, negative_trends=True)
    # candidate 1 gets an out-of-range column, candidate 2 a bad offset span
    bad_cols = cols.copy()
    bad_cols[3] = 99
    bad_off = np.array([0, 3, 5, 50], dtype=np.int32)
    with ebic.Context(a) as ctx:
        for path in PATHS:
            ctx.set_path(path)
            _note(f"malformed path={path}")
            counts = torch.zeros(3, dtype=torch.int32, device=dev)
            fit = torch.zeros(3, dtype=torch.float64, device=dev)
            ctx.evaluate_device(torch.from_numpy(bad_off).to(dev), torch.from_numpy(bad_cols).to(dev),
                                counts, fit, sigma=3, negative_trends=True)
            torch.cuda.synchronize()
            c = counts.cpu().numpy()
            f = fit.cpu().numpy()
            assert c[0] == ref["counts"][0] and f[0] == ref["fitness"][0]
            assert c[1] == -1 and np.isnan(f[1])
            assert c[2] == -1 and np.isnan(f[2])
            # the context is still healthy afterwards
            got = ctx.evaluate(off, cols, sigma=3, negative_trends=True)
            assert np.array_equal(got["counts"], ref["counts"])


def test_host_entry_point_errors(ebic):
    rng = np.random.default_rng(9)
    a = rng.standard_normal((100, 6)).astype(np.float32)
    with ebic.Context(a) as ctx:
        E = ebic.binding
        cases = [
            (np.array([0, 2]), np.array([0, 6]), 3, 0, E.EBIC_E_RANGE),
            (np.array([0, 2]), np.array([1, 1]), 3, 0, E.EBIC_E_ARG),
            (np.array([1, 2]), np.array([1, 2]), 3, 0, E.EBIC_E_ARG),
            (np.array([0, 0]), np.array([1]), 3, 0, E.EBIC_E_ARG),
            (np.array([0, 2]), np.array([1, 2]), -1, 0, E.EBIC_E_RANGE),
            (np.array([0, 2]), np.array([1, 2]), 3, -2, E.EBIC_E_RANGE),
        ]
        for off, cols, sigma, k, st in cases:
            with pytest.raises(ebic.EbicError) as ex:
                ctx.evaluate(off, cols, sigma=sigma, max_violations=k)
            assert ex.value.status == st
        empty = ctx.evaluate(np.array([0]), np.array([], dtype=np.int32), sigma=1)
        assert empty["counts"].size == 0
