"""Pins for the CPU oracle's evaluation (no GPU).

Each test fixes the oracle to something other than itself: values worked by
hand from Eq. (1), the Fig. 2 CBF example, an independent NumPy formulation
(brute force over every short series), exact invariants of the trend rule,
planted structure, and the match statistics of i.i.d. data (Eulerian
numbers) that the Motivation's halving argument rests on.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute


def _eval(a, series, **kw):
    off, cols = synth.pack_cbf(series)
    return oracle.evaluate(a, off, cols, want_masks=True, **kw)


def _bool_masks(res, n):
    """uint64 words [P,2,W] -> bool [P,2,N]."""
    words = res["masks"]
    P = words.shape[0]
    out = np.zeros((P, 2, n), dtype=bool)
    for r in range(n):
        out[:, :, r] = (words[:, :, r // 64] >> np.uint64(r % 64)) & np.uint64(1)
    return out


# --- Eq. (1) ---------------------------------------------------------------

def test_fitness_hand_values(golden_dir):
    with open(os.path.join(golden_dir, "fitness_eq1.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        got = oracle.fitness(c["count"], c["length"], c["sigma"])
        assert got == c["fitness"], c


def test_fitness_through_evaluate():
    # 30 planted rows x 8 columns, sigma 20: the evaluate path must give the
    # same Eq. (1) value as the hand computation 8 ln 29 (golden above).
    rng = np.random.default_rng(5)
    n, L = 30, 8
    a = np.sort(rng.standard_normal((n, L)), axis=1).astype(np.float32)
    res = _eval(a, [list(range(L))], sigma=20)
    assert res["counts"][0] == 30
    assert res["fitness"][0] == 26.938366639891793


def test_fitness_sigma_scaling_is_exact_power_of_two():
    # Below sigma each missing row halves f exactly.
    for count in range(2, 40):
        f = oracle.fitness(count, 7, 40)
        g = oracle.fitness(count, 7, count)   # exponent 0
        assert f == math.ldexp(g, count - 40)


# --- CBF, Fig. 2 -------------------------------------------------------------

def test_cbf_fig2(golden_dir):
    with open(os.path.join(golden_dir, "cbf_fig2.json")) as f:
        g = json.load(f)
    series = [[c - 1 for c in s] for s in g["series_1based"]]
    off, cols = synth.pack_cbf(series)
    assert off.tolist() == g["offsets"]
    assert off[:-1].tolist() == g["starts"]
    assert cols.tolist() == g["cols_0based"]
    back = synth.unpack_cbf(off, cols)
    assert [b.tolist() for b in back] == series
    # Evaluating the packed population equals evaluating each series alone.
    rng = np.random.default_rng(0)
    a = rng.standard_normal((300, 5)).astype(np.float32)
    whole = oracle.evaluate(a, off, cols, sigma=3, negative_trends=True, want_masks=True)
    for i, s in enumerate(series):
        one = _eval(a, [s], sigma=3, negative_trends=True)
        assert one["counts"][0] == whole["counts"][i]
        assert one["fitness"][0] == whole["fitness"][i]
        assert np.array_equal(one["masks"][0], whole["masks"][i])


# --- brute force over every short series ---------------------------------------

@pytest.mark.parametrize("seed,n,m,max_len", [(0, 70, 6, 4), (1, 130, 7, 3), (2, 64, 5, 4)])
def test_brute_force_every_series(seed, n, m, max_len):
    rng = np.random.default_rng(seed)
    a = synth.tiny_tie_matrix(rng, n, m)
    series = list(brute.all_series(m, max_len))
    for k in (0, 1, 2):
        for neg in (False, True):
            res = _eval(a, series, sigma=2, max_violations=k, negative_trends=neg)
            bm = _bool_masks(res, n)
            for i, s in enumerate(series):
                up, dn, cnt = brute.evaluate_series(a, s, k, neg)
                assert np.array_equal(bm[i, 0], up), (s, k, neg)
                assert np.array_equal(bm[i, 1], dn), (s, k, neg)
                assert res["counts"][i] == cnt


def test_rank_formulation_exact():
    rng = np.random.default_rng(11)
    a = synth.tiny_tie_matrix(rng, 200, 6)
    series = list(brute.all_series(6, 4))
    res = _eval(a, series, sigma=1, negative_trends=True)
    bm = _bool_masks(res, 200)
    for i, s in enumerate(series):
        up, dn = brute.evaluate_exact_rank(a, s)
        assert np.array_equal(bm[i, 0], up)
        assert np.array_equal(bm[i, 1], dn)


def test_adversarial_values_against_brute():
    rng = np.random.default_rng(3)
    a = synth.adversarial_matrix(rng, 257, 9)
    pop = synth.random_population(rng, 9, 300, 1, 9)
    for k in (0, 1, 3):
        res = _eval(a, pop, sigma=4, max_violations=k, negative_trends=True)
        bm = _bool_masks(res, 257)
        for i, s in enumerate(pop):
            up, dn, cnt = brute.evaluate_series(a, s, k, True)
            assert np.array_equal(bm[i, 0], up)
            assert np.array_equal(bm[i, 1], dn)
            assert res["counts"][i] == cnt


def test_special_values_semantics():
    # Strict comparison (Motivation): ties, +0/-0 and NaN break both
    # directions; infinities order normally; denormals are ordered.
    f = np.float32
    tiny = np.float32(1e-45)
    rows = [
        ([1, 2], (True, False)),
        ([2, 1], (False, True)),
        ([1, 1], (False, False)),
        ([0.0, -0.0], (False, False)),
        ([np.nan, 1], (False, False)),
        ([1, np.nan], (False, False)),
        ([-np.inf, np.inf], (True, False)),
        ([np.inf, np.inf], (False, False)),
        ([-tiny, tiny], (True, False)),
        ([0.0, tiny], (True, False)),
        ([tiny, 0.0], (False, True)),
    ]
    a = np.array([r for r, _ in rows], dtype=f)
    res = _eval(a, [[0, 1]], sigma=0, negative_trends=True)
    bm = _bool_masks(res, len(rows))
    for i, (_, (up, dn)) in enumerate(rows):
        assert (bool(bm[0, 0, i]), bool(bm[0, 1, i])) == (up, dn), rows[i]


# --- closed-form special cases -------------------------------------------------

def test_single_column_and_large_tolerance_accept_every_row():
    rng = np.random.default_rng(4)
    a = synth.adversarial_matrix(rng, 150, 12)
    pop = synth.random_population(rng, 12, 40, 1, 12)
    singles = [[j] for j in range(12)]
    r1 = _eval(a, singles, sigma=0)
    assert np.all(r1["counts"] == 150)
    for s in pop:
        r = _eval(a, [s], sigma=0, max_violations=len(s) - 1)
        assert r["counts"][0] == 150


# --- invariants -------------------------------------------------------------------

def _pop(rng, m, p, lo, hi):
    return synth.random_population(rng, m, p, lo, hi)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_reversal_swaps_directions(k):
    rng = np.random.default_rng(10 + k)
    a = synth.adversarial_matrix(rng, 190, 11)
    pop = _pop(rng, 11, 120, 2, 8)
    fwd = _eval(a, pop, sigma=0, max_violations=k, negative_trends=True)
    rev = _eval(a, [s[::-1] for s in pop], sigma=0, max_violations=k, negative_trends=True)
    assert np.array_equal(fwd["masks"][:, 0], rev["masks"][:, 1])
    assert np.array_equal(fwd["masks"][:, 1], rev["masks"][:, 0])
    assert np.array_equal(fwd["counts"], rev["counts"])


@pytest.mark.parametrize("k", [0, 1])
def test_negation_swaps_directions(k):
    rng = np.random.default_rng(20 + k)
    a = synth.adversarial_matrix(rng, 200, 10)
    pop = _pop(rng, 10, 100, 2, 7)
    pos = _eval(a, pop, sigma=0, max_violations=k, negative_trends=True)
    neg = _eval(-a, pop, sigma=0, max_violations=k, negative_trends=True)
    assert np.array_equal(pos["masks"][:, 0], neg["masks"][:, 1])
    assert np.array_equal(pos["masks"][:, 1], neg["masks"][:, 0])


@pytest.mark.parametrize("k", [0, 1, 2])
def test_subsequence_never_loses_rows(k):
    rng = np.random.default_rng(30 + k)
    a = synth.adversarial_matrix(rng, 170, 12)
    pop = _pop(rng, 12, 80, 3, 9)
    subs = []
    for s in pop:
        keep = np.sort(rng.choice(len(s), size=int(rng.integers(1, len(s))), replace=False))
        subs.append(s[keep])
    full = _eval(a, pop, sigma=0, max_violations=k, negative_trends=True)
    part = _eval(a, subs, sigma=0, max_violations=k, negative_trends=True)
    # Every row matching the series matches the order-preserving subsequence.
    assert np.all((full["masks"] & ~part["masks"]) == 0)
    assert np.all(part["counts"] >= full["counts"])


def test_row_permutation_and_column_relabel():
    rng = np.random.default_rng(40)
    n, m = 230, 13
    a = synth.adversarial_matrix(rng, n, m)
    pop = _pop(rng, m, 90, 2, 9)
    base = _eval(a, pop, sigma=5, max_violations=1, negative_trends=True)
    perm = rng.permutation(n)
    pr = _eval(a[perm], pop, sigma=5, max_violations=1, negative_trends=True)
    assert np.array_equal(base["counts"], pr["counts"])
    assert np.array_equal(base["fitness"], pr["fitness"])
    bb, pb = _bool_masks(base, n), _bool_masks(pr, n)
    assert np.array_equal(bb[:, :, perm], pb)
    relabel = rng.permutation(m)             # new column relabel[j] holds old column j
    a2 = np.empty_like(a)
    a2[:, relabel] = a
    pop2 = [relabel[s] for s in pop]
    rl = _eval(a2, pop2, sigma=5, max_violations=1, negative_trends=True)
    assert np.array_equal(base["masks"], rl["masks"])


def test_exact_scaling_by_two():
    rng = np.random.default_rng(50)
    a = rng.standard_normal((300, 10)).astype(np.float32)
    a[rng.random(a.shape) < 0.05] = 0.0
    pop = _pop(rng, 10, 100, 2, 8)
    x = _eval(a, pop, sigma=3, max_violations=1, negative_trends=True)
    y = _eval(a * np.float32(2), pop, sigma=3, max_violations=1, negative_trends=True)
    assert np.array_equal(x["masks"], y["masks"])


# --- planted structure ----------------------------------------------------------------

@pytest.mark.parametrize("name", ["tiny"])
def test_planted_rows_match(name):
    w = synth.WORKLOADS[name]
    a, planted = synth.make_matrix(w)
    n = a.shape[0]
    rng = np.random.default_rng(99)
    for pb in planted:
        series = [pb.cols]
        for _ in range(5):
            keep = np.sort(rng.choice(len(pb.cols), size=int(rng.integers(2, len(pb.cols) + 1)), replace=False))
            series.append(pb.cols[keep])
        res = _eval(a, series, sigma=w.sigma, negative_trends=True)
        bm = _bool_masks(res, n)
        d = 1 if pb.descending else 0
        for i in range(len(series)):
            assert np.all(bm[i, d, pb.rows]), (pb.cols, series[i])


def test_planted_rows_match_expression_subset():
    # Same check on the expression-shaped recipe (both directions planted),
    # restricted to the planted rows to keep it quick.
    w = synth.WORKLOADS["expression"]
    a, planted = synth.make_matrix(w)
    for pb in planted:
        sub = a[pb.rows]
        res = _eval(sub, [pb.cols, pb.cols[::-1]], sigma=0, negative_trends=True)
        d = 1 if pb.descending else 0
        assert res["counts"][0] == len(pb.rows)
        bm = _bool_masks(res, len(pb.rows))
        assert np.all(bm[0, d]) and np.all(bm[1, 1 - d])


# --- statistics of i.i.d. data (Motivation) ---------------------------------------------

def test_eulerian_probabilities_closed_form():
    assert brute.match_probability(3, 0) == 1 / 6
    assert abs(brute.match_probability(3, 1) - 5 / 6) < 1e-15
    assert abs(brute.match_probability(5, 1) - 0.225) < 1e-15
    assert brute.match_probability(4, 3) == 1.0


@pytest.mark.parametrize("L,k,neg", [(2, 0, False), (3, 0, False), (4, 0, True), (5, 1, False),
                                     (5, 1, True), (6, 2, False)])
def test_match_rate_of_iid_rows(L, k, neg):
    rng = np.random.default_rng(1000 + 10 * L + k)
    n = 60000
    a = rng.standard_normal((n, L)).astype(np.float32)
    res = _eval(a, [list(range(L))], sigma=0, max_violations=k, negative_trends=neg)
    p = brute.match_probability(L, k)
    if neg:
        # both directions; the union double-counts rows accepted both ways
        q = sum(brute.eulerian(L, d) for d in range(max(0, L - 1 - k), min(k, L - 1) + 1)) / math.factorial(L)
        p = 2 * p - q
    mean, sd = n * p, math.sqrt(n * p * (1 - p))
    assert abs(res["counts"][0] - mean) < 5 * sd + 1e-9, (res["counts"][0], mean, sd)


# --- bytes accounting -------------------------------------------------------------------

def test_values_read_by_brute_force():
    rng = np.random.default_rng(60)
    a = synth.tiny_tie_matrix(rng, 90, 7)
    pop = _pop(rng, 7, 60, 1, 7)
    for k in (0, 1):
        for neg in (False, True):
            off, cols = synth.pack_cbf(pop)
            res = oracle.evaluate(a, off, cols, sigma=0, max_violations=k,
                                  negative_trends=neg, want_reads=True, want_depth=True)
            assert np.array_equal(res["depth"].sum(axis=1), res["reads"])
            for i, s in enumerate(pop):
                total = 0
                for r in range(a.shape[0]):
                    v = a[r, s].astype(np.float64)
                    d = len(s)
                    for t in range(1, len(s)):
                        up_ok, dn_ok = brute.row_matches(v[:t + 1], k)
                        # decided once every enabled direction already fails
                        if (not up_ok) and (not neg or not dn_ok):
                            d = t + 1
                            break
                    assert res["depth"][i, r] == d
                    total += d
                assert res["reads"][i] == total


# --- error handling -----------------------------------------------------------------------

def test_population_errors():
    a = np.zeros((10, 4), dtype=np.float32)
    E_ARG, E_RANGE = 1, 2
    assert oracle.check_population(np.array([0, 2]), np.array([0, 4]), 4) == E_RANGE
    assert oracle.check_population(np.array([0, 2]), np.array([-1, 2]), 4) == E_RANGE
    assert oracle.check_population(np.array([0, 2]), np.array([1, 1]), 4) == E_ARG
    assert oracle.check_population(np.array([1, 2]), np.array([1, 2]), 4) == E_ARG
    assert oracle.check_population(np.array([0, 0]), np.array([], dtype=np.int32), 4) == E_ARG
    assert oracle.check_population(np.array([0]), np.array([], dtype=np.int32), 4) == 0
    with pytest.raises(oracle.OracleError):
        oracle.evaluate(a, np.array([0, 1]), np.array([7]), sigma=0)
    with pytest.raises(oracle.OracleError):
        oracle.evaluate(a, np.array([0, 1]), np.array([1]), sigma=-1)
