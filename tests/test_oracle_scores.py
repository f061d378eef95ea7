"""CPU pins of the Step 6 row lists and the accuracy scores (Section 3,
Eqs. 2-3) in oracle/scores.py: a hand-worked example, brute force over cell
sets, bit-level unpacking by an independent route, and the identities the
definitions imply."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import scores

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "jaccard_eq2_eq3.json")


def _cells(rows, cols):
    return {(int(r), int(c)) for r in rows for c in cols}


def _brute_jaccard(a, b):
    A, B = _cells(*a), _cells(*b)
    u = A | B
    return len(A & B) / len(u) if u else 0.0


def _random_bicluster(rng, n, m):
    rows = rng.choice(n, size=int(rng.integers(0, n + 1)), replace=False)
    cols = rng.choice(m, size=int(rng.integers(1, m + 1)), replace=False)
    if rng.random() < 0.3:                      # a repeated column counts once
        cols = np.concatenate([cols, cols[:1]])
    return np.sort(rows), cols


def test_hand_worked_example():
    g = json.load(open(GOLDEN))
    found = [(f["rows"], f["cols"]) for f in g["found"]]
    expected = [(e["rows"], e["cols"]) for e in g["expected"]]
    J, rec, rel = scores.match_scores(found, expected)
    assert np.allclose(J, g["jaccard"], rtol=0, atol=1e-15)
    assert rec == pytest.approx(g["recovery"], abs=1e-15)
    assert rel == pytest.approx(g["relevance"], abs=1e-15)


def test_jaccard_equals_cell_set_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(400):
        n, m = int(rng.integers(1, 12)), int(rng.integers(1, 8))
        a, b = _random_bicluster(rng, n, m), _random_bicluster(rng, n, m)
        assert scores.jaccard(*a, *b) == _brute_jaccard(a, b)


def test_scores_identities():
    rng = np.random.default_rng(1)
    for _ in range(50):
        n, m = 30, 10
        E = [_random_bicluster(rng, n, m) for _ in range(int(rng.integers(1, 5)))]
        F = [_random_bicluster(rng, n, m) for _ in range(int(rng.integers(1, 6)))]
        J, rec, rel = scores.match_scores(F, E)
        J2, rec2, rel2 = scores.match_scores(E, F)
        assert np.array_equal(J, J2.T)
        assert rec == rel2 and rel == rec2           # the two scores swap with the roles
        assert 0.0 <= rec <= 1.0 and 0.0 <= rel <= 1.0
        nonempty = [e for e in E if len(e[0])]
        if nonempty:
            _, r_self, l_self = scores.match_scores(nonempty, nonempty)
            assert r_self == 1.0 and l_self == 1.0   # a perfect answer scores 1
        # adding a found bicluster can only raise recovery
        _, rec3, _ = scores.match_scores(F + [_random_bicluster(rng, n, m)], E)
        assert rec3 >= rec


def test_subset_and_disjoint_closed_forms():
    big = (np.arange(10), np.arange(4))
    small = (np.arange(3), np.arange(2))
    assert scores.jaccard(*small, *big) == 6 / 40
    assert scores.jaccard(*big, *(np.arange(10, 20), np.arange(4))) == 0.0
    assert scores.jaccard(*big, *(np.arange(10), np.arange(4, 8))) == 0.0
    assert scores.jaccard([], [0], [], [1]) == 0.0
    J, rec, rel = scores.match_scores([], [big])
    assert J.shape == (0, 1) and rec == 0.0 and rel == 0.0


def test_mask_rows_matches_unpackbits():
    rng = np.random.default_rng(2)
    for n in (1, 63, 64, 65, 200, 1000):
        W = (n + 63) // 64
        K, planes = 7, int(rng.integers(1, 3))
        masks = rng.integers(0, 2**63, size=(K, planes, W), dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, size=(K, planes, W), dtype=np.uint64)
        masks[0] = 0
        got = scores.mask_rows(masks, n)
        union = np.bitwise_or.reduce(masks, axis=1)
        bits = np.unpackbits(union.view(np.uint8).reshape(K, W, 8), axis=2, bitorder="little")
        for k in range(K):
            want = np.flatnonzero(bits[k].reshape(-1)[:n])
            assert np.array_equal(got[k], want), (n, k)


def test_mask_rows_inverts_row_packing():
    rng = np.random.default_rng(3)
    n = 333
    rows = [np.sort(rng.choice(n, size=int(rng.integers(0, n)), replace=False)) for _ in range(9)]
    masks = synth.rows_to_masks(rows, n)
    for k, r in enumerate(scores.mask_rows(masks, n)):
        assert np.array_equal(r, rows[k])
