"""CPU oracle for the outputs of Steps 6-7 and the accuracy scores of
Section 3 (Eqs. 2-3).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

* ``mask_rows``    -- Step 6: the indices of the rows a bicluster matches,
                      read bit by bit from its 64-row masks (bit r mod 64 of
                      word r // 64; several planes, e.g. the rising and the
                      falling direction, are united; bits at or beyond
                      ``n_rows`` are not rows).
* ``jaccard``      -- the Jaccard index of two biclusters taken as sets of
                      matrix cells (rows x columns).  A bicluster's column
                      series counts as the set of its columns.
* ``match_scores`` -- Eq. (2) recovery and Eq. (3) relevance.  The paper
                      prints both as bare sums but reports them as shares
                      up to 100 %; we divide recovery by the number of
                      expected biclusters and relevance by the number found.
                      Sums run in index order.  With nothing expected or
                      nothing found both scores are 0, and the index of two
                      empty biclusters is 0.
"""
from __future__ import annotations

import numpy as np


def mask_rows(masks, n_rows: int):
    """masks: uint64 array [K][planes][W] (or [K][W]).  Returns a list of K
    int32 arrays of row indices in increasing order."""
    m = np.asarray(masks, dtype=np.uint64)
    if m.ndim == 2:
        m = m[:, None, :]
    K, planes, W = m.shape
    out = []
    for k in range(K):
        rows = []
        for w in range(W):
            word = 0
            for p in range(planes):
                word |= int(m[k, p, w])
            for b in range(64):
                r = w * 64 + b
                if r < n_rows and (word >> b) & 1:
                    rows.append(r)
        out.append(np.array(rows, dtype=np.int32))
    return out


def jaccard(rows_a, cols_a, rows_b, cols_b) -> float:
    """|A n B| / |A u B| for A = rows_a x set(cols_a), B = rows_b x set(cols_b)."""
    ra, rb = set(int(r) for r in rows_a), set(int(r) for r in rows_b)
    ca, cb = set(int(c) for c in cols_a), set(int(c) for c in cols_b)
    inter = len(ra & rb) * len(ca & cb)
    union = len(ra) * len(ca) + len(rb) * len(cb) - inter
    if union == 0:
        return 0.0
    return float(inter) / float(union)


def match_scores(found, expected):
    """found, expected: sequences of (rows, cols).  Returns (J, recovery,
    relevance) with J[f][e] the Jaccard index of found f and expected e."""
    F, E = len(found), len(expected)
    J = np.zeros((F, E), dtype=np.float64)
    for f in range(F):
        for e in range(E):
            J[f, e] = jaccard(found[f][0], found[f][1], expected[e][0], expected[e][1])
    if F == 0 or E == 0:
        return J, 0.0, 0.0
    rec = 0.0
    for e in range(E):
        rec += float(J[:, e].max())
    rel = 0.0
    for f in range(F):
        rel += float(J[f, :].max())
    return J, rec / E, rel / F
