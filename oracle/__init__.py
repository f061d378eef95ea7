"""CPU oracle for EBIC's population evaluation and evolutionary run.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and
the benchmark's ``cpu_baseline`` leg may import this package.  It shares no
code with the HIP library under ``paper_1801_03039_amd/``; the only module
both sides use is ``synth`` (seeded inputs, no method arithmetic).

* ``evaluate``   -- the plain definition of one evaluation (C, ``ebic_oracle.c``)
* ``brute``      -- an independent NumPy formulation for tiny inputs
* ``evolve``     -- the evolutionary run, Steps 1-7, in plain Python
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ebic_oracle.c")
_LIB = os.path.join(_HERE, "libebic_oracle.so")

BUILD_CMD = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared",
             "-fno-fast-math", "-ffp-contract=off", "-o", _LIB, _SRC, "-lm"]

_lib = None


def build() -> str:
    """Compile the C oracle into ``oracle/libebic_oracle.so``."""
    subprocess.run(BUILD_CMD, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i32, i64, p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    lib.oracle_evaluate.restype = ctypes.c_int
    lib.oracle_evaluate.argtypes = [p, i64, i32, i64, p, p, i32, i32, i32, i32,
                                    p, p, p, p, p, i32]
    lib.oracle_fitness.restype = ctypes.c_double
    lib.oracle_fitness.argtypes = [i64, i64, i64]
    lib.oracle_check_population.restype = ctypes.c_int
    lib.oracle_check_population.argtypes = [p, p, i32, i32]
    lib.oracle_max_threads.restype = i32
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def fitness(count: int, length: int, sigma: int) -> float:
    """Eq. (1) for one bicluster with ``count`` rows and ``length`` columns."""
    return float(_load().oracle_fitness(int(count), int(length), int(sigma)))


def evaluate(a: np.ndarray, offsets: np.ndarray, cols: np.ndarray, *, sigma: int,
             max_violations: int = 0, negative_trends: bool = False,
             want_masks: bool = False, want_reads: bool = False,
             want_depth: bool = False, nthreads: int = 0) -> dict:
    """Evaluate a CBF population on the row-major FP32 matrix ``a``.

    Returns ``counts`` (int32[P]), ``fitness`` (float64[P]) and, when asked,
    ``masks`` (uint64[P, 2, W]; dir 0 rising, dir 1 falling) and ``reads``
    (int64[P], the per-candidate sum of values each row must read before its
    decision is fixed) and ``depth`` (int32[P, N], that count per row).
    """
    lib = _load()
    a = np.ascontiguousarray(a, dtype=np.float32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    n, m = a.shape
    P = len(offsets) - 1
    w = (n + 63) // 64
    counts = np.zeros(P, dtype=np.int32)
    fit = np.zeros(P, dtype=np.float64)
    masks = np.zeros((P, 2, w), dtype=np.uint64) if want_masks else None
    reads = np.zeros(P, dtype=np.int64) if want_reads else None
    depth = np.zeros((P, n), dtype=np.int32) if want_depth else None
    st = lib.oracle_evaluate(_ptr(a), n, m, m, _ptr(offsets), _ptr(cols), P,
                             int(sigma), int(max_violations), int(bool(negative_trends)),
                             _ptr(masks), _ptr(counts), _ptr(fit), _ptr(reads), _ptr(depth),
                             int(nthreads))
    if st != 0:
        raise OracleError(st)
    out = {"counts": counts, "fitness": fit}
    if want_masks:
        out["masks"] = masks
    if want_reads:
        out["reads"] = reads
    if want_depth:
        out["depth"] = depth
    return out


def check_population(offsets: np.ndarray, cols: np.ndarray, n_cols: int) -> int:
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    return int(_load().oracle_check_population(_ptr(offsets), _ptr(cols), len(offsets) - 1, n_cols))


def max_threads() -> int:
    return int(_load().oracle_max_threads())
