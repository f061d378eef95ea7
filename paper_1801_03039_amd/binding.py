"""ctypes binding of libebic (include/ebic.h).

Argument marshalling only: every step of an evaluation runs in the HIP
kernels of ``libebic.so``.  There is no CPU fallback -- importing this module
without the built library raises ``ImportError``.

PyTorch is used only for device memory and streams: the ``*_device`` calls
take CUDA/HIP tensors and launch on torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebic.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libebic.so is not built ({LIB_PATH}); run "
                      "`python -m paper_1801_03039_amd.build` (or __graft_entry__.build())")

# PyTorch-ROCm ships its own HIP runtime under the same SONAME
# (libamdhip64.so.7) as /opt/rocm's.  Loading torch first makes the dynamic
# loader bind libebic to torch's already-loaded runtime, so the process holds
# one HIP/HSA runtime and torch's device pointers and streams are valid for
# libebic.  Loading libebic first would bring in a second runtime.
try:
    import torch  # noqa: F401
except ImportError:  # CPU-only use (argument checks, ebic_evolve_with)
    torch = None

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- ABI types --

EBIC_OK, EBIC_E_ARG, EBIC_E_RANGE, EBIC_E_NOMEM, EBIC_E_DEVICE, EBIC_E_STATE = range(6)
EBIC_ROW_MAJOR, EBIC_COL_MAJOR = 0, 1
EBIC_PATH_AUTO, EBIC_PATH_DIRECT, EBIC_PATH_INDEX = 0, 1, 2
PATHS = {"auto": EBIC_PATH_AUTO, "direct": EBIC_PATH_DIRECT, "index": EBIC_PATH_INDEX}

STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_RANGE", 3: "E_NOMEM", 4: "E_DEVICE", 5: "E_STATE"}

_i32, _i64, _u32, _u64, _vp, _dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                     ctypes.c_uint64, ctypes.c_void_p, ctypes.c_double)


class Params(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("sigma", _i32), ("max_violations", _i32),
                ("negative_trends", _i32), ("want_masks", _i32)]


class CtxInfo(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("device", _i32), ("n_rows", _i64), ("n_cols", _i32),
                ("rows_padded", _i64), ("mask_words", _i64), ("path", _i32),
                ("index_built", _i32), ("index_bytes", _i64), ("index_budget", _i64),
                ("index_build_ms", _dbl), ("index_ties", _i32)]


GENERATION_FN = ctypes.CFUNCTYPE(None, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                 _i32, ctypes.POINTER(_i32), ctypes.POINTER(_dbl))
EVAL_FN = ctypes.CFUNCTYPE(_i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32,
                           ctypes.POINTER(Params), ctypes.POINTER(_u64), ctypes.POINTER(_i32),
                           ctypes.POINTER(_dbl))


class EvolveParamsC(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("population", _i32), ("len_min", _i32),
                ("len_max", _i32), ("tournament", _i32), ("op_weight", _i32 * 5),
                ("elite_num", _i32), ("elite_den", _i32), ("penalty_base", _dbl),
                ("overlap", _dbl), ("toplist_size", _i32), ("tabu_limit", _i32),
                ("eval", Params), ("expand", Params), ("on_generation", GENERATION_FN),
                ("user", _vp)]


class RunStats(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("generations_run", _i32), ("stopped_by_tabu", _i32),
                ("candidates_evaluated", _i64), ("wall_ms", _dbl), ("eval_ms", _dbl),
                ("host_ms", _dbl)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_P = ctypes.POINTER
_create = _sig("ebic_create", _i32, [_vp, _i64, _i32, _i64, _i32, _i32, _P(_vp)])
_create_device = _sig("ebic_create_device", _i32, [_vp, _i64, _i32, _i64, _i32, _i32, _P(_vp)])
_destroy = _sig("ebic_destroy", _i32, [_vp])
_mask_words = _sig("ebic_mask_words", _i64, [_i64])
_set_path = _sig("ebic_set_path", _i32, [_vp, _i32])
_set_budget = _sig("ebic_set_index_budget", _i32, [_vp, _i64])
_get_info = _sig("ebic_get_info", _i32, [_vp, _P(CtxInfo)])
_evaluate = _sig("ebic_evaluate", _i32, [_vp, _vp, _vp, _i32, _P(Params), _vp, _vp, _vp])
_evaluate_device = _sig("ebic_evaluate_device", _i32,
                        [_vp, _vp, _vp, _i32, _i64, _P(Params), _vp, _vp, _vp, _vp])
_evaluate_device_noalloc = _sig("ebic_evaluate_device_noalloc", _i32,
                                [_vp, _vp, _vp, _i32, _i64, _P(Params), _vp, _vp, _vp, _vp])
NOALLOC_MAX_CANDIDATES = 65536
_synchronize = _sig("ebic_synchronize", _i32, [_vp])
_last_error = _sig("ebic_last_error", ctypes.c_char_p, [_vp])

EXPORTED = ["ebic_create", "ebic_create_device", "ebic_destroy", "ebic_mask_words",
            "ebic_set_path", "ebic_set_index_budget", "ebic_get_info", "ebic_evaluate",
            "ebic_evaluate_device", "ebic_evaluate_device_noalloc", "ebic_synchronize",
            "ebic_last_error"]


class EbicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(st: int, ctx=None):
    if st != EBIC_OK:
        raise EbicError(st, _last_error(ctx).decode(errors="replace"))


def mask_words(n_rows: int) -> int:
    return int(_mask_words(int(n_rows)))


def make_params(sigma: int, max_violations: int = 0, negative_trends: bool = False,
                want_masks: bool = False) -> Params:
    return Params(ctypes.sizeof(Params), int(sigma), int(max_violations),
                  int(bool(negative_trends)), int(bool(want_masks)))


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_vp)


def _strided_layout(shape, strides):
    """(layout, ld) of a 2-D float32 view with element strides, if the
    library can read it in place: rows or columns contiguous with a leading
    dimension at least the row or column length; else None."""
    n, m = shape
    s0, s1 = strides
    if s1 == 1 and (s0 >= m or n == 1):
        return EBIC_ROW_MAJOR, max(s0, m) if n > 1 else m
    if s0 == 1 and (s1 >= n or m == 1):
        return EBIC_COL_MAJOR, max(s1, n) if m > 1 else n
    return None


class Context:
    """A matrix resident on one GPU (``ebic_create``).  A float32 matrix view
    whose rows (or columns) are contiguous is read in place, with its leading
    dimension (EBIC_ROW_MAJOR / EBIC_COL_MAJOR); other views are copied."""

    def __init__(self, a, device: int = 0, path: str = "auto"):
        h = _vp()
        if hasattr(a, "is_cuda") and a.is_cuda:
            t = a
            if t.dtype.itemsize != 4 or not t.dtype.is_floating_point:
                raise TypeError("matrix must be float32")
            if t.dim() != 2:
                raise ValueError("matrix must be 2-D")
            n, m = t.shape
            lay = _strided_layout((n, m), t.stride())
            if lay is None:
                t = t.contiguous()
                lay = (EBIC_ROW_MAJOR, m)
            _check(_create_device(_vp(t.data_ptr()), n, m, lay[1], lay[0],
                                  int(t.device.index or 0), ctypes.byref(h)))
        else:
            arr = np.asarray(a)
            if arr.dtype != np.float32 or arr.ndim != 2:
                arr = np.asarray(arr, dtype=np.float32)
            if arr.ndim != 2:
                raise ValueError("matrix must be 2-D")
            n, m = arr.shape
            lay = _strided_layout((n, m), tuple(x // 4 for x in arr.strides))
            if lay is None or any(x % 4 for x in arr.strides):
                arr = np.ascontiguousarray(arr)
                lay = (EBIC_ROW_MAJOR, m)
            _check(_create(_vp(arr.ctypes.data), n, m, lay[1], lay[0], int(device),
                           ctypes.byref(h)))
        self._h = h
        self.n_rows, self.n_cols = int(n), int(m)
        self.W = mask_words(self.n_rows)
        if path != "auto":
            self.set_path(path)

    @property
    def handle(self):
        if not self._h:
            raise EbicError(EBIC_E_STATE, "context is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_path(self, path: str):
        _check(_set_path(self.handle, PATHS[path]), self.handle)

    def set_index_budget(self, nbytes: int):
        _check(_set_budget(self.handle, int(nbytes)), self.handle)

    def info(self) -> dict:
        inf = CtxInfo()
        inf.struct_size = ctypes.sizeof(CtxInfo)
        _check(_get_info(self.handle, ctypes.byref(inf)), self.handle)
        return {f: getattr(inf, f) for f, _ in CtxInfo._fields_ if f != "struct_size"}

    def synchronize(self):
        _check(_synchronize(self.handle), self.handle)

    # -- host arrays ------------------------------------------------------------
    def evaluate(self, offsets, cols, *, sigma: int, max_violations: int = 0,
                 negative_trends: bool = False, want_masks: bool = False) -> dict:
        """Blocking evaluation of a CBF population given as host arrays."""
        off = np.ascontiguousarray(offsets, dtype=np.int32)
        cl = np.ascontiguousarray(cols, dtype=np.int32)
        P = len(off) - 1
        counts = np.zeros(P, dtype=np.int32)
        fit = np.zeros(P, dtype=np.float64)
        masks = np.zeros((P, 2, self.W), dtype=np.uint64) if want_masks else None
        prm = make_params(sigma, max_violations, negative_trends, want_masks)
        if cl.size == 0:
            cl = np.zeros(1, dtype=np.int32)
        _check(_evaluate(self.handle, _np_ptr(off), _np_ptr(cl), P, ctypes.byref(prm),
                         _np_ptr(masks), _np_ptr(counts), _np_ptr(fit)), self.handle)
        out = {"counts": counts, "fitness": fit}
        if want_masks:
            out["masks"] = masks
        return out

    # -- device tensors ---------------------------------------------------------
    def evaluate_device(self, offsets, cols, counts, fitness, masks=None, *, sigma: int,
                        max_violations: int = 0, negative_trends: bool = False,
                        stream=None, noalloc: bool = False) -> None:
        """Stream-ordered evaluation of device tensors (int32 offsets/cols,
        int32 counts, float64 fitness, optional uint64/int64 masks [P,2,W]).
        Launches on ``stream`` (default: torch's current stream) and returns
        without waiting.  ``noalloc`` calls ``ebic_evaluate_device_noalloc``
        (no device allocation; P <= NOALLOC_MAX_CANDIDATES)."""
        self.device_call(offsets, cols, counts, fitness, masks, sigma=sigma,
                         max_violations=max_violations, negative_trends=negative_trends,
                         stream=stream, noalloc=noalloc)()

    def device_call(self, offsets, cols, counts, fitness, masks=None, *, sigma: int,
                    max_violations: int = 0, negative_trends: bool = False, stream=None,
                    noalloc: bool = False):
        """Validate the tensors once and return a no-argument callable that
        launches ``ebic_evaluate_device`` (``ebic_evaluate_device_noalloc``
        with ``noalloc``) on them (the tensors must stay alive and keep their
        storage while the callable is used)."""
        import torch
        P = offsets.numel() - 1
        for t, name in ((offsets, "offsets"), (cols, "cols"), (counts, "counts"),
                        (fitness, "fitness")):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous device tensor")
        if offsets.dtype != torch.int32 or cols.dtype != torch.int32 or counts.dtype != torch.int32:
            raise TypeError("offsets, cols and counts must be int32")
        if fitness.dtype != torch.float64:
            raise TypeError("fitness must be float64")
        if counts.numel() < P or fitness.numel() < P:
            raise ValueError("counts/fitness hold fewer than P entries")
        want = masks is not None
        if want and (masks.element_size() != 8 or masks.numel() < 2 * P * self.W
                     or not masks.is_contiguous()):
            raise ValueError("masks must be a contiguous 64-bit tensor of 2*P*W words")
        if stream is None:
            stream = torch.cuda.current_stream(offsets.device)
        prm = make_params(sigma, max_violations, negative_trends, want)
        h = self.handle
        args = (h, _vp(offsets.data_ptr()), _vp(cols.data_ptr()), P, cols.numel(),
                ctypes.byref(prm), _vp(masks.data_ptr()) if want else None,
                _vp(counts.data_ptr()), _vp(fitness.data_ptr()), _vp(stream.cuda_stream))
        fn = _evaluate_device_noalloc if noalloc else _evaluate_device

        def call():
            st = fn(*args)
            if st != EBIC_OK:
                _check(st, h)
        call.params = prm          # keep the struct alive with the callable
        return call


# ------------------------------------------------------------------ evolution --

_evolve = _sig("ebic_evolve", _i32, [_vp, _u64, _i32, _P(EvolveParamsC), _P(_vp)])
_evolve_with = _sig("ebic_evolve_with", _i32,
                    [EVAL_FN, _vp, _i64, _i32, _u64, _i32, _P(EvolveParamsC), _P(_vp)])
_evolve_defaults = _sig("ebic_evolve_defaults", None, [_P(EvolveParamsC), _i32, _i32, _i32, _i32])
_result_size = _sig("ebic_result_size", _i32, [_vp])
_result_get = _sig("ebic_result_get", _i32,
                   [_vp, _i32, _P(_P(_i32)), _P(_i32), _P(_i32), _P(_dbl), _P(_P(_u64))])
_result_stats = _sig("ebic_result_stats", _i32, [_vp, _P(RunStats)])
_result_free = _sig("ebic_result_free", None, [_vp])

EXPORTED += ["ebic_evolve", "ebic_evolve_with", "ebic_evolve_defaults", "ebic_result_size",
             "ebic_result_get", "ebic_result_stats", "ebic_result_free"]


@dataclass
class Trend:
    """Trend and fitness parameters (sigma of Eq. (1), tolerance k, negative trends)."""
    sigma: int
    max_violations: int = 0
    negative_trends: bool = False


@dataclass
class EvolveConfig:
    population: int
    len_min: int
    len_max: int
    eval: Trend
    expand: Trend
    tournament: int = 3
    op_weight: Tuple[int, int, int, int, int] = (1, 1, 1, 1, 1)
    elite_num: int = 1
    elite_den: int = 4
    penalty_base: float = 1.2
    overlap: float = 0.5
    toplist_size: int = 100
    tabu_limit: int = -1


@dataclass
class Generation:
    gen: int
    offsets: np.ndarray
    cols: np.ndarray
    counts: np.ndarray
    fitness: np.ndarray

    @property
    def population(self) -> List[tuple]:
        o, c = self.offsets, self.cols
        return [tuple(int(x) for x in c[o[i]:o[i + 1]]) for i in range(len(o) - 1)]


@dataclass
class EvolveResult:
    biclusters: List[dict]
    stats: dict


def _trend_c(t: Trend, want_masks: bool) -> Params:
    return make_params(t.sigma, t.max_violations, t.negative_trends, want_masks)


def _params_c(cfg: EvolveConfig, on_gen) -> EvolveParamsC:
    p = EvolveParamsC()
    p.struct_size = ctypes.sizeof(EvolveParamsC)
    p.population, p.len_min, p.len_max = cfg.population, cfg.len_min, cfg.len_max
    p.tournament = cfg.tournament
    for i, w in enumerate(cfg.op_weight):
        p.op_weight[i] = int(w)
    p.elite_num, p.elite_den = cfg.elite_num, cfg.elite_den
    p.penalty_base, p.overlap = float(cfg.penalty_base), float(cfg.overlap)
    p.toplist_size, p.tabu_limit = cfg.toplist_size, cfg.tabu_limit
    p.eval = _trend_c(cfg.eval, False)
    p.expand = _trend_c(cfg.expand, True)
    p.on_generation = on_gen
    p.user = None
    return p


def _best_callback(fn: Callable[[int, float], None]):
    """The C callback reporting (generation, best fitness of the scored
    population) without copying the population."""
    def cb(user, gen, off, cols, P, counts, fit):
        f = np.ctypeslib.as_array(fit, shape=(max(P, 1),))[:P]
        fn(int(gen), float(f.max(initial=0.0)))
    return GENERATION_FN(cb)


def _run_callback(on_generation, on_best, only=None):
    if on_generation is not None and on_best is not None:
        raise ValueError("give on_generation or on_best, not both")
    return _best_callback(on_best) if on_best is not None else _gen_callback(on_generation, only)


def _gen_callback(fn: Optional[Callable[[Generation], None]], only=None):
    """The C callback for ``fn``; with ``only`` (a set of generation
    numbers), other generations return at once without copying anything."""
    if fn is None:
        return GENERATION_FN()

    def cb(user, gen, off, cols, P, counts, fit):
        if only is not None and gen not in only:
            return
        o = np.ctypeslib.as_array(off, shape=(P + 1,)).copy()
        n = int(o[-1])
        c = np.ctypeslib.as_array(cols, shape=(max(n, 1),))[:n].copy()
        fn(Generation(int(gen), o, c, np.ctypeslib.as_array(counts, shape=(P,)).copy(),
                      np.ctypeslib.as_array(fit, shape=(P,)).copy()))
    return GENERATION_FN(cb)


def _collect(res_ptr) -> EvolveResult:
    try:
        out = []
        for i in range(_result_size(res_ptr)):
            cols, L, cnt, fit, mask = _P(_i32)(), _i32(), _i32(), _dbl(), _P(_u64)()
            _check(_result_get(res_ptr, i, ctypes.byref(cols), ctypes.byref(L), ctypes.byref(cnt),
                               ctypes.byref(fit), ctypes.byref(mask)))
            out.append({"cols": tuple(int(x) for x in cols[:L.value]), "count": cnt.value,
                        "fitness": fit.value, "mask_ptr": mask})
        st = RunStats()
        st.struct_size = ctypes.sizeof(RunStats)
        _check(_result_stats(res_ptr, ctypes.byref(st)))
        stats = {f: getattr(st, f) for f, _ in RunStats._fields_ if f != "struct_size"}
        return EvolveResult(out, stats)
    except Exception:
        _result_free(res_ptr)
        raise


def _finish(res_ptr, n_rows: int) -> EvolveResult:
    r = _collect(res_ptr)
    W = mask_words(n_rows)
    for b in r.biclusters:
        b["mask_words"] = np.ctypeslib.as_array(b.pop("mask_ptr"), shape=(W,)).copy()
    _result_free(res_ptr)
    return r


def evolve(ctx: Context, seed: int, generations: int, cfg: EvolveConfig,
           on_generation: Optional[Callable[[Generation], None]] = None,
           report_generations=None,
           on_best: Optional[Callable[[int, float], None]] = None) -> EvolveResult:
    """EBIC run (Steps 1-7) on the GPU context ``ctx``.  ``on_generation``
    receives every generation, or only those in ``report_generations``;
    ``on_best(generation, best fitness)`` is a lighter alternative."""
    cb = _run_callback(on_generation, on_best,
                       None if report_generations is None else set(report_generations))
    p = _params_c(cfg, cb)
    res = _vp()
    st = _evolve(ctx.handle, int(seed) & ((1 << 64) - 1), int(generations), ctypes.byref(p),
                 ctypes.byref(res))
    if st != EBIC_OK:
        msg = _last_error(ctx.handle).decode(errors="replace") or _last_error(None).decode(errors="replace")
        raise EbicError(st, msg)
    return _finish(res, ctx.n_rows)


def evolve_with(evaluate: Callable, n_rows: int, n_cols: int, seed: int, generations: int,
                cfg: EvolveConfig,
                on_generation: Optional[Callable[[Generation], None]] = None) -> EvolveResult:
    """The same run with a Python evaluator in place of the GPU.

    ``evaluate(offsets, cols, sigma, max_violations, negative_trends,
    want_masks)`` returns (counts, fitness, masks-or-None) as NumPy arrays;
    masks are uint64 [P, 2, W]."""
    W = mask_words(n_rows)
    errors = []

    def cb(user, off, cols, P, prm, masks, counts, fit):
        try:
            o = np.ctypeslib.as_array(off, shape=(P + 1,)).copy()
            n = int(o[-1])
            c = np.ctypeslib.as_array(cols, shape=(max(n, 1),))[:n].copy()
            pr = prm.contents
            cnt, f, m = evaluate(o, c, pr.sigma, pr.max_violations, bool(pr.negative_trends),
                                 bool(pr.want_masks))
            np.ctypeslib.as_array(counts, shape=(P,))[:] = cnt
            np.ctypeslib.as_array(fit, shape=(P,))[:] = f
            if pr.want_masks:
                np.ctypeslib.as_array(masks, shape=(P * 2 * W,))[:] = np.asarray(m, dtype=np.uint64).ravel()
            return EBIC_OK
        except Exception as ex:  # reported after the run
            errors.append(ex)
            return EBIC_E_DEVICE

    efn = EVAL_FN(cb)
    gcb = _gen_callback(on_generation)
    p = _params_c(cfg, gcb)
    res = _vp()
    st = _evolve_with(efn, None, int(n_rows), int(n_cols), int(seed) & ((1 << 64) - 1),
                      int(generations), ctypes.byref(p), ctypes.byref(res))
    if errors:
        raise errors[0]
    _check(st)
    return _finish(res, n_rows)


SCORE_FN = ctypes.CFUNCTYPE(_i32, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32,
                            ctypes.POINTER(ctypes.c_double))
_evolve_screened_with = _sig("ebic_evolve_screened_with", _i32,
                             [EVAL_FN, _vp, SCORE_FN, _vp, _i64, _i32, _u64, _i32, _i32, _i32, _i32,
                              _P(EvolveParamsC), _P(_vp)])
EXPORTED += ["ebic_evolve_screened_with"]


def evolve_screened_with(evaluate: Callable, score: Callable, n_rows: int, n_cols: int, seed: int,
                         generations: int, cfg: EvolveConfig, oversample: int = 8,
                         warmup_generations: int = 3, host_threads: int = 0,
                         on_generation: Optional[Callable[[Generation], None]] = None) -> EvolveResult:
    """Offspring-screened run with caller-supplied evaluator and ranking
    (``ebic_evolve_screened_with``).  ``evaluate`` as in ``evolve_with``;
    ``score(offsets, cols)`` returns one float64 per pooled child (higher is
    better)."""
    W = mask_words(n_rows)
    errors = []

    def ecb(user, off, cols, P, prm, masks, counts, fit):
        try:
            o = np.ctypeslib.as_array(off, shape=(P + 1,)).copy()
            n = int(o[-1])
            c = np.ctypeslib.as_array(cols, shape=(max(n, 1),))[:n].copy()
            pr = prm.contents
            cnt, f, m = evaluate(o, c, pr.sigma, pr.max_violations, bool(pr.negative_trends),
                                 bool(pr.want_masks))
            np.ctypeslib.as_array(counts, shape=(P,))[:] = cnt
            np.ctypeslib.as_array(fit, shape=(P,))[:] = f
            if pr.want_masks:
                np.ctypeslib.as_array(masks, shape=(P * 2 * W,))[:] = np.asarray(m, dtype=np.uint64).ravel()
            return EBIC_OK
        except Exception as ex:  # reported after the run
            errors.append(ex)
            return EBIC_E_DEVICE

    def scb(user, off, cols, B, out):
        try:
            o = np.ctypeslib.as_array(off, shape=(B + 1,)).copy()
            n = int(o[-1])
            c = np.ctypeslib.as_array(cols, shape=(max(n, 1),))[:n].copy()
            np.ctypeslib.as_array(out, shape=(B,))[:] = np.asarray(score(o, c), dtype=np.float64)
            return EBIC_OK
        except Exception as ex:
            errors.append(ex)
            return EBIC_E_DEVICE

    efn, sfn = EVAL_FN(ecb), SCORE_FN(scb)
    gcb = _gen_callback(on_generation)
    p = _params_c(cfg, gcb)
    res = _vp()
    st = _evolve_screened_with(efn, None, sfn, None, int(n_rows), int(n_cols),
                               int(seed) & ((1 << 64) - 1), int(generations), int(oversample),
                               int(warmup_generations), int(host_threads), ctypes.byref(p),
                               ctypes.byref(res))
    if errors:
        raise errors[0]
    _check(st)
    return _finish(res, n_rows)


_evolve_oversampled = _sig("ebic_evolve_oversampled", _i32,
                           [_vp, _u64, _i32, _i32, _i32, _P(EvolveParamsC), _P(_vp)])
EXPORTED += ["ebic_evolve_oversampled"]


def evolve_oversampled(ctx: Context, seed: int, generations: int, cfg: EvolveConfig,
                       oversample: int = 8, warmup_generations: int = 3,
                       on_generation: Optional[Callable[[Generation], None]] = None,
                       on_best: Optional[Callable[[int, float], None]] = None) -> EvolveResult:
    """Offspring screening by exact GPU fitness (``ebic_evolve_oversampled``)."""
    cb = _run_callback(on_generation, on_best)
    p = _params_c(cfg, cb)
    res = _vp()
    st = _evolve_oversampled(ctx.handle, int(seed) & ((1 << 64) - 1), int(generations),
                             int(oversample), int(warmup_generations), ctypes.byref(p),
                             ctypes.byref(res))
    if st != EBIC_OK:
        msg = _last_error(ctx.handle).decode(errors="replace") or _last_error(None).decode(errors="replace")
        raise EbicError(st, msg)
    return _finish(res, ctx.n_rows)


class RunProgressC(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("next_generation", _i32), ("generations_run", _i32),
                ("stopped_by_tabu", _i32), ("toplist", _i32), ("best_fitness", _dbl),
                ("tabu_size", _i64), ("candidates_evaluated", _i64), ("eval_ms", _dbl),
                ("wall_ms", _dbl)]


_run_create = _sig("ebic_run_create", _i32, [_vp, _u64, _i32, _P(EvolveParamsC), _P(_vp)])
_run_create_with = _sig("ebic_run_create_with", _i32,
                        [EVAL_FN, _vp, _i64, _i32, _u64, _i32, _P(EvolveParamsC), _P(_vp)])
_run_advance = _sig("ebic_run_advance", _i32, [_vp, _i32, _P(_i32)])
_run_get_progress = _sig("ebic_run_get_progress", _i32, [_vp, _P(RunProgressC)])
_run_save = _sig("ebic_run_save", _i32, [_vp, _vp, _i64, _P(_i64)])
_run_load = _sig("ebic_run_load", _i32, [_vp, _P(EvolveParamsC), _vp, _i64, _P(_vp)])
_run_load_with = _sig("ebic_run_load_with", _i32,
                      [EVAL_FN, _vp, _i64, _i32, _P(EvolveParamsC), _vp, _i64, _P(_vp)])
_run_result = _sig("ebic_run_result", _i32, [_vp, _P(_vp)])
_run_destroy = _sig("ebic_run_destroy", None, [_vp])
EXPORTED += ["ebic_run_create", "ebic_run_create_with", "ebic_run_advance",
             "ebic_run_get_progress", "ebic_run_save", "ebic_run_load", "ebic_run_load_with",
             "ebic_run_result", "ebic_run_destroy"]


def _eval_callback(evaluate: Callable, n_rows: int, errors: list):
    W = mask_words(n_rows)

    def cb(user, off, cols, P, prm, masks, counts, fit):
        try:
            o = np.ctypeslib.as_array(off, shape=(P + 1,)).copy()
            n = int(o[-1])
            c = np.ctypeslib.as_array(cols, shape=(max(n, 1),))[:n].copy()
            pr = prm.contents
            cnt, f, m = evaluate(o, c, pr.sigma, pr.max_violations, bool(pr.negative_trends),
                                 bool(pr.want_masks))
            np.ctypeslib.as_array(counts, shape=(P,))[:] = cnt
            np.ctypeslib.as_array(fit, shape=(P,))[:] = f
            if pr.want_masks:
                np.ctypeslib.as_array(masks, shape=(P * 2 * W,))[:] = np.asarray(m, dtype=np.uint64).ravel()
            return EBIC_OK
        except Exception as ex:  # reported by the caller
            errors.append(ex)
            return EBIC_E_DEVICE
    return EVAL_FN(cb)


class Run:
    """A stateful EBIC run (``ebic_run_*``): advance, checkpoint, resume.

    ``Run(cfg, seed, generations, ctx=ctx)`` evaluates on a GPU context;
    ``Run(cfg, seed, generations, evaluate=fn, n_rows=N, n_cols=M)`` on a
    Python evaluator (as ``evolve_with``).  ``Run.load(cfg, data, ...)``
    resumes from ``save()`` bytes."""

    def __init__(self, cfg: EvolveConfig, seed: int = 0, generations: int = 0, *, ctx=None,
                 evaluate: Optional[Callable] = None, n_rows: int = 0, n_cols: int = 0,
                 on_generation: Optional[Callable[[Generation], None]] = None, _data=None):
        self._errors = []
        self._gcb = _gen_callback(on_generation)
        self._p = _params_c(cfg, self._gcb)
        self._ctx = ctx
        self.n_rows = ctx.n_rows if ctx is not None else int(n_rows)
        h = _vp()
        if ctx is not None:
            st = (_run_create(ctx.handle, int(seed) & ((1 << 64) - 1), int(generations),
                              ctypes.byref(self._p), ctypes.byref(h)) if _data is None else
                  _run_load(ctx.handle, ctypes.byref(self._p), _data, len(_data), ctypes.byref(h)))
        else:
            self._efn = _eval_callback(evaluate, n_rows, self._errors)
            st = (_run_create_with(self._efn, None, int(n_rows), int(n_cols),
                                   int(seed) & ((1 << 64) - 1), int(generations),
                                   ctypes.byref(self._p), ctypes.byref(h)) if _data is None else
                  _run_load_with(self._efn, None, int(n_rows), int(n_cols), ctypes.byref(self._p),
                                 _data, len(_data), ctypes.byref(h)))
        self._raise(st)
        self._h = h

    @classmethod
    def load(cls, cfg: EvolveConfig, data: bytes, **kw) -> "Run":
        return cls(cfg, _data=bytes(data), **kw)

    def _raise(self, st):
        if self._errors:
            raise self._errors.pop(0)
        if st != EBIC_OK:
            msg = _last_error(None).decode(errors="replace")
            if self._ctx is not None and not msg:
                msg = _last_error(self._ctx.handle).decode(errors="replace")
            raise EbicError(st, msg)

    def advance(self, generations: int) -> bool:
        """Run up to ``generations`` more generations; True when the run is over."""
        fin = _i32()
        self._raise(_run_advance(self._h, int(generations), ctypes.byref(fin)))
        return bool(fin.value)

    def progress(self) -> dict:
        pr = RunProgressC()
        pr.struct_size = ctypes.sizeof(RunProgressC)
        self._raise(_run_get_progress(self._h, ctypes.byref(pr)))
        return {f: getattr(pr, f) for f, _ in RunProgressC._fields_ if f != "struct_size"}

    def save(self) -> bytes:
        n = _i64()
        self._raise(_run_save(self._h, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._raise(_run_save(self._h, buf, n.value, ctypes.byref(n)))
        return buf.raw[:n.value]

    def result(self) -> EvolveResult:
        res = _vp()
        self._raise(_run_result(self._h, ctypes.byref(res)))
        return _finish(res, self.n_rows)

    def close(self):
        if getattr(self, "_h", None):
            _run_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# -------------------------------------------------------------- batched runs --

class BatchTuning(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("workgroups", _i32), ("unroll", _i32),
                ("best_ms", _dbl), ("words_per_lane", _i32), ("whole_candidates", _i32),
                ("use_graph", _i32)]


BATCH_GENERATION_FN = ctypes.CFUNCTYPE(None, _vp, _i32, _i32, ctypes.POINTER(_i32),
                                       ctypes.POINTER(_i32), _i32, ctypes.POINTER(_i32),
                                       ctypes.POINTER(_dbl))
_batch_create = _sig("ebic_batch_create", _i32, [_i32, _vp, _vp, _vp, _i32, _P(_vp)])
_batch_destroy = _sig("ebic_batch_destroy", _i32, [_vp])
_batch_get_tuning = _sig("ebic_batch_get_tuning", _i32, [_vp, _P(BatchTuning)])
_batch_set_tuning = _sig("ebic_batch_set_tuning", _i32, [_vp, _P(BatchTuning)])
_batch_evaluate = _sig("ebic_batch_evaluate", _i32,
                       [_vp, _vp, _vp, _vp, _P(Params), _vp, _vp, _vp, _i32])
_batch_evolve = _sig("ebic_batch_evolve", _i32,
                     [_vp, _vp, _i32, _P(EvolveParamsC), BATCH_GENERATION_FN, _vp, _i32, _vp])
_batch_evolve_device = _sig("ebic_batch_evolve_device", _i32,
                            [_vp, _vp, _i32, _P(EvolveParamsC), BATCH_GENERATION_FN, _vp, _vp])
_batch_last_ms = _sig("ebic_batch_last_ms", _dbl, [_vp])
_batch_index_build_ms = _sig("ebic_batch_index_build_ms", _dbl, [_vp])
_batch_time_replays = _sig("ebic_batch_time_replays", _i32, [_vp, _i32, _P(_dbl)])
EXPORTED += ["ebic_batch_evolve_device", "ebic_batch_last_ms", "ebic_batch_index_build_ms", "ebic_batch_time_replays", "ebic_batch_create", "ebic_batch_destroy", "ebic_batch_get_tuning",
             "ebic_batch_set_tuning", "ebic_batch_evaluate", "ebic_batch_evolve"]


def _ptr_array(arrs, ctype):
    out = (ctypes.c_void_p * len(arrs))()
    for i, a in enumerate(arrs):
        out[i] = None if a is None else a.ctypes.data
    return out


class Batch:
    """Many matrices on one GPU, evaluated or evolved together (``ebic_batch_*``)."""

    def __init__(self, matrices, device: int = 0):
        mats = [np.ascontiguousarray(m, dtype=np.float32) for m in matrices]
        n = np.array([m.shape[0] for m in mats], dtype=np.int64)
        mcols = np.array([m.shape[1] for m in mats], dtype=np.int32)
        ptrs = _ptr_array(mats, ctypes.c_float)
        h = _vp()
        _check(_batch_create(len(mats), ptrs, n.ctypes.data, mcols.ctypes.data, int(device),
                             ctypes.byref(h)))
        self._h = h
        self.n_rows = [int(x) for x in n]
        self.n_cols = [int(x) for x in mcols]

    def close(self):
        if getattr(self, "_h", None):
            _batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def last_ms(self) -> float:
        """Device time (ms) of the last batched launch (the kernel)."""
        return float(_batch_last_ms(self._h))

    def index_build_ms(self) -> float:
        """Device ms spent building the runs' order indexes (sum over runs)."""
        return float(_batch_index_build_ms(self._h))

    def time_replays(self, reps: int) -> float:
        """Mean device ms of ``reps`` back-to-back replays of the last launch."""
        ms = _dbl()
        _check(_batch_time_replays(self._h, int(reps), ctypes.byref(ms)))
        return float(ms.value)

    def tuning(self) -> dict:
        t = BatchTuning()
        t.struct_size = ctypes.sizeof(BatchTuning)
        _check(_batch_get_tuning(self._h, ctypes.byref(t)))
        return {"workgroups": t.workgroups, "unroll": t.unroll, "best_ms": t.best_ms,
                "words_per_lane": t.words_per_lane, "whole_candidates": t.whole_candidates,
                "use_graph": t.use_graph}

    def set_tuning(self, workgroups: int = 0, unroll: int = 4, words_per_lane: int = 1,
                   whole_candidates: int = 0, use_graph: int = 0):
        t = BatchTuning(ctypes.sizeof(BatchTuning), int(workgroups), int(unroll), 0.0,
                        int(words_per_lane), int(whole_candidates), int(use_graph))
        _check(_batch_set_tuning(self._h, ctypes.byref(t)))

    def evaluate(self, pops, *, sigma: int, max_violations: int = 0,
                 negative_trends: bool = False, want_masks: bool = False, tune: bool = False):
        """``pops[r]`` is (offsets, cols) for run r, or None to skip it.
        Returns one dict (counts, fitness[, masks]) per run (None if skipped)."""
        R = len(self.n_rows)
        assert len(pops) == R
        offs, cls, Ps, msks = [], [], [], []
        for r in range(R):
            if pops[r] is None or len(pops[r][0]) <= 1:
                offs.append(None); cls.append(None); Ps.append(0); msks.append(None)
                continue
            o = np.ascontiguousarray(pops[r][0], dtype=np.int32)
            c = np.ascontiguousarray(pops[r][1], dtype=np.int32)
            offs.append(o); cls.append(c); Ps.append(len(o) - 1)
            msks.append(np.zeros((len(o) - 1, 2, mask_words(self.n_rows[r])), dtype=np.uint64)
                        if want_masks else None)
        P_arr = np.array(Ps, dtype=np.int32)
        # one allocation per output; run r's results are a slice of it
        base = np.zeros(R + 1, dtype=np.int64)
        np.cumsum(P_arr, out=base[1:])
        counts = np.empty(int(base[-1]), dtype=np.int32)
        fitness = np.empty(int(base[-1]), dtype=np.float64)
        cnt_p = (ctypes.c_void_p * R).from_buffer_copy(
            (counts.ctypes.data + 4 * base[:-1]).astype(np.uint64).tobytes())
        fit_p = (ctypes.c_void_p * R).from_buffer_copy(
            (fitness.ctypes.data + 8 * base[:-1]).astype(np.uint64).tobytes())
        prm = make_params(sigma, max_violations, negative_trends, want_masks)
        _check(_batch_evaluate(self._h, _ptr_array(offs, None), _ptr_array(cls, None),
                               P_arr.ctypes.data, ctypes.byref(prm),
                               _ptr_array(msks, None) if want_masks else None,
                               cnt_p, fit_p, int(bool(tune))))
        out = []
        for r in range(R):
            if Ps[r] == 0:
                out.append(None)
                continue
            d = {"counts": counts[base[r]:base[r + 1]], "fitness": fitness[base[r]:base[r + 1]]}
            if want_masks:
                d["masks"] = msks[r]
            out.append(d)
        return out

    def evolve(self, seeds, generations: int, cfg: EvolveConfig, on_generation=None,
               host_threads: int = 0, device_steps: bool = False):
        """EBIC runs, one per matrix, seeds[r] for run r; returns one
        EvolveResult per run.  ``on_generation(run, Generation)``.
        ``device_steps`` runs Steps 1-3 and 5 on the GPU
        (``ebic_batch_evolve_device``); the runs are the same."""
        R = len(self.n_rows)
        sd = np.array([int(s) & ((1 << 64) - 1) for s in seeds], dtype=np.uint64)
        assert len(sd) == R
        if on_generation is None:
            gcb = BATCH_GENERATION_FN()
        else:
            def cb(user, run, gen, off, cols, P, counts, fit):
                o = np.ctypeslib.as_array(off, shape=(P + 1,)).copy()
                n = int(o[-1])
                c = np.ctypeslib.as_array(cols, shape=(max(n, 1),))[:n].copy()
                on_generation(int(run), Generation(int(gen), o, c,
                                                   np.ctypeslib.as_array(counts, shape=(P,)).copy(),
                                                   np.ctypeslib.as_array(fit, shape=(P,)).copy()))
            gcb = BATCH_GENERATION_FN(cb)
        p = _params_c(cfg, GENERATION_FN())
        res = (ctypes.c_void_p * R)()
        if device_steps:
            _check(_batch_evolve_device(self._h, sd.ctypes.data, int(generations),
                                        ctypes.byref(p), gcb, None, res))
        else:
            _check(_batch_evolve(self._h, sd.ctypes.data, int(generations), ctypes.byref(p), gcb,
                                 None, int(host_threads), res))
        return [_finish(_vp(res[r]), self.n_rows[r]) for r in range(R)]


# ------------------------------------------------------------- surrogate MLP --

class MlpConfig(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("embed_dim", _i32), ("hidden", _i32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


_mlp_defaults = _sig("ebic_mlp_defaults", None, [_P(MlpConfig)])
_mlp_create = _sig("ebic_mlp_create", _i32, [_i32, _P(MlpConfig), _u64, _i32, _P(_vp)])
_mlp_destroy = _sig("ebic_mlp_destroy", _i32, [_vp])
_mlp_param_count = _sig("ebic_mlp_param_count", _i64, [_vp])
_mlp_get_params = _sig("ebic_mlp_get_params", _i32, [_vp, _vp])
_mlp_set_params = _sig("ebic_mlp_set_params", _i32, [_vp, _vp])
_mlp_predict = _sig("ebic_mlp_predict", _i32, [_vp, _vp, _vp, _i32, _vp])
_mlp_gradients = _sig("ebic_mlp_gradients", _i32, [_vp, _vp, _vp, _i32, _vp, _vp, _P(ctypes.c_float)])
_mlp_train_step = _sig("ebic_mlp_train_step", _i32, [_vp, _vp, _vp, _i32, _vp, _P(ctypes.c_float)])
_mlp_train = _sig("ebic_mlp_train", _i32, [_vp, _vp, _vp, _i32, _vp, _i32, _P(ctypes.c_float)])
EXPORTED += ["ebic_mlp_train", "ebic_mlp_defaults", "ebic_mlp_create", "ebic_mlp_destroy", "ebic_mlp_param_count",
             "ebic_mlp_get_params", "ebic_mlp_set_params", "ebic_mlp_predict",
             "ebic_mlp_gradients", "ebic_mlp_train_step"]


class Mlp:
    """Surrogate fitness model on one GPU (``ebic_mlp_*``)."""

    def __init__(self, n_cols: int, seed: int = 0, embed_dim: int = 32, hidden: int = 256,
                 lr: float = 1e-3, device: int = 0):
        cfg = MlpConfig()
        _mlp_defaults(ctypes.byref(cfg))
        cfg.embed_dim, cfg.hidden, cfg.lr = int(embed_dim), int(hidden), float(lr)
        h = _vp()
        _check(_mlp_create(int(n_cols), ctypes.byref(cfg), int(seed) & ((1 << 64) - 1),
                           int(device), ctypes.byref(h)))
        self._h = h
        self.n_cols, self.embed_dim, self.hidden = int(n_cols), int(embed_dim), int(hidden)
        self.n_params = int(_mlp_param_count(h))

    def close(self):
        if getattr(self, "_h", None):
            _mlp_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, p):
        arr = np.ascontiguousarray(p, dtype=np.float32)
        assert arr.size == self.n_params
        _check(_mlp_set_params(self._h, arr.ctypes.data))

    @staticmethod
    def _cbf(offsets, cols):
        o = np.ascontiguousarray(offsets, dtype=np.int32)
        c = np.ascontiguousarray(cols, dtype=np.int32)
        return o, c, len(o) - 1

    def predict(self, offsets, cols) -> np.ndarray:
        o, c, B = self._cbf(offsets, cols)
        y = np.zeros(B, dtype=np.float32)
        _check(_mlp_predict(self._h, o.ctypes.data, c.ctypes.data, B, y.ctypes.data))
        return y

    def gradients(self, offsets, cols, target):
        o, c, B = self._cbf(offsets, cols)
        t = np.ascontiguousarray(target, dtype=np.float32)
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_mlp_gradients(self._h, o.ctypes.data, c.ctypes.data, B, t.ctypes.data,
                              g.ctypes.data, ctypes.byref(loss)))
        return float(loss.value), g

    def train_step(self, offsets, cols, target) -> float:
        o, c, B = self._cbf(offsets, cols)
        t = np.ascontiguousarray(target, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_mlp_train_step(self._h, o.ctypes.data, c.ctypes.data, B, t.ctypes.data,
                               ctypes.byref(loss)))
        return float(loss.value)

    def train(self, offsets, cols, target, steps: int) -> float:
        """``steps`` Adam steps on one batch; returns the loss before the last."""
        o, c, B = self._cbf(offsets, cols)
        t = np.ascontiguousarray(target, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_mlp_train(self._h, o.ctypes.data, c.ctypes.data, B, t.ctypes.data, int(steps),
                          ctypes.byref(loss)))
        return float(loss.value)


# ------------------------------------------------------ surrogate-screened run --

SURROGATE_FN = ctypes.CFUNCTYPE(None, _vp, _i32, _i32, _dbl, _dbl, _i32)


class SurrogateParamsC(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("oversample", _i32), ("warmup_generations", _i32),
                ("train_steps", _i32), ("replay_generations", _i32), ("min_rank_corr", _dbl),
                ("mlp_seed", _u64), ("mlp", MlpConfig), ("on_surrogate", SURROGATE_FN),
                ("user", _vp), ("check_sample", _i32), ("exact_rerank", _i32)]


_surrogate_defaults = _sig("ebic_surrogate_defaults", None, [_P(SurrogateParamsC)])
_evolve_surrogate = _sig("ebic_evolve_surrogate", _i32,
                         [_vp, _u64, _i32, _P(EvolveParamsC), _P(SurrogateParamsC), _P(_vp)])
EXPORTED += ["ebic_surrogate_defaults", "ebic_evolve_surrogate"]


def evolve_surrogate(ctx: Context, seed: int, generations: int, cfg: EvolveConfig,
                     on_generation: Optional[Callable[[Generation], None]] = None,
                     on_surrogate: Optional[Callable[[dict], None]] = None,
                     on_best: Optional[Callable[[int, float], None]] = None,
                     **surrogate) -> EvolveResult:
    """Surrogate-screened EBIC run (``ebic_evolve_surrogate``).  Keyword
    arguments override ebic_surrogate_defaults: oversample, warmup_generations,
    train_steps, replay_generations, min_rank_corr, mlp_seed, check_sample,
    exact_rerank, lr, hidden, embed_dim."""
    sp = SurrogateParamsC()
    _surrogate_defaults(ctypes.byref(sp))
    for k in ("oversample", "warmup_generations", "train_steps", "replay_generations",
              "min_rank_corr", "mlp_seed", "check_sample", "exact_rerank"):
        if k in surrogate:
            setattr(sp, k, surrogate.pop(k))
    for k in ("lr", "hidden", "embed_dim"):
        if k in surrogate:
            setattr(sp.mlp, k, surrogate.pop(k))
    if surrogate:
        raise TypeError(f"unknown surrogate options {sorted(surrogate)}")
    if on_surrogate is None:
        scb = SURROGATE_FN()
    else:
        def _s(user, gen, screened, corr, loss, pool):
            on_surrogate({"gen": int(gen), "screened": bool(screened), "rank_corr": float(corr),
                          "loss": float(loss), "pool": int(pool)})
        scb = SURROGATE_FN(_s)
    sp.on_surrogate = scb
    gcb = _run_callback(on_generation, on_best)
    p = _params_c(cfg, gcb)
    res = _vp()
    st = _evolve_surrogate(ctx.handle, int(seed) & ((1 << 64) - 1), int(generations),
                           ctypes.byref(p), ctypes.byref(sp), ctypes.byref(res))
    if st != EBIC_OK:
        msg = _last_error(ctx.handle).decode(errors="replace") or _last_error(None).decode(errors="replace")
        raise EbicError(st, msg)
    return _finish(res, ctx.n_rows)


# ------------------------------------------------- Step 6 rows and accuracy --

class BiclusterSetC(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("count", _i32), ("planes", _i32), ("row_masks", _vp),
                ("col_offsets", _vp), ("cols", _vp)]


_mask_rows = _sig("ebic_mask_rows", _i32, [_vp, _i32, _i32, _i64, _vp, _vp, _i64, _vp])
_match_scores = _sig("ebic_match_scores", _i32,
                     [_P(BiclusterSetC), _P(BiclusterSetC), _i64, _vp, _vp, _vp])
EXPORTED += ["ebic_mask_rows", "ebic_match_scores"]


def _dev_check(t, name, dtype, stream):
    import torch as _t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


def _mask_shape(masks, n_rows: int):
    """[K][W] or [K][planes][W] 64-bit masks -> (K, planes)."""
    W = mask_words(n_rows)
    if masks.element_size() != 8:
        raise TypeError("masks must hold 64-bit words")
    if masks.dim() == 2:
        K, planes, w = masks.shape[0], 1, masks.shape[1]
    elif masks.dim() == 3:
        K, planes, w = masks.shape
    else:
        raise ValueError("masks must be [K][W] or [K][planes][W]")
    if w != W:
        raise ValueError(f"masks hold {w} words per plane, n_rows needs {W}")
    return int(K), int(planes)


def mask_rows(masks, n_rows: int, capacity: Optional[int] = None, stream=None):
    """Row indices of each bicluster (``ebic_mask_rows``) from device masks
    [K][W] or [K][planes][W] (planes united).  Returns device tensors
    (offsets int64 [K+1], rows int32 [capacity]); with capacity None the
    offsets are read back first and rows is sized to hold every list."""
    import torch as _t
    if not masks.is_cuda or not masks.is_contiguous():
        raise ValueError("masks must be a contiguous device tensor")
    K, planes = _mask_shape(masks, n_rows)
    dev = masks.device
    if stream is None:
        stream = _t.cuda.current_stream(dev)
    offsets = _t.empty(K + 1, dtype=_t.int64, device=dev)
    size_first = capacity is None
    cap = 0 if size_first else int(capacity)
    rows = _t.empty(max(cap, 1), dtype=_t.int32, device=dev)
    args = [_vp(masks.data_ptr()), K, planes, int(n_rows), _vp(offsets.data_ptr()),
            _vp(rows.data_ptr()), cap, _vp(stream.cuda_stream)]
    _check(_mask_rows(*args))
    if size_first:
        stream.synchronize()
        cap = int(offsets[-1].item())
        rows = _t.empty(max(cap, 1), dtype=_t.int32, device=dev)
        args[5], args[6] = _vp(rows.data_ptr()), cap
        _check(_mask_rows(*args))
    return offsets, rows[:cap]


def _set_c(s, n_rows, keep):
    import torch as _t
    masks, col_off, cols = s
    K, planes = _mask_shape(masks, n_rows)
    _dev_check(masks, "row masks", masks.dtype, None)
    _dev_check(col_off, "col_offsets", _t.int32, None)
    _dev_check(cols, "cols", _t.int32, None)
    if col_off.numel() != K + 1:
        raise ValueError("col_offsets must hold count + 1 entries")
    keep.extend([masks, col_off, cols])
    return BiclusterSetC(ctypes.sizeof(BiclusterSetC), K, planes, _vp(masks.data_ptr()),
                         _vp(col_off.data_ptr()), _vp(cols.data_ptr()))


def match_scores(found, expected, n_rows: int, stream=None):
    """Recovery and relevance (``ebic_match_scores``).  found / expected:
    (row masks [K][W] or [K][planes][W], col_offsets int32 [K+1], cols int32)
    device tensors.  Returns (J [F][E] float64 device tensor, recovery,
    relevance)."""
    import torch as _t
    keep = []
    fc, ec = _set_c(found, n_rows, keep), _set_c(expected, n_rows, keep)
    dev = found[0].device
    if stream is None:
        stream = _t.cuda.current_stream(dev)
    J = _t.empty((fc.count, ec.count), dtype=_t.float64, device=dev)
    scores = _t.empty(2, dtype=_t.float64, device=dev)
    _check(_match_scores(ctypes.byref(fc), ctypes.byref(ec), int(n_rows),
                         _vp(J.data_ptr()) if J.numel() else None, _vp(scores.data_ptr()),
                         _vp(stream.cuda_stream)))
    s = scores.cpu().numpy()
    return J, float(s[0]), float(s[1])
