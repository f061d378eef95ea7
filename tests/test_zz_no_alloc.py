"""GPU: ebic_evaluate_device_noalloc (accumulators in the library's fixed
device array, nothing allocated by the call) gives the same counts, fitness
bits and row masks as ebic_evaluate_device on the same inputs, on two calls
in a row with the second smaller, on every evaluator that uses the
accumulators (direct kernel with row slices, flattened index tiles)."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[noalloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_03039_amd as e
    return e


def _both(ctx, off, cols, W, kw, noalloc_first=False):
    """Outputs of the regular and the no-allocation entry point (in that
    order, or the no-allocation call first)."""
    import torch
    dev = torch.device("cuda:0")
    d_off = torch.from_numpy(off).to(dev)
    d_cols = torch.from_numpy(cols).to(dev)
    P = len(off) - 1
    outs = {}
    for noalloc in ((True, False) if noalloc_first else (False, True)):
        cnt = torch.full((P,), -7, dtype=torch.int32, device=dev)
        fit = torch.full((P,), 3.5, dtype=torch.float64, device=dev)
        masks = torch.full((P, 2, W), 5, dtype=torch.int64, device=dev)
        ctx.evaluate_device(d_off, d_cols, cnt, fit, masks, noalloc=noalloc, **kw)
        torch.cuda.synchronize(dev)
        outs[noalloc] = (cnt.cpu().numpy(), fit.cpu().numpy().view(np.int64), masks.cpu().numpy())
        if noalloc_first and noalloc:
            # under AUTO the no-allocation call does not build the index
            assert not ctx.info()["index_built"]
    return outs[False], outs[True]


def _population(seed, n_cols, P, len_min=3, len_max=12):
    rng = np.random.default_rng(seed)
    pop = synth.random_population(rng, n_cols, P, len_min, len_max)
    return synth.pack_cbf(pop)


@pytest.mark.parametrize("n_rows,n_cols,path,k,neg", [
    (5000, 40, "direct", 1, True),      # 79 words: 8 row slices share each accumulator
    (70000, 24, "index", 1, True),      # 1094 words: flattened index tiles
    (70000, 24, "index", 0, False),
    (3000, 30, "auto", 2, True),        # first call: index not built, the direct kernel runs
])
def test_noalloc_equals_regular_entry_point(E, n_rows, n_cols, path, k, neg):
    import torch
    rng = np.random.default_rng(n_rows + n_cols)
    a = rng.standard_normal((n_rows, n_cols)).astype(np.float32)
    kw = dict(sigma=20, max_violations=k, negative_trends=neg)
    with E.Context(torch.from_numpy(a).to("cuda:0")) as ctx:
        if path != "auto":
            ctx.set_path(path)
        for call, P in enumerate((3000, 700)):       # second call smaller
            off, cols = _population(100 * call + n_rows, n_cols, P)
            _note(f"{n_rows}x{n_cols} path={path} k={k} neg={neg} call={call} P={P}")
            (c0, f0, m0), (c1, f1, m1) = _both(ctx, off, cols, ctx.W, kw,
                                               noalloc_first=path == "auto" and call == 0)
            assert np.array_equal(c0, c1)
            assert np.array_equal(f0, f1)
            assert np.array_equal(m0, m1)
            assert (c0 >= 0).all()


def test_noalloc_limits(E):
    import torch
    from paper_1801_03039_amd import binding as b
    a = np.random.default_rng(3).standard_normal((100, 10)).astype(np.float32)
    dev = torch.device("cuda:0")
    kw = dict(sigma=5, max_violations=0, negative_trends=True)
    with E.Context(torch.from_numpy(a).to(dev)) as ctx:
        # the largest accepted population, then one more candidate
        P = b.NOALLOC_MAX_CANDIDATES
        off, cols = _population(7, 10, P, 2, 4)
        _note(f"limit P={P}")
        (c0, f0, _), (c1, f1, _) = _both(ctx, off, cols, ctx.W, kw)
        assert np.array_equal(c0, c1) and np.array_equal(f0, f1)
        off2 = np.concatenate([off, [off[-1] + 2]]).astype(np.int32)
        cols2 = np.concatenate([cols, [0, 1]]).astype(np.int32)
        d_off = torch.from_numpy(off2).to(dev)
        d_cols = torch.from_numpy(cols2).to(dev)
        cnt = torch.empty(P + 1, dtype=torch.int32, device=dev)
        fit = torch.empty(P + 1, dtype=torch.float64, device=dev)
        with pytest.raises(b.EbicError, match="E_RANGE"):
            ctx.evaluate_device(d_off, d_cols, cnt, fit, noalloc=True, **kw)
        # P = 0 is accepted and touches nothing
        prm = E.make_params(5)
        st = b._evaluate_device_noalloc(ctx.handle, None, None, 0, 0, ctypes.byref(prm), None, None,
                                       None, None)
        assert st == b.EBIC_OK
