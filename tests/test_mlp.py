"""GPU: the surrogate MLP's forward pass, gradients and Adam step against the
CPU oracle (float64 with the same bfloat16 rounding points), training
progress and run-to-run determinism."""
import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[mlp] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1801_03039_amd as e
    return e


def _batch(rng, M, B, lmin=1, lmax=12):
    series = [rng.choice(M, size=int(rng.integers(lmin, min(lmax, M) + 1)), replace=False)
              for _ in range(B)]
    off = np.zeros(B + 1, dtype=np.int32)
    off[1:] = np.cumsum([len(s) for s in series])
    return off, np.concatenate(series).astype(np.int32)


def _blocks(M, D, H):
    sizes = [("E", M * D), ("F", M * D), ("T", M * D), ("Z", (M + 1) * D), ("W1", H * 2 * D),
             ("b1", H), ("W2", H * H),
             ("b2", H), ("w3", H), ("b3", 1)]
    out, i = {}, 0
    for n, s in sizes:
        out[n] = slice(i, i + s)
        i += s
    return out


SHAPES = [(50, 32, 256, 300), (37, 20, 72, 65), (200, 32, 256, 1), (500, 32, 256, 2048)]


@pytest.mark.parametrize("M,D,H,B", SHAPES)
def test_forward_and_gradients_match_oracle(E, M, D, H, B):
    rng = np.random.default_rng(M + D + H + B)
    off, cols = _batch(rng, M, B)
    t = rng.standard_normal(B).astype(np.float32) * 3
    with E.Mlp(M, seed=7, embed_dim=D, hidden=H) as net:
        p = net.params()
        _note(f"forward M={M} D={D} H={H} B={B}")
        y = net.predict(off, cols)
        y_ref, _ = omlp.forward(p, off, cols, M, D, H, bf16=True)
        scale = max(1.0, float(np.max(np.abs(y_ref))))
        assert np.max(np.abs(y - y_ref)) <= 1e-2 * scale
        _note(f"gradients M={M} D={D} H={H} B={B}")
        loss, g = net.gradients(off, cols, t)
        l_ref, g_ref, _ = omlp.loss_and_grad(p, off, cols, t, M, D, H, bf16=True)
        assert abs(loss - l_ref) <= 1e-2 * max(1.0, l_ref)
        # element by element within 1e-2 of the block's largest reference
        # gradient (FP32 accumulation in a different order than the float64
        # oracle, same BF16 rounding points)
        for name, sl in _blocks(M, D, H).items():
            ref = g_ref[sl]
            bound = 1e-2 * max(float(np.max(np.abs(ref))), 1e-30)
            err = float(np.max(np.abs(g[sl] - ref)))
            _note(f"  {name}: max |g - g_ref| = {err:.3e}, bound {bound:.3e}")
            assert err <= bound, (name, err, bound)


def test_adam_step_matches_oracle(E):
    rng = np.random.default_rng(3)
    M, D, H, B = 60, 32, 256, 512
    off, cols = _batch(rng, M, B)
    t = rng.standard_normal(B).astype(np.float32)
    with E.Mlp(M, seed=1, lr=3e-3) as net:
        p0 = net.params().astype(np.float64)
        _, g = net.gradients(off, cols, t)
        net.train_step(off, cols, t)
        p1 = net.params().astype(np.float64)
    want, _, _ = omlp.adam_step(p0, g.astype(np.float64), np.zeros_like(p0), np.zeros_like(p0), 1,
                                lr=3e-3)
    assert np.allclose(p1, want, rtol=1e-5, atol=1e-6)


def test_training_reduces_loss_and_is_deterministic(E):
    rng = np.random.default_rng(4)
    M, B = 80, 1024
    off, cols = _batch(rng, M, B, 3, 10)
    # a learnable target: sum of hidden per-column scores over the series
    score = rng.standard_normal(M)
    t = np.array([score[cols[off[b]:off[b + 1]]].mean() for b in range(B)], dtype=np.float32)
    runs = []
    for rep in range(2):
        with E.Mlp(M, seed=5, lr=3e-3) as net:
            losses = [net.train_step(off, cols, t) for _ in range(60)]
            runs.append((losses, net.params()))
    losses = runs[0][0]
    assert losses[-1] < 0.3 * losses[0], (losses[0], losses[-1])
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])


def test_multi_step_training_equals_single_steps(E):
    rng = np.random.default_rng(8)
    M, B = 70, 700
    off, cols = _batch(rng, M, B, 2, 12)
    t = rng.standard_normal(B).astype(np.float32)
    with E.Mlp(M, seed=3, lr=3e-3) as a, E.Mlp(M, seed=3, lr=3e-3) as b:
        losses = [a.train_step(off, cols, t) for _ in range(5)]
        last = b.train(off, cols, t, 5)
        assert np.array_equal(a.params(), b.params())
        assert last == losses[-1]
