"""Pins for the surrogate model's CPU oracle (no GPU): central finite
differences of the plain float64 network, bfloat16 rounding against torch's
own float32 -> bfloat16 conversion and hand-picked values, and the closed
form of a first Adam step."""
import numpy as np
import pytest

from oracle import mlp


def _batch(rng, M, B, lmin=1, lmax=6):
    series = [rng.choice(M, size=int(rng.integers(lmin, lmax + 1)), replace=False) for _ in range(B)]
    off = np.zeros(B + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(s) for s in series])
    return off, np.concatenate(series)


@pytest.mark.parametrize("M,D,H,B", [(6, 3, 5, 7), (9, 4, 8, 11)])
def test_gradients_match_finite_differences(M, D, H, B):
    rng = np.random.default_rng(M * 100 + H)
    off, cols = _batch(rng, M, B)
    p = rng.standard_normal(mlp.n_params(M, D, H))
    t = rng.standard_normal(B)
    loss, g, _ = mlp.loss_and_grad(p, off, cols, t, M, D, H, bf16=False)
    h = 1e-6
    num = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp = mlp.loss_and_grad(p + e, off, cols, t, M, D, H, bf16=False)[0]
        lm = mlp.loss_and_grad(p - e, off, cols, t, M, D, H, bf16=False)[0]
        num[i] = (lp - lm) / (2 * h)
    assert np.allclose(g, num, rtol=1e-5, atol=1e-7), np.max(np.abs(g - num))


def test_bf16_rounding_values():
    f = np.float32
    cases = [
        (1.0, 1.0),
        (1.0 + 2 ** -8, 1.0),                 # halfway: ties to even (down)
        (1.0 + 3 * 2 ** -8, 1.0 + 2 ** -6),   # halfway: ties to even (up)
        (1.0 + 2 ** -8 + 2 ** -20, 1.0 + 2 ** -7),
        (-2.5, -2.5),
        (np.finfo(f).max, np.inf),            # rounds past the largest bfloat16
        (0.0, 0.0),
    ]
    for x, want in cases:
        assert mlp.bf16_round(np.array([x], dtype=f))[0] == f(want), x
    assert np.isnan(mlp.bf16_round(np.array([np.nan], dtype=f))[0])


def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    scale = (10.0 ** rng.integers(-30, 30, 100000)).astype(np.float32)
    x = np.concatenate([rng.standard_normal(100000).astype(np.float32) * scale,
                        rng.integers(0, 2 ** 32, 100000, dtype=np.uint64).astype(np.uint32).view(np.float32)])
    x = x[np.isfinite(x)]
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = mlp.bf16_round(x)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(1)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m1, m2 = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=0.01, eps=1e-8)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(new, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
