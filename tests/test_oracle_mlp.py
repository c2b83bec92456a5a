"""CPU pins of the FP64 MLP reference: backward against central finite differences."""
import numpy as np

from oracle import mlp_ref


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    w = rng.normal(0, 0.3, mlp_ref.NPARAM)
    x = rng.normal(0, 1, (5, 32))
    dy = rng.normal(0, 1, (5, 16))
    y, cache = mlp_ref.forward(w, x)
    g = mlp_ref.backward(w, cache, dy)
    h = 1e-6
    for q in rng.choice(mlp_ref.NPARAM, 60, replace=False):
        e = np.zeros_like(w)
        e[q] = h
        fp = np.sum(dy * mlp_ref.forward(w + e, x)[0])
        fm = np.sum(dy * mlp_ref.forward(w - e, x)[0])
        assert abs((fp - fm) / (2 * h) - g[q]) <= 1e-7 * max(1.0, abs(g[q]))


def test_bf16_rounding_is_nearest_even():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to the even mantissa (1.0)
    assert mlp_ref.bf16_round(np.float32(1 + 2 ** -8)) == 1.0
    assert mlp_ref.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6
    a = np.random.default_rng(1).normal(0, 1, 1000)
    r = mlp_ref.bf16_round(a)
    assert np.all(np.abs(r - a) <= 2 ** -8 * np.abs(a) * 1.0001)
