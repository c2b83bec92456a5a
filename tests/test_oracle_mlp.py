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


def test_stored_precision_reference_reduces_to_the_plain_one():
    """With the identity in place of the bf16 rounding, the stored-precision forward and
    backward are the plain FP64 ones, bit for bit; with the rounding, every stored value
    is a bf16 number and the gradient moves by about the rounding's size."""
    rng = np.random.default_rng(5)
    w = rng.normal(0, 0.3, mlp_ref.NPARAM)
    x = rng.normal(0, 1, (40, 32))
    dy = rng.normal(0, 1, (40, 16))
    ident = lambda a: np.asarray(a, dtype=np.float64)   # noqa: E731
    y, c = mlp_ref.forward(w, x)
    ys, cs = mlp_ref.forward_stored(w, x, q=ident)
    assert np.array_equal(y, ys)
    assert np.array_equal(mlp_ref.backward(w, c, dy), mlp_ref.backward_stored(w, cs, dy, q=ident))
    yq, cq = mlp_ref.forward_stored(w, x)
    for h in cq[1:]:
        assert np.array_equal(h, mlp_ref.bf16_round(h))
    gq = mlp_ref.backward_stored(w, cq, dy)
    g = mlp_ref.backward(w, c, dy)
    rel = np.linalg.norm(gq - g) / np.linalg.norm(g)
    assert 1e-4 < rel < 2e-2
