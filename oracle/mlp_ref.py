"""FP64 NumPy reference of the reaction-surrogate MLP (test infrastructure only).

32 inputs -> 64 tanh -> 64 tanh -> 16 linear outputs; parameters packed as
W1[64][32] b1[64] W2[64][64] b2[64] W3[16][64] b3[16] (the library's layout).
"""
import numpy as np

SHAPES = [("W1", (64, 32)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (16, 64)), ("b3", (16,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(w):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def forward(w, x):
    """x [n][32] -> (y [n][16], cache)."""
    p = unpack(w)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.tanh(x @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, h1, h2)


def backward(w, cache, dy):
    """Gradient of sum(dy * y) with respect to the packed parameters."""
    p = unpack(w)
    x, h1, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    g = {"W3": dy.T @ h2, "b3": dy.sum(0)}
    d2 = (dy @ p["W3"]) * (1 - h2 ** 2)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1 - h1 ** 2)
    g["W1"], g["b1"] = d1.T @ x, d1.sum(0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])


def bf16_round(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(a):
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def forward_stored(w, x, q=bf16_round):
    """The forward with the values a bf16 implementation stores rounded by q: each hidden
    activation is rounded after its tanh before it feeds the next layer (the weights and
    inputs are the caller's, already rounded as the implementation holds them); all
    arithmetic in FP64.  With q the identity this is `forward`."""
    p = unpack(w)
    x = np.asarray(x, dtype=np.float64)
    h1 = q(np.tanh(x @ p["W1"].T + p["b1"]))
    h2 = q(np.tanh(h1 @ p["W2"].T + p["b2"]))
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, h1, h2)


def backward_stored(w, cache, dy, q=bf16_round):
    """`backward` with the values a bf16 implementation stores rounded by q: the incoming
    dy and each layer's delta are rounded before they enter a product or a bias sum (the
    activations come rounded in the cache of `forward_stored`).  With q the identity this
    is `backward`."""
    p = unpack(w)
    x, h1, h2 = cache
    d3 = q(np.asarray(dy, dtype=np.float64))
    g = {"W3": d3.T @ h2, "b3": d3.sum(0)}
    d2 = q((d3 @ p["W3"]) * (1 - h2 ** 2))
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = q((d2 @ p["W2"]) * (1 - h1 ** 2))
    g["W1"], g["b1"] = d1.T @ x, d1.sum(0)
    return np.concatenate([g[name].ravel() for name, _ in SHAPES])
