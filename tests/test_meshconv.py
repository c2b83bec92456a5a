"""Host logic of the mesh-convergence driver: interpolation between nested meshes and
the least-squares rate (no GPU)."""
import numpy as np

from paper_2304_09180_amd import meshconv


def test_linear_fields_are_resampled_exactly():
    ny, nx = 5, 8
    yc = (np.arange(ny) + 0.5) / ny
    xc = (np.arange(nx) + 0.5) / nx
    f = 2.0 + 3.0 * xc[None, :] - 1.5 * yc[:, None]
    g = meshconv.to_fine(f, (4 * ny, 4 * nx))
    Yc = (np.arange(4 * ny) + 0.5) / (4 * ny)
    Xc = (np.arange(4 * nx) + 0.5) / (4 * nx)
    assert np.allclose(g, 2.0 + 3.0 * Xc[None, :] - 1.5 * Yc[:, None], atol=1e-13)


def test_smooth_field_errors_fall_at_second_order_and_the_rate_fit_sees_it():
    def field(ny, nx):
        yc = (np.arange(ny) + 0.5) / ny
        xc = (np.arange(nx) + 0.5) / nx
        return {n: np.sin(np.pi * xc)[None, :] * np.exp(yc)[:, None] * (k + 1)
                for k, n in enumerate(("S1", "E1", "PMU", "E2", "E2B"))}
    hs = [1.0, 0.5, 0.25, 0.0625]
    sols = [field(int(8 / h), int(32 / h)) for h in hs]
    out = meshconv.errors_and_rates(hs, sols)
    for q in meshconv.QUANTITIES:
        e = out[q]["errors"]
        assert e[0] > e[1] > e[2] > 0.0
        assert 1.8 < out[q]["rate"] < 2.4, (q, out[q])


def test_the_study_meshes_are_nested_and_square():
    for h in (3.0, 1.5, 0.75, 0.375):
        d = meshconv.channel(h, 4e-6)
        assert d["nx"] == round(120 / h) and d["ny"] == round(30 / h)
        assert abs(d["Lx"] / d["nx"] - d["Ly"] / d["ny"]) < 1e-15
        assert abs((d["inj_x1"] - d["inj_x0"]) - 0.045) < 1e-12
