"""The seeded generator: reproducible, the counts and classification the
workloads state, zero provisional velocity at virtual points."""
import numpy as np

from paper_2304_14690_amd import inputs


def test_config1_counts_and_kinds():
    c = inputs.config1()
    cnt = c.counts()
    assert c.n == (64, 64) and c.k_grid == 12
    assert cnt["F"] + cnt["V"] == 4096
    assert cnt["B"] == round(2 * np.pi * 0.1 * 64)
    lat = c.x[:, :4096].T
    r = np.linalg.norm(lat - 0.5, axis=1)
    assert np.all((r < 0.1) == (c.kind[:4096] == inputs.KIND_V))
    bpts = c.x[:, 4096:].T
    np.testing.assert_allclose(np.linalg.norm(bpts - 0.5, axis=1), 0.1, rtol=1e-14)
    assert np.all(c.u[:, c.kind == inputs.KIND_V] == 0.0)
    assert np.all(c.u[:, c.kind != inputs.KIND_V] != 0.0)


def test_jitter_bounds_and_reproducible():
    a = inputs.jittered_lattice((16, 8), (1 / 16, 1 / 8), 5)
    b = inputs.jittered_lattice((16, 8), (1 / 16, 1 / 8), 5)
    np.testing.assert_array_equal(a, b)
    i = np.arange(128) % 16
    j = np.arange(128) // 16
    assert np.all(np.abs(a[0] - (i + 0.5) / 16) <= 0.3 / 16 + 1e-15)
    assert np.all(np.abs(a[1] - (j + 0.5) / 8) <= 0.3 / 8 + 1e-15)


def test_velocity_modes_formula():
    x = np.random.default_rng(0).uniform(size=(2, 50))
    u = inputs.fourier_velocity(x, 3, 9)
    rng = np.random.Generator(np.random.PCG64(9))
    km = rng.integers(1, 5, size=(3, 2))
    sg = rng.choice(np.array([-1, 1]), size=(3, 2))
    th = rng.uniform(0, 2 * np.pi, size=3)
    a = rng.standard_normal(size=(3, 2))
    k = km * sg
    want = np.zeros((2, 50))
    for m in range(3):
        want += a[m][:, None] * np.cos(2 * np.pi * (k[m] @ x) + th[m])[None, :]
    np.testing.assert_allclose(u, want, atol=1e-13)


def test_3d_and_box_obstacle():
    c = inputs.make_case("t", 3, 16, [inputs.Obstacle("sphere", (0.3, 0.5, 0.5), (0.1,)),
                                      inputs.Obstacle("box", (0.6, 0.4, 0.4), (0.8, 0.6, 0.6))],
                         27, 27, 4, 7, 8)
    cnt = c.counts()
    assert cnt["V"] > 0 and cnt["B"] > 0
    assert cnt["F"] + cnt["V"] == 16 ** 3
