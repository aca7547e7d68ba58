"""The seeded input generators (host only): the batch of independent
problems has the sizes, kinds and CFL numbers its description states."""

import math

import numpy as np

from paper_1908_05834_amd import inputs


def test_mixed_problem_is_seeded_and_sized():
    a, b = inputs.mixed_problem(7), inputs.mixed_problem(7)
    assert a["name"] == b["name"] and a["dt"] == b["dt"]
    assert np.array_equal(a["c0"], b["c0"])
    kinds = set()
    for p in range(24):
        rng = np.random.default_rng(p)
        tri = rng.random() < 0.5
        N = math.exp(rng.uniform(math.log(4e3), math.log(2e5)))
        q = inputs.mixed_problem(p)
        nc = inputs.n_cells(q["mesh"])
        kinds.add(q["layout"])
        if tri:
            n = round(math.sqrt(N / 2))
            assert q["layout"] == "equal_measure" and nc == 2 * n * n
        else:
            n = round(N ** (1 / 3))
            assert q["layout"] == "subcell" and nc == n ** 3
        assert 0.5 <= q["cfl"] <= 4.0
        assert np.all((q["c0"] >= 0) & (q["c0"] <= 1))
    assert kinds == {"equal_measure", "subcell"}


def test_mixed_problem_cfl_definition():
    # dt max over cell centroids |u| / h equals the drawn CFL number; the
    # lattice holds the same field at its nodes
    for p in (0, 2):
        q = inputs.mixed_problem(p, 2000.0, 2000.0)
        mesh = q["mesh"]
        dim = len(q["vel"]["m"])
        n = q["vel"]["m"][0] - 1
        f = inputs.fourier_modes_field(dim, seed=p)
        u = f(inputs.cell_centroids(mesh))
        umax = np.max(np.sqrt(np.sum(u ** 2, axis=1)))
        assert abs(q["dt"] * umax * n - q["cfl"]) <= 1e-12 * q["cfl"]
        nodes = inputs.lattice_nodes(q["vel"]["m"], q["vel"]["origin"], q["vel"]["spacing"])
        assert np.allclose(q["vel"]["u"].T, f(nodes), rtol=0, atol=1e-15)


def test_fourier_modes_are_divergence_free_and_tangential():
    # central differences of the field: zero divergence inside, zero normal
    # component on the box faces
    for dim in (2, 3):
        f = inputs.fourier_modes_field(dim, seed=11)
        rng = np.random.default_rng(3)
        x = rng.uniform(0.1, 0.9, size=(64, dim))
        eps = 1e-5
        div = np.zeros(64)
        for a in range(dim):
            e = np.zeros(dim)
            e[a] = eps
            div += (f(x + e)[:, a] - f(x - e)[:, a]) / (2 * eps)
        assert np.max(np.abs(div)) <= 1e-6
        for a in range(dim):
            for side in (0.0, 1.0):
                y = x.copy()
                y[:, a] = side
                assert np.max(np.abs(f(y)[:, a])) <= 1e-12
