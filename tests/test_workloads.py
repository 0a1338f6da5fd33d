"""Host-side checks of the seeded workload recipes used by the benchmarks (no GPU)."""
import numpy as np
from scipy.spatial import cKDTree

from oracle import geometry
from paper_1912_04501_amd import workloads as W


def test_random_islands_area_fraction_and_clearance():
    """The islands recipe: one island size at the requested area fraction (the boundary
    quadrature of the areas against pi s^2 (1 + A^2 / 2) each), and every pair of islands,
    periodic images included, at least s/5 apart (the clearance of the bounding circles)."""
    wl = W.random_stars(150, 0.2, seed=4, n_nodes=128)
    g = geometry.build_geometry(wl)
    s, A = wl["params"][0, 0], wl["params"][0, 1]
    areas = geometry.areas(g)
    assert np.allclose(areas, np.pi * s * s * (1 + 0.5 * A * A), rtol=1e-12, atol=0)
    assert abs(areas.sum() - 0.2) < 1e-12
    pts = np.concatenate([g.x + sh for sh in g.shifts(1)])
    pid = np.tile(g.pid, 9)
    img = np.repeat(np.arange(9), g.N)
    tree = cKDTree(pts)
    d, j = tree.query(g.x, k=400)
    other = (pid[j] != g.pid[:, None]) | (img[j] != 4)
    dmin = np.where(other, d, np.inf).min()
    assert dmin >= 0.2 * s, (dmin, s)


def test_random_islands_are_seeded():
    a = W.random_stars(40, 0.2, seed=9)
    b = W.random_stars(40, 0.2, seed=9)
    c = W.random_stars(40, 0.2, seed=10)
    assert np.array_equal(a["centers"], b["centers"]) and np.array_equal(a["params"], b["params"])
    assert not np.array_equal(a["centers"], c["centers"])
    assert a["n_nodes"].sum() == 40 * 350
