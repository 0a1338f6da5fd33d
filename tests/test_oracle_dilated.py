"""Pins of the oracle's dilated-cell near set (the paper's own G_near of Sec. 4.2):
image combinatorics, the consistency theorem for its discrepancy, and agreement of the
periodic operator and of the solve with the 3x3 image set (both periodize the same
G_per; they differ by the proxy-fit error only)."""
import numpy as np
import pytest

from oracle import dilated, near, periodizer
from oracle import operator as op
from oracle import readout as ro
from oracle.geometry import build_geometry
from paper_1912_04501_amd import workloads as W

DIL = dict(near_set="dilated", M=64, R=1.0)
DIL_WALLS = dict(near_set="dilated", proxy_surface="walls", M=64, m=24, rcond=1e-8)


def test_four_images_per_node_inside_dilated_cell():
    g = build_geometry(W.random_ellipses(6, 0.3, seed=5, skew=0.3, nodes=64))
    xw = dilated.wrap_nodes(g)
    ab = dilated.lattice_coords(g, xw)
    assert np.all((ab >= -0.5) & (ab < 0.5))
    src, pts, mn = dilated.image_sources(g)
    assert np.array_equal(np.bincount(src, minlength=g.N), np.full(g.N, 4))
    ab = dilated.lattice_coords(g, pts)
    assert np.all((ab >= -1.0) & (ab < 1.0))
    # per node: two shifts along e1 and two along e2, the unshifted one among them
    for j in range(0, g.N, 37):
        s = mn[src == j]
        assert len(set(s[:, 0])) == 2 and len(set(s[:, 1])) == 2 and 0 in s[:, 0] and 0 in s[:, 1]
    # a wrapped node differs from the node by a lattice vector
    d = dilated.lattice_coords(g, xw) - dilated.lattice_coords(g, g.x)
    assert np.abs(d - np.round(d)).max() < 1e-12


def test_fast_sum_equals_plain_loops():
    g = build_geometry(W.random_ellipses(3, 0.25, seed=2, nodes=64))
    s2 = np.random.default_rng(0).standard_normal((g.N, 2))
    assert np.abs(dilated.near_traction(g, s2) - dilated.near_traction_fast(g, s2)).max() < 1e-13


def test_dilated_discrepancy_is_consistent():
    """Theorem (consistency): W^T (g0 - g) = 0 for the discrepancy of this near sum."""
    prob = op.make_problem(W.random_ellipses(8, 0.3, seed=3, skew=0.2), **DIL)
    g = prob.geom
    f = near.forces(g, np.random.default_rng(1).standard_normal((g.N, 2)))
    d = dilated.discrepancy(g, prob.W, f, 1.0)
    Wc = periodizer.consistency_W(g, prob.W)
    res = Wc @ (periodizer.g0_vector(g, prob.W, f.sum(0)) - d)
    assert np.abs(res).max() < 1e-12 * max(1.0, np.abs(d).max())


def test_wall_proxies_on_the_dilated_cell_boundary():
    """M / 4 proxies on each side of U~ (corners c_U +- e1 +- e2), evenly spaced along it."""
    g = build_geometry(W.random_ellipses(4, 0.2, seed=1, skew=0.3, nodes=64))
    P = dilated.wall_proxies(g, 64)
    ab = dilated.lattice_coords(g, P)
    on = np.abs(np.abs(ab) - 1.0) < 1e-12
    assert np.all(on.sum(1) == 1)                         # on exactly one wall, never at a corner
    for side in ((1, -1), (0, 1), (1, 1), (0, -1)):         # bottom, right, top, left
        k = on[:, side[0]] & (np.sign(ab[:, side[0]]) == side[1])
        assert k.sum() == 16
        t = np.sort(ab[k, 1 - side[0]])
        assert np.abs(np.diff(t) - 0.125).max() < 1e-12 and abs(t[0] + 1 - 0.0625) < 1e-12
    with pytest.raises(ValueError):
        dilated.wall_proxies(g, 30)


@pytest.mark.parametrize("per", [DIL, DIL_WALLS], ids=["circle_proxies", "wall_proxies"])
@pytest.mark.parametrize("wl", [W.single_ellipse(), W.random_ellipses(10, 0.3, seed=3)])
def test_same_periodic_operator_and_solution_as_3x3(wl, per):
    """Both near sets periodize the same G_per: the operator on a smooth force-free
    density and the solution's omega, relative velocities and mu_eff agree to the
    proxy-fit level, with the U~ set's proxies on a circle or on U~'s walls. (With a net
    force F the periodic pressure grows linearly across the cell, so values at a node and
    at its wrapped copy differ by F . shift / |U| times n: a comparison needs F = 0, as
    every solution has.)"""
    p3 = op.make_problem(wl)
    pd = op.make_problem(wl, **per)
    g = p3.geom
    t = np.arange(p3.N)
    s2 = np.stack([np.cos(2 * np.pi * t / 97), np.sin(2 * np.pi * t / 61)], axis=1)
    for q in range(g.No):
        sl = g.particle_slice(q)
        s2[sl] -= (g.w[sl, None] * s2[sl]).sum(0) / g.w[sl].sum()
    sig = op.to1(s2)
    a, b = op.apply(p3, sig), op.apply(pd, sig)
    assert np.abs(a - b).max() < 1e-6 * np.abs(a).max()
    x3, _ = op.solve(p3, tol=1e-12)
    xd, _ = op.solve(pd, tol=1e-12)
    v3, o3 = ro.velocities(p3, x3)
    vd, od = ro.velocities(pd, xd)
    assert np.abs(o3 - od).max() < 1e-6
    assert np.abs((v3 - v3.mean(0)) - (vd - vd.mean(0))).max() < 1e-6
    assert abs(ro.mu_eff(p3, x3) - ro.mu_eff(pd, xd)) < 1e-6


def test_rejects_large_particles():
    wl = W.single_ellipse(a=0.3, b=0.1)
    with pytest.raises(ValueError):
        op.make_problem(wl, **DIL)
