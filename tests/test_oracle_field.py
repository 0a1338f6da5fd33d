"""Pins of the oracle's flow field u(x), p(x) (Sec. 3, Sec. 5 eqs. BIEurep/BIEprep, Sec. 6.3)
against properties the field must have: no slip on every particle, the periodicity of the
disturbance, incompressibility, the rigid motion inside the particles, and agreement of
the refined close rule with the plain rule where both are accurate."""
import numpy as np
import pytest

from oracle import field
from oracle import operator as op
from oracle import readout as ro
from paper_1912_04501_amd import workloads as W


@pytest.fixture(scope="module", params=["ellipses", "star"])
def solved(request):
    wl = W.two_ellipses(2e-2, n_nodes=256, skew=0.2) if request.param == "ellipses" else W.star_and_ellipse()
    prob = op.make_problem(wl)
    x, _ = op.solve(prob, tol=1e-13)
    v, om = ro.velocities(prob, x)
    return prob, x, v, om


def test_no_slip_limit(solved):
    """Approaching a boundary point x_b along its normal, u(x_b + d n) tends to the
    particle's rigid motion v + omega (x_b - c)^perp: the quadratic extrapolation to d = 0
    from d = 1, 2, 3 times 1e-4 hits it to 1e-7 (the O(d^3) term: 2.4e-8 at the tip of the
    0.25 x 0.125 ellipse, falling eightfold per halving of d, the same at 256 and 512 nodes;
    the plain rule's error at these distances is O(1))."""
    prob, x, v, om = solved
    g = prob.geom
    for i0 in (10, 100, 200):
        q = g.pid[i0]
        rel = g.x[i0] - g.centers[q]
        ur = v[q] + om[q] * np.array([-rel[1], rel[0]])
        d = np.array([1e-4, 2e-4, 3e-4])
        u, p = field.field(prob, x, g.x[i0][None] + d[:, None] * g.n[i0][None])
        e0 = 3.0 * u[0] - 3.0 * u[1] + u[2]
        assert np.abs(e0 - ur).max() < 1e-7, (i0, e0, ur)
        assert np.all(np.isfinite(p))


def test_periodic_disturbance(solved):
    prob, x, v, om = solved
    g = prob.geom
    pts = np.array([[0.05, 0.41], [-0.33, 0.2], [0.47, -0.46]])
    u1, p1 = field.field(prob, x, pts)
    u2, p2 = field.field(prob, x, pts + g.e1)
    u3, p3 = field.field(prob, x, pts + g.e2)
    assert np.abs(u2 - u1).max() < 1e-14 and np.abs(p2 - p1).max() < 1e-13
    # u0 = (gamma y, 0) grows by gamma e2_2 = gamma along e2
    assert np.abs(u3 - u1 - np.array([prob.cfg.gamma, 0.0])).max() < 1e-14 and np.abs(p3 - p1).max() < 1e-13


def test_incompressible(solved):
    prob, x, v, om = solved
    h = 1e-5
    c = np.array([[0.0, 0.45], [-0.4, 0.3]])
    ux = (field.field(prob, x, c + [h, 0])[0] - field.field(prob, x, c - [h, 0])[0]) / (2 * h)
    uy = (field.field(prob, x, c + [0, h])[0] - field.field(prob, x, c - [0, h])[0]) / (2 * h)
    div = ux[:, 0] + uy[:, 1]
    assert np.abs(div).max() < 1e-8 * max(1.0, np.abs(ux).max(), np.abs(uy).max())


def test_interior_rigid_motion(solved):
    prob, x, v, om = solved
    g = prob.geom
    pts = np.array([g.centers[0], g.centers[1] + 0.3 * (g.x[g.offsets[1]] - g.centers[1])])
    u, p = field.field(prob, x, pts)
    assert np.abs(u[0] - v[0]).max() < 1e-15
    rel = pts[1] - g.centers[1]
    assert np.abs(u[1] - (v[1] + om[1] * np.array([-rel[1], rel[0]]))).max() < 1e-15
    assert np.all(np.isnan(p))


def test_refined_rule_matches_plain_rule_away_from_curves(solved):
    """Between 10 h and 20 h from a curve both rules are accurate to near rounding:
    widening the close reach (more points on the refined rule) changes nothing."""
    prob, x, v, om = solved
    g = prob.geom
    i0 = 50
    h = g.w[g.particle_slice(g.pid[i0])].sum() / g.n_nodes[g.pid[i0]]
    pts = g.x[i0][None] + np.array([12 * h, 15 * h, 18 * h])[:, None] * g.n[i0][None]
    u1, p1 = field.field(prob, x, pts, close_factor=10.0)
    u2, p2 = field.field(prob, x, pts, close_factor=20.0)
    assert np.abs(u1 - u2).max() < 1e-12 * np.abs(u1).max()
    assert np.abs(p1 - p2).max() < 1e-11 * max(1.0, np.abs(p1).max())
