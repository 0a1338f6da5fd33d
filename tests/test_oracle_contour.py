"""Pins of the contour-deformation effective viscosity (Sec. 7, efficient evaluation of the
effective viscosity; re-derived for the 3x3 near set, oracle/readout.py).

* Gauss' law for one curve (Sec. 4.1 lemma on net quantities): around a closed loop the
  single-layer traction integrates to -int sigma if the loop holds the curve, to 0 if not.
  The contour form rests on exactly this balance.
* With D clear of particles the deformed contour and eq. (mueff) on D itself agree to
  rounding.
* With particles across D, eq. (mueff) on D is wrong while the contour form agrees with
  the particle-stresslet identity and with D's integral for the same suspension moved
  off D (translation invariance, to the MFS periodizer's error).
"""
import numpy as np
import pytest

from oracle import _clib, geometry, near, periodizer
from oracle import operator as op
from oracle import readout
from paper_1912_04501_amd import workloads as W


def _loop(x0, x1, y0, y1, m=40):
    """Gauss-Legendre nodes on the rectangle's four sides, outward normals, weights."""
    t, w = periodizer.gauss_legendre(m)
    s = 0.5 * (t + 1.0)
    pts, nrm, wts = [], [], []
    for a, b, n in (((x0, y0), (x1, y0), (0.0, -1.0)), ((x1, y0), (x1, y1), (1.0, 0.0)),
                    ((x1, y1), (x0, y1), (0.0, 1.0)), ((x0, y1), (x0, y0), (-1.0, 0.0))):
        a, b = np.array(a), np.array(b)
        pts.append(a + s[:, None] * (b - a))
        nrm.append(np.tile(n, (m, 1)))
        wts.append(0.5 * w * np.linalg.norm(b - a))
    return np.concatenate(pts), np.concatenate(nrm), np.concatenate(wts)


def test_gauss_law_on_closed_loops():
    g = geometry.build_geometry(W.single_ellipse(n_nodes=96, theta=0.4))
    rng = np.random.default_rng(3)
    s2 = rng.standard_normal((g.N, 2))
    f = near.forces(g, s2)
    F = f.sum(0)
    for (x0, x1, y0, y1), enclosed in (((-0.4, 0.5, -0.35, 0.3), True), ((0.35, 1.2, -0.4, 0.4), False)):
        pts, nrm, wts = _loop(x0, x1, y0, y1)
        T = _clib.near_traction(pts, nrm, g.x, f, np.zeros((1, 2)))
        flux = (wts[:, None] * T).sum(0)
        want = -F if enclosed else np.zeros(2)
        assert np.abs(flux - want).max() < 1e-10 * np.abs(F).max(), (flux, want)


def _solved(wl):
    prob = op.make_problem(wl)
    x, _ = op.solve(prob, tol=1e-12)
    return prob, x


@pytest.mark.parametrize("center", [(0.0, 0.0), (0.13, -0.21)])
def test_contour_equals_wall_when_D_is_clear(center):
    prob, x = _solved(W.single_ellipse(skew=0.2, center=center))
    a = readout.mu_eff_contour(prob, x)
    b = readout.mu_eff_wall(prob, x)
    assert abs(a - b) < 1e-12, (a, b)


def test_contour_quadrature_converged():
    prob, x = _solved(W.random_ellipses(3, 0.2, seed=21, nodes=96, skew=0.15))
    assert abs(readout.mu_eff_contour(prob, x, m=16) - readout.mu_eff_contour(prob, x, m=32)) < 1e-13


@pytest.mark.parametrize("delta", [(0.0, -0.45), (0.31, 0.42)])
def test_contour_with_particles_across_D(delta):
    wl = W.single_ellipse(skew=0.2, theta=0.7)
    prob0, x0 = _solved(wl)
    clear = readout.mu_eff_wall(prob0, x0)
    prob, x = _solved(dict(wl, centers=wl["centers"] + np.array(delta)))
    wall = readout.mu_eff_wall(prob, x)
    cont = readout.mu_eff_contour(prob, x)
    assert abs(wall - clear) > 1e-2                       # D's own integral breaks
    assert abs(cont - clear) < 3e-6                       # MFS translation error (P15)
    assert abs(cont - readout.mu_eff(prob, x)) < 1e-7


def test_contour_many_particles_across_walls():
    wl = W.random_ellipses(3, 0.2, seed=21, nodes=96, skew=0.15)
    for delta in ((0.0, 0.0), (0.13, -0.21)):
        prob, x = _solved(dict(wl, centers=wl["centers"] + np.array(delta)))
        assert abs(readout.mu_eff_contour(prob, x) - readout.mu_eff(prob, x)) < 1e-7


def test_contour_rejects_other_near_sets():
    prob = op.make_problem(W.single_ellipse(), image_range=2, R=2.5, M=96, m=64)
    with pytest.raises(NotImplementedError):
        readout.mu_eff_contour(prob, np.zeros(2 * prob.geom.N))
