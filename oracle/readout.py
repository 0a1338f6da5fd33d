"""Rigid-body velocities and effective viscosity (Sec. 3).

Velocities. Inside particle i the total flow u + u0 is the rigid motion
v_i + omega_i (x - c_i)^perp (eq. RigidBodyMotion; the BIE makes the interior
traction vanish, Sec. 5), so both are read at the centroid c_i:

    v_i     = u0(c_i) + u_near(c_i) + [u_corr(c_i) - u_corr(c_U)]
    omega_i = (1/2) [vort_near(c_i) + vort_corr(c_i)] - gamma/2

u is defined only up to a constant velocity (Sec. 3 nullspace lemma; Sec. 4.2,
G_per up to a constant), and the expression above fixes it at the value the near sum
takes at the cell centre, which depends on where the particles sit relative to c_U.
Moving every particle by the same vector is a symmetry of the periodic problem, so the
velocities are reported in the gauge that does not depend on that position: the
area-weighted mean over the particles of the disturbance v_i - u0(c_i) is zero,

    v_i <- v_i - sum_k |Omega_k| (v_k - u0(c_k)) / sum_k |Omega_k|.

(Under the fixed-point gauge a stiff configuration drifts as a whole with a speed that
depends on its position, and forward Euler amplifies that drift.) omega is gauge-free.
u0 = (gamma x_2, 0) has vorticity -gamma.

Effective viscosity. eq. (mueff) integrates the shear traction through the
bottom wall D. The particle-stresslet form used here equals it by the force
balance of the cell (Gauss law, Sec. 4.1 lemma on net quantities): the force on
particle i is -int sigma_i, and the cell-averaged shear stress gives

    mu_eff = mu - (1/(2 gamma |U|)) sum_i sum_k w_k [(x_k - c_i)_1 sigma_k,2 + (x_k - c_i)_2 sigma_k,1],

|U| = |det(e1, e2)|. ``mu_eff_wall`` evaluates eq. (mueff) directly with
Gauss-Legendre on D; it is valid only when no particle comes near D.

``mu_eff_contour`` is the contour-deformation form of eq. (mueff) (Sec. 7, the
proposition on efficient evaluation of the effective viscosity), re-derived for the
near set used here (3x3 images of whole particles, centres wrapped into U). The force
through a curve C joining D's end points around the particles is
int_C T = int_C T_near + int_D T_corr, and by translation invariance of G^t

    int_C T_near = sum_q sum_{n=-1,0,1} J_q(-n),   J_q(a) = int over l + a e2 of S^t_{Gamma_q}[sigma],

where l = (C - e1) u C u (C + e1) runs three cells along e1 and only the unshifted
curve Gamma_q is a source. Gauss' law (Sec. 4.1 lemma on net quantities, the exterior
traction of a single layer integrates to -int sigma) on the region between l + a e2 and
l + b e2, closed by the two straight sides through the corners p0 - e1 + k e2 and
p0 + 2 e1 + k e2 (p0 = c_U - e1/2 - e2/2, outward normals), gives
J(b) - J(a) + sides(a, b) = -(force of Gamma_q if it lies between them). With C taken
so that every particle lies in the deformed copy of the cell that holds its centre, the
strips (-1, 0) and (1, 2) hold no source, so

    int_C T_near = sum_q [2 J_q(-1) + J_q(2) - sides_q(-1, 0) + sides_q(1, 2)],

and J(-1), J(2) may be taken on the straight lines D - e2, D + 2 e2. Every target is
at least about half a cell (less the particle radius) from its source curve, so
Gauss-Legendre with m nodes per cell edge and the plain trapezoid rule on the curves
suffice, however the particles sit on D; the correction part is smooth on D.
"""
from __future__ import annotations

import numpy as np

from . import _clib, dilated, geometry, near, periodizer
from .operator import proxy_strengths, to2


def velocities(prob, sigma):
    g = prob.geom
    s2 = to2(np.asarray(sigma, dtype=np.float64))
    f = near.forces(g, s2)
    xi, _, _ = proxy_strengths(prob, s2)
    if prob.cfg.near_set == "dilated":
        un, vn = dilated.near_velocity(g, f, g.centers, prob.cfg.mu)
    else:
        un, vn = _clib.stokeslet_velocity(g.centers, g.x, f, g.shifts(prob.cfg.image_range), prob.cfg.mu)
    uc = periodizer.correction_velocity(prob.P, xi, g.centers, prob.cfg.mu)
    uc0 = periodizer.correction_velocity(prob.P, xi, g.cU[None, :], prob.cfg.mu)
    vc = periodizer.correction_vorticity(prob.P, xi, g.centers, prob.cfg.mu)
    u0 = np.stack([prob.cfg.gamma * g.centers[:, 1], np.zeros(g.No)], axis=1)
    v = u0 + un + uc - uc0
    area = geometry.areas(g)
    v = v - (area[:, None] * (v - u0)).sum(0) / area.sum()
    omega = 0.5 * (vn + vc) - 0.5 * prob.cfg.gamma
    return v, omega


def mu_eff(prob, sigma):
    g = prob.geom
    s2 = to2(np.asarray(sigma, dtype=np.float64))
    rel = g.x - g.centers[g.pid]
    st = (g.w * (rel[:, 0] * s2[:, 1] + rel[:, 1] * s2[:, 0])).sum()
    area = abs(g.e1[0] * g.e2[1] - g.e1[1] * g.e2[0])
    return prob.cfg.mu - st / (2.0 * prob.cfg.gamma * area)


def mu_eff_wall(prob, sigma, nq=64):
    g = prob.geom
    s2 = to2(np.asarray(sigma, dtype=np.float64))
    f = near.forces(g, s2)
    xi, _, _ = proxy_strengths(prob, s2)
    t, wt = periodizer.gauss_legendre(nq)
    xq = g.cU - 0.5 * g.e2 + (0.5 * t)[:, None] * g.e1
    wq = 0.5 * wt * np.linalg.norm(g.e1)
    nD = np.repeat(np.array([[0.0, 1.0]]), nq, axis=0)
    if prob.cfg.near_set == "dilated":
        _, pts, _ = dilated.image_sources(g)
        src, _, _ = dilated.image_sources(g)
        Tn = _clib.near_traction(xq, nD, pts, f[src], np.zeros((1, 2)))
    else:
        Tn = _clib.near_traction(xq, nD, g.x, f, g.shifts(prob.cfg.image_range))
    Tc = periodizer.correction_traction(prob.P, xi, xq, nD)
    T1 = Tn[:, 0] + Tc[:, 0]
    return prob.cfg.mu + (wq * T1).sum() / (prob.cfg.gamma * np.linalg.norm(g.e1))


def contour_points(geom, m):
    """Quadrature of the deformed contour: points [10 m, 2], normals [10 m, 2] and
    signed weights [10 m] (J(-1) twice, J(2) once, the four straight sides with the signs
    of the Gauss-law balance), then the points, normals and weights of D [m]."""
    t, wt = periodizer.gauss_legendre(m)
    t, w = 0.5 * t, 0.5 * wt
    e1, e2 = geom.e1, geom.e2
    l1, l2 = np.linalg.norm(e1), np.linalg.norm(e2)
    p0 = geom.cU - 0.5 * e1 - 0.5 * e2
    nh = np.array([-e1[1], e1[0]]) / l1       # left normal of e1: (0, 1) on D
    nv = np.array([e2[1], -e2[0]]) / l2       # right normal of e2: outward on the right side
    pts, nrm, wts = [], [], []
    for a, coef in ((-1, 2.0), (2, 1.0)):
        for k in (-1, 0, 1):
            pts.append(p0 + a * e2 + (k + 0.5 + t)[:, None] * e1)
            nrm.append(np.tile(nh, (m, 1)))
            wts.append(coef * w * l1)
    for corner, coef in ((p0 + 2 * e1 - e2, -1.0), (p0 - e1 - e2, 1.0), (p0 + 2 * e1 + e2, 1.0), (p0 - e1 + e2, -1.0)):
        pts.append(corner + (0.5 + t)[:, None] * e2)
        nrm.append(np.tile(nv, (m, 1)))
        wts.append(coef * w * l2)
    xD = p0 + (0.5 + t)[:, None] * e1
    return (np.concatenate(pts), np.concatenate(nrm), np.concatenate(wts),
            xD, np.tile(nh, (m, 1)), w * l1)


def mu_eff_contour(prob, sigma, m=16, xi=None):
    """eq. (mueff) by contour deformation (module docstring); valid whether or not
    particles cross D. 3x3 near set only. xi: proxy strengths to use instead of the
    ones this density gives (to separate the proxy solve from the rest in comparisons)."""
    if prob.cfg.near_set != "3x3" or prob.cfg.image_range != 1:
        raise NotImplementedError("contour form derived for the 3x3 near set")
    g = prob.geom
    s2 = to2(np.asarray(sigma, dtype=np.float64))
    f = near.forces(g, s2)
    if xi is None:
        xi, _, _ = proxy_strengths(prob, s2)
    pts, nrm, wts, xD, nD, wD = contour_points(g, m)
    Tn = _clib.near_traction(pts, nrm, g.x, f, np.zeros((1, 2)))
    Tc = periodizer.correction_traction(prob.P, xi, xD, nD)
    F = (wts[:, None] * Tn).sum(0) + (wD[:, None] * Tc).sum(0)
    l1 = np.linalg.norm(g.e1)
    return prob.cfg.mu + (g.e1 / l1) @ F / (prob.cfg.gamma * l1)
