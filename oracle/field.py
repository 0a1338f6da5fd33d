"""Velocity and pressure of the flow at points of the fluid (Sec. 3; Sec. 5 eqs. BIEurep,
BIEprep; Sec. 7: the quasi-static solver also returns u(x) and p(x)). Test infrastructure.

For a solved density sigma the disturbance field is the periodic single layer plus the
proxy correction (Sec. 6.2), evaluated at the target's periodic copy x_w in the cell U:

    u(x) = u0(x) + sum_q sum_{s in S9} S_{Gamma_q + s}[sigma](x_w) + u_corr(x_w) - u_corr(c_U) - V,
    p(x) =         sum_q sum_{s in S9} P_{Gamma_q + s}[sigma](x_w) + p_corr(x_w),

with S the Stokeslet single layer (eq. Gv) and P its pressure (eq. Gp), u0 = (gamma x_2, 0),
V the velocity gauge of the readout (the area-weighted mean disturbance of the particles)
and p defined up to the constant of this representation.

Near a curve the trapezoid rule loses accuracy (Sec. 6.3). Here the layer potential of
such a (target, curve image) pair is evaluated as the integral of the trigonometric
interpolant of sigma over the exact curve, by the trapezoid rule on a refined grid: the
curve is re-sampled from its shape at K times the node count and sigma by FFT
interpolation. This is an independent check of the device's Laplace-decomposition
(barycentric Cauchy) rule; K is chosen from the target's distance so that the refined
rule's error exp(-2 pi d K / h) is below 1e-14.

Targets inside a particle (image) get the rigid motion of that particle and p = NaN.
"""
from __future__ import annotations

import numpy as np

from . import _clib, geometry, near, periodizer
from .kernels import pressure_apply, stokeslet_apply
from .operator import proxy_strengths, to2


def wrap_points(geom, x):
    """(x_w, L): x_w = x - L in U, L a lattice vector."""
    B = np.stack([geom.e1, geom.e2], axis=1)
    ab = np.linalg.solve(B, (np.asarray(x, float) - geom.cU).T).T
    k = np.floor(ab + 0.5)
    L = k[:, :1] * geom.e1 + k[:, 1:] * geom.e2
    return x - L, L


def _inside(geom, q, pts):
    """Mask of points inside particle q (unshifted), from its shape."""
    c = geom.centers[q]
    th = geom.theta[q]
    d = pts - c
    bu = np.cos(th) * d[:, 0] + np.sin(th) * d[:, 1]
    bv = -np.sin(th) * d[:, 0] + np.cos(th) * d[:, 1]
    kind = 0 if geom.kind is None else int(geom.kind[q])
    if kind == 0:
        a, b = (geom.a[q], geom.b[q]) if geom.params is None else geom.params[q][:2]
        return (bu / a) ** 2 + (bv / b) ** 2 < 1.0
    s, A, om, ph = geom.params[q]
    r = s * (1.0 + A * np.cos(om * np.arctan2(bv, bu) + ph))
    return bu * bu + bv * bv < r * r


def _refined_curve(geom, q, sigma2, K):
    """Curve q re-sampled at K N_q points from its shape, sigma by FFT interpolation:
    (points, weights, sigma) on the fine grid."""
    sl = geom.particle_slice(q)
    n = geom.n_nodes[q]
    kind = 0 if geom.kind is None else int(geom.kind[q])
    prm = np.array([geom.a[q], geom.b[q], 0, 0]) if geom.params is None else geom.params[q]
    nf = K * n
    x, xp, tau, nrm, w, kap = geometry.particle_nodes(geom.centers[q], float(geom.theta[q]), kind, prm, nf)
    out = np.zeros((nf, 2))
    for comp in range(2):
        c = np.fft.fft(sigma2[sl, comp])
        if n % 2 == 0:      # split the Nyquist mode symmetrically
            c[n // 2] *= 0.5
            cf = np.zeros(nf, complex)
            cf[:n // 2 + 1] = c[:n // 2 + 1]
            cf[nf - n // 2:] = c[n // 2:]
        else:
            cf = np.zeros(nf, complex)
            cf[:(n + 1) // 2] = c[:(n + 1) // 2]
            cf[nf - (n - 1) // 2:] = c[(n + 1) // 2:]
        out[:, comp] = np.real(np.fft.ifft(cf)) * K
    return x, w, out


def field(prob, sigma, targets, close_factor=10.0):
    """u [n, 2] (total velocity) and p [n] at the targets [n, 2] for the density sigma (SoA)."""
    g = prob.geom
    mu, gamma = prob.cfg.mu, prob.cfg.gamma
    s2 = to2(np.asarray(sigma, float))
    f = near.forces(g, s2)
    xi, _, _ = proxy_strengths(prob, s2)
    targets = np.asarray(targets, float).reshape(-1, 2)
    xw, L = wrap_points(g, targets)
    shifts = g.shifts(1)
    nt = len(targets)
    # rigid-body gauge of the readout
    from .readout import velocities
    v, om = velocities(prob, sigma)
    # near images (plain rule), proxy correction
    un, _ = _clib.stokeslet_velocity(xw, g.x, f, shifts, mu)
    pn = np.zeros(nt)
    for s in shifts:
        r = xw[:, None, :] - (g.x + s)[None]
        pn += pressure_apply(r, f[None]).sum(1)
    fx = periodizer.xi_to_forces(xi)
    uc = periodizer.correction_velocity(prob.P, xi, xw, mu) - periodizer.correction_velocity(prob.P, xi, g.cU[None], mu)
    pc = pressure_apply(xw[:, None, :] - prob.P[None], fx[None]).sum(1)
    # the gauge constant V: velocities() returns v already gauged; recover V from one particle
    ung, _ = _clib.stokeslet_velocity(g.centers, g.x, f, shifts, mu)
    ucg = periodizer.correction_velocity(prob.P, xi, g.centers, mu) - periodizer.correction_velocity(prob.P, xi,
                                                                                                      g.cU[None], mu)
    u0c = np.stack([gamma * g.centers[:, 1], np.zeros(g.No)], axis=1)
    V = (u0c + ung + ucg - v)[0]
    u = np.stack([gamma * targets[:, 1], np.zeros(nt)], axis=1) + un + uc - V[None]
    p = pn + pc
    # interior points: the rigid motion of the particle image that holds them
    inside = np.full(nt, -1)
    inside_s = np.zeros((nt, 2))
    for q in range(g.No):
        for s in shifts:
            ins = _inside(g, q, xw - s)
            inside[ins] = q
            inside_s[ins] = s
    # close pairs of fluid points: replace the plain rule of a curve image by the refined one
    for q in range(g.No):
        sl = g.particle_slice(q)
        h = g.w[sl].sum() / g.n_nodes[q]
        for s in shifts:
            pts = g.x[sl] + s
            d = np.sqrt(((xw[:, None, :] - pts[None]) ** 2).sum(-1)).min(1)
            close_t = np.nonzero((d < close_factor * h) & (inside < 0))[0]
            if len(close_t) == 0:
                continue
            r_plain = xw[close_t][:, None, :] - pts[None]
            u[close_t] -= stokeslet_apply(r_plain, f[sl][None], mu).sum(1)
            p[close_t] -= pressure_apply(r_plain, f[sl][None]).sum(1)
            for i in close_t:
                # local node spacing can exceed the mean by about half on the stars
                K = int(np.ceil(1.5 * 35.0 * h / (2.0 * np.pi * d[i])))
                if K > 2048:
                    raise ValueError("target too close to a curve for the refined rule")
                xf, wf, sf = _refined_curve(g, q, s2, max(K, 2))
                ff = wf[:, None] * sf
                r = xw[i][None, :] - (xf + s)
                u[i] += stokeslet_apply(r, ff, mu).sum(0)
                p[i] += pressure_apply(r, ff).sum(0)
    for i in np.nonzero(inside >= 0)[0]:
        q, s = inside[i], inside_s[i]
        rel = xw[i] - (g.centers[q] + s)
        u[i] = v[q] + np.array([gamma * (s[1] + targets[i, 1] - xw[i, 1]), 0.0]) + om[q] * np.array([-rel[1], rel[0]])
        p[i] = np.nan
    return u, p
