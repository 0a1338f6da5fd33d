"""Lattice and particle discretisation (Sec. 2, Sec. 6 trapezoid rule, Sec. 7).

* Lattice: e1 = (1, 0), e2 = (s, 1). The skew is reduced to [-1/2, 1/2) with
  s <- s - floor(s + 1/2); this is the integer shift e2 <- e2 - round(s) e1 of
  Sec. 7 (same lattice, bounded skewness).
* Cell: centre c_U = (0, 0); a particle centre is wrapped into the cell by
  reducing its lattice coordinates (alpha, beta) = [e1 e2]^{-1} (c - c_U) the same way.
* Ellipse i: x(t) = c + R(theta) (a cos t, b sin t), t_k = 2 pi k / N_i.
  Periodic trapezoid rule (Sec. 6): w_k = (2 pi / N_i) |x'(t_k)|.
  Tangent tau = x'/|x'|, outward normal n = (tau_2, -tau_1), curvature
  kappa = a b / |x'|^3. The perimeter centroid (Sec. 2) of an ellipse is c.
* Star (the smooth star-shaped curves of Sec. 8 Examples 2 and 4): in the body frame
  x(t) = r(t) (cos t, sin t), r(t) = s (1 + A cos(omega t + phi)), with the same rule,
  tangent and normal, and the signed curvature kappa = (x' y'' - y' x'') / |x'|^3. Its
  reference point c (the polar origin, inside the curve) carries the rigid motion; any
  body-fixed point inside serves, since the particles are force- and torque-free.
  For stars, ``a`` holds the largest radius s (1 + |A|) and ``b`` the smallest.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def reduce_skew(s: float) -> float:
    return float(s - np.floor(s + 0.5))


def lattice(skew: float):
    s = reduce_skew(skew)
    return np.array([1.0, 0.0]), np.array([s, 1.0])


def wrap_centers(c, e1, e2, cU=(0.0, 0.0)):
    B = np.stack([e1, e2], axis=1)  # columns e1, e2
    ab = np.linalg.solve(B, (np.asarray(c, float) - np.asarray(cU)).T).T
    ab = ab - np.floor(ab + 0.5)
    return np.asarray(cU) + ab @ B.T


@dataclass
class Geometry:
    e1: np.ndarray
    e2: np.ndarray
    cU: np.ndarray
    centers: np.ndarray   # (No, 2), wrapped
    theta: np.ndarray
    a: np.ndarray
    b: np.ndarray
    n_nodes: np.ndarray   # (No,)
    offsets: np.ndarray   # (No + 1,)
    x: np.ndarray         # (N, 2) nodes
    xp: np.ndarray        # (N, 2) dx/dt
    tau: np.ndarray       # (N, 2) unit tangent
    n: np.ndarray         # (N, 2) outward normal
    w: np.ndarray         # (N,) trapezoid weights
    kappa: np.ndarray     # (N,) curvature
    pid: np.ndarray       # (N,) particle index of each node
    kind: np.ndarray = None    # (No,) 0 ellipse, 1 star
    params: np.ndarray = None  # (No, 4) ellipse (a, b, 0, 0); star (s, A, omega, phi)

    @property
    def N(self) -> int:
        return int(self.offsets[-1])

    @property
    def No(self) -> int:
        return len(self.a)

    def shifts(self, rng=1):
        """Image shifts m e1 + n e2 for m, n in [-rng, rng] (the zero shift is the centre entry)."""
        out = []
        for m in range(-rng, rng + 1):
            for k in range(-rng, rng + 1):
                out.append(m * self.e1 + k * self.e2)
        return np.array(out)

    def particle_slice(self, i):
        return slice(int(self.offsets[i]), int(self.offsets[i + 1]))


def ellipse_nodes(c, theta, a, b, N):
    t = 2.0 * np.pi * np.arange(N) / N
    ct, st = np.cos(theta), np.sin(theta)
    px, py = a * np.cos(t), b * np.sin(t)
    dx, dy = -a * np.sin(t), b * np.cos(t)
    x = np.stack([c[0] + ct * px - st * py, c[1] + st * px + ct * py], axis=1)
    xp = np.stack([ct * dx - st * dy, st * dx + ct * dy], axis=1)
    sp = np.sqrt((xp * xp).sum(1))
    tau = xp / sp[:, None]
    n = np.stack([tau[:, 1], -tau[:, 0]], axis=1)
    w = 2.0 * np.pi * sp / N
    kappa = a * b / sp ** 3
    return x, xp, tau, n, w, kappa


def star_nodes(c, theta, s, A, omega, phi, N):
    t = 2.0 * np.pi * np.arange(N) / N
    u = omega * t + phi
    r = s * (1.0 + A * np.cos(u))
    rp = -s * A * omega * np.sin(u)
    rpp = -s * A * omega * omega * np.cos(u)
    ct_, st_ = np.cos(t), np.sin(t)
    X, Y = r * ct_, r * st_
    Xp, Yp = rp * ct_ - r * st_, rp * st_ + r * ct_
    Xpp = rpp * ct_ - 2.0 * rp * st_ - r * ct_
    Ypp = rpp * st_ + 2.0 * rp * ct_ - r * st_
    ca, sa = np.cos(theta), np.sin(theta)
    x = np.stack([c[0] + ca * X - sa * Y, c[1] + sa * X + ca * Y], axis=1)
    xp = np.stack([ca * Xp - sa * Yp, sa * Xp + ca * Yp], axis=1)
    sp = np.sqrt((xp * xp).sum(1))
    tau = xp / sp[:, None]
    n = np.stack([tau[:, 1], -tau[:, 0]], axis=1)
    w = 2.0 * np.pi * sp / N
    kappa = (Xp * Ypp - Yp * Xpp) / sp ** 3
    return x, xp, tau, n, w, kappa


def shape_params(wl):
    """(kind, params) of every particle; ellipses by default (params a, b)."""
    n = len(wl["theta"])
    if "kind" not in wl:
        p = np.zeros((n, 4))
        p[:, 0], p[:, 1] = wl["a"], wl["b"]
        return np.zeros(n, dtype=np.int64), p
    return np.asarray(wl["kind"], dtype=np.int64), np.asarray(wl["params"], dtype=float).reshape(n, 4)


def radii(kind, p):
    """(largest, smallest) distance from the reference point to the curve."""
    if kind == 0:
        return max(p[0], p[1]), min(p[0], p[1])
    return p[0] * (1.0 + abs(p[1])), p[0] * (1.0 - abs(p[1]))


def areas(geom):
    """Area of every particle from its shape: pi a b for an ellipse; for a star
    r = s (1 + A cos(omega t + phi)) with integer omega >= 1, (1/2) int r^2 dt =
    pi s^2 (1 + A^2 / 2)."""
    out = np.zeros(geom.No)
    for i in range(geom.No):
        if geom.kind is None or int(geom.kind[i]) == 0:
            p = (geom.a[i], geom.b[i]) if geom.params is None else geom.params[i][:2]
            out[i] = np.pi * p[0] * p[1]
        else:
            s, A = geom.params[i][0], geom.params[i][1]
            out[i] = np.pi * s * s * (1.0 + 0.5 * A * A)
    return out


def particle_nodes(c, theta, kind, p, N):
    if kind == 0:
        return ellipse_nodes(c, theta, p[0], p[1], N)
    return star_nodes(c, theta, p[0], p[1], p[2], p[3], N)


def build_geometry(wl) -> Geometry:
    e1, e2 = lattice(wl["skew"])
    cU = np.zeros(2)
    c = wrap_centers(np.asarray(wl["centers"], float), e1, e2, cU)
    nn = np.asarray(wl["n_nodes"], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(nn)])
    kind, prm = shape_params(wl)
    th = np.asarray(wl["theta"], float)
    parts = [particle_nodes(c[i], float(th[i]), int(kind[i]), prm[i], int(nn[i])) for i in range(len(nn))]
    x, xp, tau, n, w, kappa = (np.concatenate([p[k] for p in parts]) for k in range(6))
    pid = np.repeat(np.arange(len(nn)), nn)
    rr = np.array([radii(int(kind[i]), prm[i]) for i in range(len(nn))]).reshape(-1, 2)
    return Geometry(e1, e2, cU, c, th, rr[:, 0].copy(), rr[:, 1].copy(), nn, offs, x, xp, tau, n, w, kappa, pid,
                    kind, prm)
