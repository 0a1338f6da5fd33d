"""The paper's own near set (Sec. 4.2, Def. of G_near; Sec. 6.2), test infrastructure.

Every node is wrapped into the unit cell U individually (lattice coordinates reduced
to [-1/2, 1/2)), and the near sources of a node are its images inside the dilated
cell U~ (same centre, walls parallel to U's, twice the side): lattice coordinates in
[-1, 1). Each node has exactly two admissible shifts along e1 and two along e2, so
four near images, against nine for the 3x3 image set of whole particles.

Targets (nodes and particle centres) lie in U. For a target in U every image within
lattice distance 1/2 of it lies in U~, so the images a target interacts with at short
range (its own curve, close neighbours) are all present as long as a particle's
extent stays below that distance; the rest of the periodic sum is smooth in U and is
carried by the proxy correction, fitted to the discrepancy of this near sum.

Everything is written as the plain definition: explicit image lists and direct sums
(the discrepancy is the difference of near sums evaluated at both walls).
"""
from __future__ import annotations

import numpy as np

from . import _clib


def lattice_coords(geom, x):
    B = np.stack([geom.e1, geom.e2], axis=1)
    return np.linalg.solve(B, (np.asarray(x, float) - geom.cU).T).T


def wrap_nodes(geom):
    """Node positions wrapped into U one by one."""
    ab = lattice_coords(geom, geom.x)
    ab = ab - np.floor(ab + 0.5)
    return geom.cU + ab @ np.stack([geom.e1, geom.e2])


def image_sources(geom):
    """(source node index, image point, (m, n)) of every near image: xw_j + m e1 + n e2
    with lattice coordinates in [-1, 1)."""
    xw = wrap_nodes(geom)
    idx, pts, mn = [], [], []
    for m in (-1, 0, 1):
        for n in (-1, 0, 1):
            p = xw + m * geom.e1 + n * geom.e2
            ab = lattice_coords(geom, p)
            ok = np.all((ab >= -1.0) & (ab < 1.0), axis=1)
            idx.append(np.nonzero(ok)[0])
            pts.append(p[ok])
            mn.append(np.repeat(np.array([[m, n]]), ok.sum(), axis=0))
    return np.concatenate(idx), np.concatenate(pts), np.concatenate(mn)


def near_traction(geom, sigma2):
    """T_near at the wrapped nodes from the U~ images, self pair (own node, no shift) skipped."""
    f = geom.w[:, None] * sigma2
    xw = wrap_nodes(geom)
    src, pts, mn = image_sources(geom)
    out = np.zeros((geom.N, 2))
    for i in range(geom.N):
        keep = ~((src == i) & (mn[:, 0] == 0) & (mn[:, 1] == 0))
        out[i] = _clib.near_traction(xw[i:i + 1], geom.n[i:i + 1], pts[keep], f[src[keep]],
                                     np.zeros((1, 2)))[0]
    return out


def near_traction_fast(geom, sigma2):
    """The same sum through one call per shift pattern (no Python loop over targets):
    the self image is the only zero-distance pair and contributes exactly 0 once
    skipped, so it is removed by passing each target's own index."""
    f = geom.w[:, None] * sigma2
    xw = wrap_nodes(geom)
    src, pts, mn = image_sources(geom)
    zero = (mn[:, 0] == 0) & (mn[:, 1] == 0)
    # position of node i's unshifted image in the source list
    self_pos = np.full(geom.N, -1, dtype=np.int64)
    self_pos[src[zero]] = np.nonzero(zero)[0]
    return _clib.near_traction(xw, geom.n, pts, f[src], np.zeros((1, 2)), self_pos)


def near_velocity(geom, f, targets, mu):
    """Stokeslet velocity and vorticity at targets in U from the U~ images."""
    src, pts, _ = image_sources(geom)
    return _clib.stokeslet_velocity(targets, pts, f[src], np.zeros((1, 2)), mu)


def discrepancy(geom, W, f, mu):
    """g of Sec. 6.2 step 2 for the U~ near sum: [u_R - u_L; T_R - T_L; u_U - u_D; T_U - T_D]
    at the wall points, each near sum evaluated directly at both walls."""
    src, pts, _ = image_sources(geom)
    fs = f[src]
    zero = np.zeros((1, 2))
    out = []
    for (x, shift, nrm) in ((W["xL"], geom.e1, W["nL"]), (W["xD"], geom.e2, W["nD"])):
        uA, _ = _clib.stokeslet_velocity(x + shift, pts, fs, zero, mu)
        uB, _ = _clib.stokeslet_velocity(x, pts, fs, zero, mu)
        nn = np.repeat(nrm[None, :], len(x), axis=0)
        tA = _clib.near_traction(x + shift, nn, pts, fs, zero)
        tB = _clib.near_traction(x, nn, pts, fs, zero)
        out += [np.concatenate([(uA - uB)[:, 0], (uA - uB)[:, 1]]),
                np.concatenate([(tA - tB)[:, 0], (tA - tB)[:, 1]])]
    return np.concatenate(out)


def wall_proxies(geom, M):
    """Proxy points on the walls of the dilated cell U~ (Sec. 6.1 remark: the expanded unit
    cell is the proxy surface): M / 4 points on each side of the parallelogram with corners
    c_U +- e1 +- e2, equispaced at the midpoints of M / 4 equal parameter intervals (the paper
    does not state the distribution along the walls), counter-clockwise from the bottom side."""
    if M % 4:
        raise ValueError("M must be a multiple of 4")
    k = M // 4
    t = -1.0 + (np.arange(k) + 0.5) * (2.0 / k)
    e1, e2, c = geom.e1, geom.e2, geom.cU
    sides = [c - e2 + t[:, None] * e1,          # bottom, left to right
             c + e1 + t[:, None] * e2,          # right, bottom to top
             c + e2 - t[:, None] * e1,          # top, right to left
             c - e1 - t[:, None] * e2]          # left, top to bottom
    return np.concatenate(sides)


def max_extent_ok(geom, close_factor=10.0):
    """Whether every particle is small enough for the U~ near set: its diameter plus the
    close-evaluation distance stays below lattice distance 1/2 in both lattice directions."""
    s = abs(geom.e2[0])
    for q in range(geom.No):
        sl = geom.particle_slice(q)
        h = geom.w[sl].sum() / geom.n_nodes[q]
        if (1.0 + s) * (2.0 * max(geom.a[q], geom.b[q]) + close_factor * h) >= 0.5:
            return False
    return True
