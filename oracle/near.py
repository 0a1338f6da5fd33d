"""Near-image traction sum and self term (Sec. 4.2 Def. G_near; Sec. 6 Nystrom).

The near part of the periodic single-layer traction at every node x_i:

    T_near(x_i) = sum_j sum_{s in S9} G^t(x_i, y_j + s; n_i) f_j,   f_j = w_j sigma_j,

with S9 = {m e1 + n e2 : m, n in {-1, 0, 1}} applied to every particle (centres
wrapped into the cell) and only the pair (j = i, s = 0) skipped. The skipped
diagonal of the smooth kernel is replaced by its limit along the curve,

    lim_{y -> x on Gamma} G^t(x, y; n_x) = -(kappa / (2 pi)) tau tau^T,

which follows from expanding r = x - y to second order in arclength (the paper
only states that the kernel is smooth, Sec. 6).
"""
from __future__ import annotations

import numpy as np

from . import _clib
from .kernels import traction_apply


def forces(geom, sigma2):
    """f_j = w_j sigma_j, sigma2 of shape (N, 2)."""
    return geom.w[:, None] * sigma2


def near_traction(geom, sigma2, rng=1):
    f = forces(geom, sigma2)
    return _clib.near_traction(geom.x, geom.n, geom.x, f, geom.shifts(rng), np.arange(geom.N))


def near_traction_bruteforce(geom, sigma2, rng=1):
    """Pure-Python loops over targets (small N only): the same sum, written out."""
    f = forces(geom, sigma2)
    out = np.zeros((geom.N, 2))
    sh = geom.shifts(rng)
    for i in range(geom.N):
        acc = np.zeros(2)
        for s in sh:
            r = geom.x[i] - (geom.x + s)
            if not np.any(s):
                r = np.delete(r, i, axis=0)
                ff = np.delete(f, i, axis=0)
            else:
                ff = f
            acc += traction_apply(r, geom.n[i][None, :], ff).sum(0)
        out[i] = acc
    return out


def self_term(geom, sigma2):
    f = forces(geom, sigma2)
    tf = (geom.tau * f).sum(1)
    return -(geom.kappa / (2.0 * np.pi) * tf)[:, None] * geom.tau
