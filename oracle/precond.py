"""Block preconditioner of the completed BIE: the isolated-body self blocks (test infrastructure).

For particle q alone in free space, the completed operator of Sec. 5 (eq. BIEPerturbed)
restricted to its own curve is

    B_q sigma = sigma/2 + K_qq sigma + L_q sigma,

with K_qq the free-space traction single layer of the curve on itself (the Nystrom
sum over the other nodes of the curve plus the smooth diagonal limit
-(kappa/2pi) tau tau^T w, Sec. 6) and L_q the rigid-mode completion (net force plus
torque). Neither the pressure pin nor the other particles, images or proxies enter.

The traction kernel rotates with the curve, so the block of an ellipse at angle theta
is R(theta) B_body R(theta)^T node by node, with B_body the block of the same ellipse
at angle 0 centred at the origin. The preconditioner is blockdiag(B_q)^{-1}, applied
on the right: GMRES then solves A P^{-1} u = b and sigma = P^{-1} u, which changes the
iteration count but not the solution.

Layout of a block: unknowns ordered [sigma_1(0..n-1), sigma_2(0..n-1)], rows likewise.
"""
from __future__ import annotations

import numpy as np

from . import geometry
from .kernels import traction_matrix


def body_nodes(a, b, n, kind=0, params=None):
    """Nodes of the curve in its body frame (angle 0, reference point at the origin),
    t_k = 2 pi k / n, with the geometry of the periodic trapezoid rule (Sec. 6): the
    ellipse (a cos t, b sin t), or the star of the given params."""
    p = np.array([a, b, 0.0, 0.0]) if params is None else np.asarray(params, float)
    x, xp, tau, nrm, w, kap = geometry.particle_nodes(np.zeros(2), 0.0, kind, p, n)
    return x, tau, nrm, w, kap


def self_block(a, b, n, complete=True, kind=0, params=None):
    """B_body (2n x 2n) of the ellipse with semi-axes a, b (or of the given shape) and n
    nodes (without the completion L when complete is False)."""
    x, tau, nrm, w, kap = body_nodes(a, b, n, kind, params)
    B = np.zeros((2 * n, 2 * n))
    for i in range(n):
        r = x[i] - x
        r[i] = (1.0, 0.0)  # placeholder, overwritten by the diagonal limit below
        blocks = traction_matrix(r, nrm[i][None, :]) * w[:, None, None]   # (n, 2, 2): [j, c, d]
        blocks[i] = -(kap[i] / (2.0 * np.pi)) * np.outer(tau[i], tau[i]) * w[i]
        for c in range(2):
            for d in range(2):
                B[c * n + i, d * n:(d + 1) * n] = blocks[:, c, d]
    B += 0.5 * np.eye(2 * n)
    if not complete:
        return B
    perp = np.stack([-x[:, 1], x[:, 0]], axis=1)   # (x - c)^perp
    for c in range(2):
        B[c * n:(c + 1) * n, c * n:(c + 1) * n] += w[None, :]                 # net force
        for d in range(2):
            B[c * n:(c + 1) * n, d * n:(d + 1) * n] += np.outer(perp[:, c], w * perp[:, d])   # torque
    return B


def apply_inverse(geom, v):
    """P^{-1} v for the SoA vector v [2N]: per particle rotate into the body frame,
    solve with B_body (LAPACK LU), rotate back."""
    N = geom.N
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros(2 * N)
    cache = {}
    for q in range(geom.No):
        sl = geom.particle_slice(q)
        n = int(geom.n_nodes[q])
        kind = 0 if geom.kind is None else int(geom.kind[q])
        prm = np.array([geom.a[q], geom.b[q], 0.0, 0.0]) if geom.params is None else geom.params[q]
        key = (kind, tuple(float(v) for v in prm), n)
        if key not in cache:
            cache[key] = self_block(0.0, 0.0, n, kind=kind, params=prm)
        c, s = np.cos(geom.theta[q]), np.sin(geom.theta[q])
        v1, v2 = v[:N][sl], v[N:][sl]
        rhs = np.concatenate([c * v1 + s * v2, -s * v1 + c * v2])
        u = np.linalg.solve(cache[key], rhs)
        out[:N][sl] = c * u[:n] - s * u[n:]
        out[N:][sl] = s * u[:n] + c * u[n:]
    return out
