"""Free-space Stokes kernels in 2-D (Sec. 4.1), FP64, vectorised over pairs.

With r = x - y and rho = |r|:

* Stokeslet (eq. Gv):      G(x,y)   = 1/(4 pi mu) (log(1/rho) I + r r^T / rho^2)
* pressure (eq. Gp):       G^p(x,y) = r / (2 pi rho^2)
* traction (eq. Gt):       G^t(x,y;n) = -(1/pi) r r^T (r . n) / rho^4, n the normal at the target x
* vorticity of G f (derived from eq. Gv): d1 u2 - d2 u1 = -(r1 f2 - r2 f1) / (2 pi mu rho^2)

Arrays: r has shape (..., 2); forces/normals broadcast against it.
"""
from __future__ import annotations

import numpy as np


def stokeslet_apply(r, f, mu):
    """G(x,y) f for r = x - y; returns (..., 2)."""
    rr = (r * r).sum(-1)
    rf = (r * f).sum(-1)
    lg = -0.5 * np.log(rr)
    return (lg[..., None] * f + r * (rf / rr)[..., None]) / (4.0 * np.pi * mu)


def stokeslet_matrix(r, mu):
    """G(x,y) as (..., 2, 2)."""
    rr = (r * r).sum(-1)
    lg = -0.5 * np.log(rr)
    out = r[..., :, None] * r[..., None, :] / rr[..., None, None]
    out[..., 0, 0] += lg
    out[..., 1, 1] += lg
    return out / (4.0 * np.pi * mu)


def pressure_apply(r, f):
    """G^p(x,y) . f."""
    rr = (r * r).sum(-1)
    return (r * f).sum(-1) / (2.0 * np.pi * rr)


def traction_apply(r, n, f):
    """G^t(x,y;n) f = -(1/pi) r (r.n)(r.f) / rho^4."""
    rr = (r * r).sum(-1)
    rn = (r * n).sum(-1)
    rf = (r * f).sum(-1)
    return r * (-(rn * rf) / (np.pi * rr * rr))[..., None]


def traction_matrix(r, n):
    """G^t(x,y;n) as (..., 2, 2)."""
    rr = (r * r).sum(-1)
    rn = (r * n).sum(-1)
    return -(r[..., :, None] * r[..., None, :]) * (rn / (np.pi * rr * rr))[..., None, None]


def vorticity_apply(r, f, mu):
    """Vorticity (d1 u2 - d2 u1) of the Stokeslet field G f."""
    rr = (r * r).sum(-1)
    return -(r[..., 0] * f[..., 1] - r[..., 1] * f[..., 0]) / (2.0 * np.pi * mu * rr)
