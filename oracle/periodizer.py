"""Periodizing correction by proxy Stokeslets (Sec. 4.2, Sec. 6.1, Sec. 6.2).

Four steps of Sec. 6.2 for point forces f_j at the nodes:

1. near sum (``near``);
2. the discrepancy g = [u_R - u_L; T_R - T_L; u_U - u_D; T_U - T_D] of the near
   field at m Gauss-Legendre points on the walls L and D;
3. the empty-box problem (Sec. 4.2, EBVP) with data g~ = g0 - g is solved by the
   method of fundamental solutions (Sec. 6.1): Q xi = g~ in the least-squares sense;
4. the correction field of the M proxy Stokeslets xi is added at the targets.

Walls (cell centre c_U): L(t) = c_U - e1/2 + t e2 and D(t) = c_U - e2/2 + t e1,
t in [-1/2, 1/2]; R = L + e1, U = D + e2. One normal per pair of opposite walls,
n_L = (e2_2, -e2_1)/|e2| (pointing along +e1) and n_D = (0, 1).

Step 2 uses the cancellation noted in Sec. 4.2 and Sec. 6.2: with the 3x3 image
set, the images that are near a wall appear on both sides of the jump and cancel,
so only images at least about one cell away are evaluated:

    u_near(x_L + e1) - u_near(x_L) = sum_j sum_{n=-1..1} [G(x_L, y_j - 2 e1 + n e2) - G(x_L, y_j + e1 + n e2)] f_j
    u_near(x_D + e2) - u_near(x_D) = sum_j sum_{m=-1..1} [G(x_D, y_j + m e1 - 2 e2) - G(x_D, y_j + m e1 + e2)] f_j

and the same with G^t(.; n) for the traction jumps.

Jump target (Sec. 4.2, the generalized periodic Green's function): with the
normals above the periodic field's traction jumps are -F/(2|e2|) across L/R and
-F/(2|e1|) across D/U, F = sum_j f_j: the cell's fluid balances the net force F,
so the flux of traction out of the cell is -F. This fixes the sign of
g0 = [0; -F/(2|e2|); 0; -F/(2|e1|)]; with it the data g0 - g satisfies the
consistency conditions (eqs. gforce, gvol), which the tests check.

Ordering: g and the rows of Q are [g1 comp 1 (m), g1 comp 2 (m), g2 (2m), g3 (2m), g4 (2m)];
xi is [xi_1 (M), xi_2 (M)] (all first components, then all second components).
Proxies: y_p = c_U + R (cos 2 pi p / M, sin 2 pi p / M).

Least squares. The empty-box problem is unique only up to a constant velocity
and a constant pressure (Theorem EBVP, nullity 3). On the discrete side these
three modes are the three smallest singular values of Q; their size depends on
the lattice skew (about 1e-10 relative for a square cell, up to about 1e-7 for
skew near 1/2), so a fixed relative cutoff cannot separate them reliably. The
pseudo-inverse therefore keeps the 2M - 3 largest singular triplets (and drops
anything below rcond relative), which removes exactly the gauge modes: they
carry no traction after the pressure pin and no velocity after the gauge
difference of the readout.
"""
from __future__ import annotations

import numpy as np

from . import _clib
from .kernels import stokeslet_apply, traction_apply, vorticity_apply


def gauss_legendre(m):
    return np.polynomial.legendre.leggauss(m)


def walls(geom, m):
    t, wt = gauss_legendre(m)
    t = 0.5 * t
    xL = geom.cU - 0.5 * geom.e1 + t[:, None] * geom.e2
    xD = geom.cU - 0.5 * geom.e2 + t[:, None] * geom.e1
    wL = 0.5 * wt * np.linalg.norm(geom.e2)
    wD = 0.5 * wt * np.linalg.norm(geom.e1)
    nL = np.array([geom.e2[1], -geom.e2[0]]) / np.linalg.norm(geom.e2)
    nD = np.array([0.0, 1.0])
    return {"xL": xL, "xD": xD, "wL": wL, "wD": wD, "nL": nL, "nD": nD, "m": m}


def proxies(geom, M, R):
    th = 2.0 * np.pi * np.arange(M) / M
    return geom.cU + R * np.stack([np.cos(th), np.sin(th)], axis=1)


def build_Q(geom, W, P, mu):
    m, M = W["m"], len(P)
    Q = np.zeros((8 * m, 2 * M))
    for comp in range(2):
        e = np.zeros((1, 1, 2))
        e[..., comp] = 1.0
        blocks = []
        for (x, shift, nrm) in ((W["xL"], geom.e1, W["nL"]), (W["xD"], geom.e2, W["nD"])):
            rA = (x + shift)[:, None, :] - P[None, :, :]
            rB = x[:, None, :] - P[None, :, :]
            du = stokeslet_apply(rA, e, mu) - stokeslet_apply(rB, e, mu)          # (m, M, 2)
            dt = traction_apply(rA, nrm[None, None, :], e) - traction_apply(rB, nrm[None, None, :], e)
            blocks += [du, dt]
        rows = np.concatenate([np.concatenate([b[..., 0], b[..., 1]], axis=0) for b in blocks], axis=0)
        Q[:, comp * M:(comp + 1) * M] = rows
    return Q


def pinv_gauge_truncated(Q, rcond=1e-14, n_gauge=3):
    U, s, Vt = np.linalg.svd(Q, full_matrices=False)
    keep = np.arange(len(s)) < len(s) - n_gauge
    keep &= s > rcond * s[0]
    inv = np.where(keep, 1.0 / np.where(keep, s, 1.0), 0.0)
    return (Vt.T * inv[None, :]) @ U.T


def consistency_W(geom, W):
    """Left null vectors of Q: net traction flux (2 rows) and net volume flux (1 row)."""
    m = W["m"]
    out = np.zeros((3, 8 * m))
    # blocks: g1c1 g1c2 g2c1 g2c2 g3c1 g3c2 g4c1 g4c2, each of length m
    def blk(k):
        return slice(k * m, (k + 1) * m)
    out[0, blk(2)] = W["wL"]
    out[0, blk(6)] = W["wD"]
    out[1, blk(3)] = W["wL"]
    out[1, blk(7)] = W["wD"]
    out[2, blk(0)] = W["wL"] * W["nL"][0]
    out[2, blk(1)] = W["wL"] * W["nL"][1]
    out[2, blk(4)] = W["wD"] * W["nD"][0]
    out[2, blk(5)] = W["wD"] * W["nD"][1]
    return out


def _flat(v):
    return np.concatenate([v[:, 0], v[:, 1]])


def discrepancy(geom, W, f, mu, rng=1):
    """g of step 2 (telescoped), for point forces f (N, 2) at the nodes.

    With images m, n in [-rng, rng], u_near(x_L + e1) - u_near(x_L) keeps only the
    column m = -rng-1 (from the shifted target) minus the column m = rng."""
    e1, e2 = geom.e1, geom.e2
    ks = np.arange(-rng, rng + 1, dtype=float)
    # G(x, y + s) = G(x - s, y): the C routine shifts the targets by -s, so pass s
    sL_far = np.array([-(rng + 1) * e1 + k * e2 for k in ks])
    sL_near = np.array([rng * e1 + k * e2 for k in ks])
    sD_far = np.array([k * e1 - (rng + 1) * e2 for k in ks])
    sD_near = np.array([k * e1 + rng * e2 for k in ks])
    y = geom.x
    out = []
    for (x, nrm, far, near) in ((W["xL"], W["nL"], sL_far, sL_near), (W["xD"], W["nD"], sD_far, sD_near)):
        uf, _ = _clib.stokeslet_velocity(x, y, f, far, mu)
        un, _ = _clib.stokeslet_velocity(x, y, f, near, mu)
        nn = np.repeat(nrm[None, :], len(x), axis=0)
        tf = _clib.near_traction(x, nn, y, f, far)
        tn = _clib.near_traction(x, nn, y, f, near)
        out += [_flat(uf - un), _flat(tf - tn)]
    return np.concatenate(out)


def g0_vector(geom, W, F):
    m = W["m"]
    g0 = np.zeros(8 * m)
    l2, l1 = np.linalg.norm(geom.e2), np.linalg.norm(geom.e1)
    g0[2 * m:3 * m] = -F[0] / (2 * l2)
    g0[3 * m:4 * m] = -F[1] / (2 * l2)
    g0[6 * m:7 * m] = -F[0] / (2 * l1)
    g0[7 * m:8 * m] = -F[1] / (2 * l1)
    return g0


def xi_to_forces(xi):
    M = len(xi) // 2
    return np.stack([xi[:M], xi[M:]], axis=1)


def correction_traction(P, xi, xt, nt):
    fx = xi_to_forces(xi)
    r = xt[:, None, :] - P[None, :, :]
    return traction_apply(r, nt[:, None, :], fx[None]).sum(1)


def correction_velocity(P, xi, xt, mu):
    fx = xi_to_forces(xi)
    r = xt[:, None, :] - P[None, :, :]
    return stokeslet_apply(r, fx[None], mu).sum(1)


def correction_vorticity(P, xi, xt, mu):
    fx = xi_to_forces(xi)
    r = xt[:, None, :] - P[None, :, :]
    return vorticity_apply(r, fx[None], mu).sum(1)


def proxy_data_extended(geom, W, f, mu, rng=1):
    """g0 - g (steps 2 and 3) in extended precision (numpy longdouble: a 64-bit significand
    on x86-64), from the same telescoped sums as `discrepancy` and `g0_vector`.

    Test reference for the rounding of an FP64 evaluation: g is small against the sum of
    its terms' sizes, and the least-squares step amplifies its rounding by |Q+| (about
    1e6), so the accuracy of xi is set by how g and F are summed."""
    LD = np.longdouble
    pi = 4 * np.arctan(LD(1))
    e1, e2 = geom.e1.astype(LD), geom.e2.astype(LD)
    y = geom.x.astype(LD)
    fl = np.asarray(f).astype(LD)
    ks = [LD(k) for k in range(-rng, rng + 1)]

    def field(x, nrm, shifts):
        u = np.zeros((len(x), 2), LD)
        t = np.zeros((len(x), 2), LD)
        for s in shifts:
            r = x[:, None, :] - (y[None, :, :] + s)
            rr = (r * r).sum(-1)
            rf = (r * fl[None]).sum(-1)
            rn = (r * nrm[None, None, :]).sum(-1)
            u += ((-LD(0.5) * np.log(rr))[..., None] * fl[None] + r * (rf / rr)[..., None]).sum(1)
            t += (r * (rn * rf / (rr * rr))[..., None]).sum(1)
        return u / (4 * pi * LD(mu)), -t / pi

    out = []
    for (x, nrm, far, near) in ((W["xL"], W["nL"], [-(rng + 1) * e1 + k * e2 for k in ks],
                                 [rng * e1 + k * e2 for k in ks]),
                                (W["xD"], W["nD"], [k * e1 - (rng + 1) * e2 for k in ks],
                                 [k * e1 + rng * e2 for k in ks])):
        xl, nl = x.astype(LD), nrm.astype(LD)
        uf, tf = field(xl, nl, far)
        un, tn = field(xl, nl, near)
        du, dt = uf - un, tf - tn
        out += [du[:, 0], du[:, 1], dt[:, 0], dt[:, 1]]
    g = np.concatenate(out)
    F = fl.sum(0)
    m = W["m"]
    g0 = np.zeros(8 * m, LD)
    l2 = np.sqrt((e2 * e2).sum())
    l1 = np.sqrt((e1 * e1).sum())
    g0[2 * m:3 * m] = -F[0] / (2 * l2)
    g0[3 * m:4 * m] = -F[1] / (2 * l2)
    g0[6 * m:7 * m] = -F[0] / (2 * l1)
    g0[7 * m:8 * m] = -F[1] / (2 * l1)
    return g0 - g
