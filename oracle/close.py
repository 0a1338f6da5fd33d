"""Close evaluation of the single-layer traction by barycentric Cauchy quadrature
(Sec. 6.3), written for targets in the exterior of a source curve.

Sec. 6.3 writes the Stokes single-layer potential through Laplace single-layer
potentials S_L[f] = (1/2pi) int log(1/|x-y|) f ds. With the origin at the curve
centre c, sigma~ = (y - c) . sigma and mu = 1 (the traction does not depend on mu),
differentiating the velocity identity of Sec. 6.3 gives the traction

    T = H[sigma~] n - (x-c)_1 H[sigma_1] n - (x-c)_2 H[sigma_2] n
        + (d1 S_L[sigma_1] + d2 S_L[sigma_2]) n,                       (*)

where H[f] is the Hessian of S_L[f] and the last term is -p n. (*) is the overall
negative of the decomposition printed in Sec. 6.3; (*) agrees with eq. (Gt),
which the tests check at far targets.

Laplace derivatives from Cauchy integrals. With z = x1 + i x2, phi = f conj(tau)
and v(z) = (1/2 pi i) int phi(zeta)/(zeta - z) dzeta, the analytic function
A = i v satisfies A = d1 S_L[f] - i d2 S_L[f] and A' = d11 S_L - i d12 S_L.

Exterior barycentric rule (globally compensated; the exterior counterpart of
the Helsing-Ojala interior rule). With nodes y_k, W_k = y'_k / (i N) and
boundary values v+ (the exterior limit of v on the curve):

    den = -1 + sum_k W_k/(y_k - z)
    v   = sum_k v+_k W_k/(y_k - z) / den
    v'  = sum_k (v+_k - v) W_k/(y_k - z)^2 / den

since v vanishes at infinity and (1/2 pi i) int 1/(zeta - z) dzeta = 0 outside.
Boundary values: v+_j = (1/2 pi i) int (phi - phi_j)/(zeta - y_j) dzeta by Plemelj,
discretised by the trapezoid rule with the diagonal limit phi'_j / (i N) (phi'
the spectral derivative in t with the Nyquist mode zeroed).

Close pairs (Sec. 6.3 remark on the 10 h precompute split): a target x_i on
particle p and a source image Gamma_q + s, (q, s) != (p, 0), are close when
min_k |x_i - (y_k + s)| < factor * h_q, h_q = |Gamma_q| / N_q. For each close
pair the correction is T_bary minus the plain trapezoid sum over that image,
which the near sum already added.
"""
from __future__ import annotations

import numpy as np

from .kernels import traction_apply


def spectral_derivative(phi):
    N = len(phi)
    k = np.fft.fftfreq(N, d=1.0 / N)
    if N % 2 == 0:
        k[N // 2] = 0.0
    return np.fft.ifft(1j * k * np.fft.fft(phi))


def boundary_values(y, yp, phi):
    """v+ at the nodes; y, yp, phi complex (Nq,)."""
    N = len(y)
    W = yp / (1j * N)
    diff = y[None, :] - y[:, None]          # [j, k] = y_k - y_j
    np.fill_diagonal(diff, 1.0)
    terms = (phi[None, :] - phi[:, None]) * W[None, :] / diff
    np.fill_diagonal(terms, 0.0)
    return terms.sum(1) + spectral_derivative(phi) / (1j * N)


def barycentric(z, y, yp, vplus):
    """v and v' at exterior targets z (nt,) for densities vplus (nd, Nq)."""
    N = len(y)
    W = yp / (1j * N)
    d = y[None, :] - z[:, None]              # (nt, Nq)
    u = W[None, :] / d
    den = -1.0 + u.sum(1)
    v = (vplus[:, None, :] * u[None]).sum(-1) / den[None]
    vp = ((vplus[:, None, :] - v[:, :, None]) * (u / d)[None]).sum(-1) / den[None]
    return v, vp


def curve_data(geom, q):
    sl = geom.particle_slice(q)
    y = geom.x[sl, 0] + 1j * geom.x[sl, 1]
    yp = geom.xp[sl, 0] + 1j * geom.xp[sl, 1]
    tau = geom.tau[sl, 0] + 1j * geom.tau[sl, 1]
    return sl, y, yp, tau


def curve_vplus(geom, q, sigma2):
    """v+ of the three densities sigma_1, sigma_2, (y - c).sigma on curve q, (3, Nq)."""
    sl, y, yp, tau = curve_data(geom, q)
    s = sigma2[sl]
    rel = geom.x[sl] - geom.centers[q]
    dens = [s[:, 0], s[:, 1], (rel * s).sum(1)]
    return np.array([boundary_values(y, yp, f * np.conj(tau)) for f in dens])


def traction_bary(geom, q, vplus, xt, nt):
    """Single-layer traction at targets xt (nt,2) with normals nt from curve q (unshifted)."""
    sl, y, yp, tau = curve_data(geom, q)
    z = xt[:, 0] + 1j * xt[:, 1]
    v, vp = barycentric(z, y, yp, vplus)
    A, Ap = 1j * v, 1j * vp                   # (3, nt)
    g1 = np.real(A)                           # d1 S_L[f]
    g2 = -np.imag(A)                          # d2 S_L[f]
    h11, h12 = np.real(Ap), -np.imag(Ap)      # Hessian entries; h22 = -h11

    def hess_n(k):
        return np.stack([h11[k] * nt[:, 0] + h12[k] * nt[:, 1],
                         h12[k] * nt[:, 0] - h11[k] * nt[:, 1]], axis=1)

    rel = xt - geom.centers[q]
    T = hess_n(2) - rel[:, :1] * hess_n(0) - rel[:, 1:2] * hess_n(1)
    T += (g1[0] + g2[1])[:, None] * nt
    return T


def plain_traction(geom, q, sigma2, xt, nt):
    sl = geom.particle_slice(q)
    f = geom.w[sl, None] * sigma2[sl]
    r = xt[:, None, :] - geom.x[sl][None, :, :]
    return traction_apply(r, nt[:, None, :], f[None]).sum(1)


def close_pairs(geom, factor=10.0, rng=1):
    """Sorted (target, q, shift index) triples; shift index into geom.shifts(rng)."""
    sh = geom.shifts(rng)
    zero = int(np.argmin((sh ** 2).sum(1)))
    out = []
    for q in range(geom.No):
        sl = geom.particle_slice(q)
        hq = geom.w[sl].sum() / geom.n_nodes[q]
        lim = factor * hq
        for si, s in enumerate(sh):
            cs = geom.centers[q] + s
            cand = np.nonzero(np.linalg.norm(geom.x - cs, axis=1) < geom.a[q] + lim)[0]
            if si == zero:
                cand = cand[geom.pid[cand] != q]
            if len(cand) == 0:
                continue
            d = np.linalg.norm(geom.x[cand][:, None, :] - (geom.x[sl] + s)[None], axis=2).min(1)
            for i in cand[d < lim]:
                out.append((int(i), q, si))
    out.sort()
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def close_correction(geom, sigma2, pairs, rng=1):
    """Delta T at every node (zeros away from close pairs)."""
    dT = np.zeros((geom.N, 2))
    if len(pairs) == 0:
        return dT
    sh = geom.shifts(rng)
    for q in np.unique(pairs[:, 1]):
        sel = pairs[pairs[:, 1] == q]
        vplus = curve_vplus(geom, q, sigma2)
        xt = geom.x[sel[:, 0]] - sh[sel[:, 2]]     # shift the target instead of the curve
        nt = geom.n[sel[:, 0]]
        corr = traction_bary(geom, q, vplus, xt, nt) - plain_traction(geom, q, sigma2, xt, nt)
        np.add.at(dT, sel[:, 0], corr)
    return dT
