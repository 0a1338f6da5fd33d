"""Completed, periodized boundary integral operator, RHS, dense LU and GMRES.

Second-kind BIE (Sec. 5, eq. BIEPerturbed, Nystrom form eq. BIEdiscretized):

    (1/2 I + K + L) sigma = -T(u0, p0),   T(u0, p0) = mu gamma (n_2, n_1)   (Sec. 3, u0 = (gamma x_2, 0))

K sigma = T_near + self + close correction + T_corr (Sec. 6.2 eq. Stsplit).
Pressure pin (Sec. 6.2, remark on GMRES stagnation): K sigma <- K sigma - ((K sigma)(x0) . n0) n,
with x0 the first node of the first particle; applied to K only. It leaves the
rigid-mode integrals unchanged because the integrals of n and (x - c)^perp . n
over a closed curve vanish.
Completion (Sec. 5, operator L_i):
    L_i sigma (x) = sum_k w_k sigma_k + (x - c_i)^perp sum_k w_k ((x_k - c_i)^perp . sigma_k),
x^perp = (-x_2, x_1).

GMRES: modified Gram-Schmidt Arnoldi, Givens rotations, x0 = 0 unless given, no
restart, stops when the relative residual estimate drops below tol.
Densities at this interface are SoA vectors [sigma_1(0..N-1), sigma_2(0..N-1)].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import close, dilated, near, periodizer
from .geometry import Geometry, build_geometry


@dataclass
class Config:
    mu: float = 1.0
    gamma: float = 1.0
    M: int = 32
    R: float = 1.5
    m: int = 24
    close_factor: float = 10.0
    rcond: float = 1e-14
    image_range: int = 1
    near_set: str = "3x3"   # "3x3": 3x3 images of whole particles; "dilated": the U~ set of Sec. 4.2
    proxy_surface: str = "circle"   # "circle": M proxies on a circle of radius R; "walls": on U~'s walls


@dataclass
class Problem:
    geom: Geometry
    cfg: Config
    W: dict
    P: np.ndarray
    Q: np.ndarray
    Qpinv: np.ndarray
    pairs: np.ndarray
    stats: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.geom.N


def make_problem(wl, **kw) -> Problem:
    cfg = Config(**{**{"mu": wl.get("mu", 1.0), "gamma": wl.get("gamma", 1.0)}, **kw})
    g = build_geometry(wl)
    if cfg.near_set not in ("3x3", "dilated"):
        raise ValueError(cfg.near_set)
    if cfg.near_set == "dilated" and not dilated.max_extent_ok(g, cfg.close_factor):
        raise ValueError("particles too large for the dilated-cell near set")
    W = periodizer.walls(g, cfg.m)
    if cfg.proxy_surface not in ("circle", "walls"):
        raise ValueError(cfg.proxy_surface)
    P = periodizer.proxies(g, cfg.M, cfg.R) if cfg.proxy_surface == "circle" else dilated.wall_proxies(g, cfg.M)
    Q = periodizer.build_Q(g, W, P, cfg.mu)
    Qp = periodizer.pinv_gauge_truncated(Q, cfg.rcond)
    pairs = close.close_pairs(g, cfg.close_factor, cfg.image_range) if cfg.close_factor > 0 else \
        np.zeros((0, 3), dtype=np.int64)
    return Problem(g, cfg, W, P, Q, Qp, pairs)


def to2(sigma):
    N = len(sigma) // 2
    return np.stack([sigma[:N], sigma[N:]], axis=1)


def to1(v2):
    return np.concatenate([v2[:, 0], v2[:, 1]])


def proxy_strengths(prob, sigma2):
    """xi = Q^+ (g0 - g) for the point forces f = w sigma (Sec. 6.2 step 3)."""
    g = prob.geom
    f = near.forces(g, sigma2)
    F = f.sum(0)
    if prob.cfg.near_set == "dilated":
        d = dilated.discrepancy(g, prob.W, f, prob.cfg.mu)
    else:
        d = periodizer.discrepancy(g, prob.W, f, prob.cfg.mu, prob.cfg.image_range)
    return prob.Qpinv @ (periodizer.g0_vector(g, prob.W, F) - d), d, F


def targets(prob):
    """Where the periodic sums are evaluated for each node: the node itself (3x3 set) or
    the node wrapped into the cell (U~ set, whose near sum holds for targets in U)."""
    return dilated.wrap_nodes(prob.geom) if prob.cfg.near_set == "dilated" else prob.geom.x


def apply_K(prob, sigma2, parts=False):
    """Unpinned K sigma as (N, 2) (and its pieces if parts)."""
    g = prob.geom
    if prob.cfg.near_set == "dilated":
        Tn = dilated.near_traction_fast(g, sigma2)
    else:
        Tn = near.near_traction(g, sigma2, prob.cfg.image_range)
    Ts = near.self_term(g, sigma2)
    dT = close.close_correction(g, sigma2, prob.pairs, prob.cfg.image_range)
    xi, d, F = proxy_strengths(prob, sigma2)
    Tc = periodizer.correction_traction(prob.P, xi, targets(prob), g.n)
    K = Tn + Ts + dT + Tc
    if parts:
        return K, {"near": Tn, "self": Ts, "close": dT, "corr": Tc, "xi": xi, "g": d, "F": F}
    return K


def pin(prob, K):
    g = prob.geom
    alpha = -(K[0] * g.n[0]).sum()
    return K + alpha * g.n


def apply_L(prob, sigma2):
    g = prob.geom
    out = np.zeros_like(sigma2)
    for i in range(g.No):
        sl = g.particle_slice(i)
        w = g.w[sl]
        rel = g.x[sl] - g.centers[i]
        perp = np.stack([-rel[:, 1], rel[:, 0]], axis=1)
        F = (w[:, None] * sigma2[sl]).sum(0)
        tq = (w * (perp * sigma2[sl]).sum(1)).sum()
        out[sl] = F[None, :] + perp * tq
    return out


def apply(prob, sigma):
    """y = (1/2 I + K_pinned + L) sigma, SoA in and out."""
    s2 = to2(np.asarray(sigma, dtype=np.float64))
    y = 0.5 * s2 + pin(prob, apply_K(prob, s2)) + apply_L(prob, s2)
    return to1(y)


def rhs(prob):
    g = prob.geom
    c = -prob.cfg.mu * prob.cfg.gamma
    return to1(np.stack([c * g.n[:, 1], c * g.n[:, 0]], axis=1))


def dense_matrix(prob):
    n2 = 2 * prob.N
    A = np.zeros((n2, n2))
    e = np.zeros(n2)
    for k in range(n2):
        e[k] = 1.0
        A[:, k] = apply(prob, e)
        e[k] = 0.0
    return A


def gmres(matvec, b, tol=1e-10, maxiter=500, x0=None):
    """Plain GMRES (MGS Arnoldi + Givens), no restart. Returns x, info dict."""
    n = len(b)
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    r0 = b - matvec(x0) if np.any(x0) else b.copy()
    bnorm = np.linalg.norm(b)
    beta = np.linalg.norm(r0)
    if beta <= tol * bnorm:
        return x0, {"iterations": 0, "rel_residual": beta / bnorm, "history": [beta / bnorm]}
    V = np.zeros((maxiter + 1, n))
    H = np.zeros((maxiter + 1, maxiter))
    cs = np.zeros(maxiter)
    sn = np.zeros(maxiter)
    gvec = np.zeros(maxiter + 1)
    gvec[0] = beta
    V[0] = r0 / beta
    hist = [beta / bnorm]
    k = 0
    for j in range(maxiter):
        w = matvec(V[j])
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        rr = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / rr, H[j + 1, j] / rr
        H[j, j] = rr
        H[j + 1, j] = 0.0
        gvec[j + 1] = -sn[j] * gvec[j]
        gvec[j] = cs[j] * gvec[j]
        k = j + 1
        hist.append(abs(gvec[j + 1]) / bnorm)
        if abs(gvec[j + 1]) <= tol * bnorm:
            break
    y = np.linalg.solve(np.triu(H[:k, :k]), gvec[:k])
    x = x0 + V[:k].T @ y
    return x, {"iterations": k, "rel_residual": hist[-1], "history": hist}


def solve(prob, tol=1e-10, maxiter=500, method="gmres", x0=None):
    b = rhs(prob)
    if method == "lu":
        import scipy.linalg as sla
        A = dense_matrix(prob)
        x = sla.lu_solve(sla.lu_factor(A), b)
        return x, {"iterations": 0, "rel_residual": np.linalg.norm(b - A @ x) / np.linalg.norm(b)}
    return gmres(lambda v: apply(prob, v), b, tol, maxiter, x0)


def apply_rows(prob, sigma, rows):
    """Rows `rows` (node indices) of y = (1/2 I + K_pinned + L) sigma, without forming
    the whole product: the same sums evaluated at the selected targets only (the pin
    needs node 0, which is always evaluated). Returns (len(rows), 2). 3x3 near set only."""
    if prob.cfg.near_set != "3x3":
        raise ValueError("apply_rows evaluates the 3x3 near set only")
    g = prob.geom
    s2 = to2(np.asarray(sigma, dtype=np.float64))
    rows = np.asarray(rows, dtype=np.int64)
    tgt = np.unique(np.concatenate([[0], rows]))
    f = near.forces(g, s2)
    from . import _clib
    Tn = _clib.near_traction(g.x[tgt], g.n[tgt], g.x, f, g.shifts(prob.cfg.image_range), tgt)
    tf = (g.tau[tgt] * f[tgt]).sum(1)
    Ts = -(g.kappa[tgt] / (2.0 * np.pi) * tf)[:, None] * g.tau[tgt]
    xi, _, _ = proxy_strengths(prob, s2)
    Tc = periodizer.correction_traction(prob.P, xi, g.x[tgt], g.n[tgt])
    sel = prob.pairs[np.isin(prob.pairs[:, 0], tgt)]
    dT_full = close.close_correction(g, s2, sel, prob.cfg.image_range)
    K = Tn + Ts + Tc + dT_full[tgt]
    alpha = -(K[0] * g.n[0]).sum()
    K = K + alpha * g.n[tgt]
    L = apply_L(prob, s2)[tgt]
    y = 0.5 * s2[tgt] + K + L
    pos = np.searchsorted(tgt, rows)
    return y[pos]
