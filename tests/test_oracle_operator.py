"""Pins of the oracle's operator, periodizer, close evaluation, solver and
readouts against identities, closed forms and limits fixed by the paper and by
Stokes theory (P2-P16 of the test plan)."""
import numpy as np
import pytest

import oracle
from oracle import close, geometry, near, periodizer, readout
from oracle import operator as op
from paper_1912_04501_amd import workloads as W


def smooth_density(geom, seed=0, K=5):
    """Band-limited random density on every curve (Fourier modes |k| <= K)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((geom.N, 2))
    for i in range(geom.No):
        sl = geom.particle_slice(i)
        t = 2 * np.pi * np.arange(geom.n_nodes[i]) / geom.n_nodes[i]
        for c in range(2):
            a = rng.standard_normal(K + 1)
            b = rng.standard_normal(K + 1)
            out[sl, c] = sum(a[k] * np.cos(k * t) + b[k] * np.sin(k * t) for k in range(K + 1))
    return out


def rigid_moments(geom, v2):
    """Per particle: sum_k w_k r.v for r = e1, e2, (x - c)^perp."""
    out = np.zeros((geom.No, 3))
    for i in range(geom.No):
        sl = geom.particle_slice(i)
        w = geom.w[sl]
        rel = geom.x[sl] - geom.centers[i]
        out[i, 0] = (w * v2[sl, 0]).sum()
        out[i, 1] = (w * v2[sl, 1]).sum()
        out[i, 2] = (w * (-rel[:, 1] * v2[sl, 0] + rel[:, 0] * v2[sl, 1])).sum()
    return out


def free_space_K(geom, s2, with_close=True):
    K = near.near_traction(geom, s2, rng=0) + near.self_term(geom, s2)
    if with_close:
        pairs = close.close_pairs(geom, 10.0, rng=0)
        K = K + close.close_correction(geom, s2, pairs, rng=0)
    return K


def test_interior_gauss_law_free_space_close_pair():
    """Lemma (jump relation) + interior Gauss law (Sec. 4.1): the interior traction
    1/2 sigma + K sigma has zero net force and torque on every body (P2). With a
    gap of 2e-3 the plain rule fails and the close correction restores it."""
    g = geometry.build_geometry(W.two_ellipses(2e-3, n_nodes=256))
    s2 = smooth_density(g)
    scale = np.abs(rigid_moments(g, np.abs(s2))).max()
    good = rigid_moments(g, 0.5 * s2 + free_space_K(g, s2, True))
    bad = rigid_moments(g, 0.5 * s2 + free_space_K(g, s2, False))
    assert np.abs(good).max() < 1e-10 * scale
    assert np.abs(bad).max() > 1e-4 * scale  # plain rule: 1.6e-3 at this gap


def test_normal_density_free_space_and_periodic():
    """S[n] == 0 outside the bodies and p = -1 inside, so K n = n/2 (Sec. 4.1);
    the periodic correction vanishes too because F = 0 and the near field is zero."""
    g = geometry.build_geometry(W.two_ellipses(1e-2, n_nodes=96))
    Kf = free_space_K(g, g.n, True)
    assert np.abs(Kf - 0.5 * g.n).max() < 1e-10
    prob = op.make_problem(W.two_ellipses(1e-2, n_nodes=96))
    Kp = op.apply_K(prob, g.n)
    assert np.abs(Kp - 0.5 * g.n).max() < 1e-8


def test_periodic_rigid_mode_identity():
    """The periodic correction carries no net force or torque (Sec. 4.2 lemma), and
    the pin adds a multiple of n: 1/2 sigma + K_pinned sigma still has zero rigid moments."""
    prob = op.make_problem(W.random_ellipses(4, 0.25, seed=11, nodes=96))
    g = prob.geom
    s2 = smooth_density(g, seed=2)
    K = op.pin(prob, op.apply_K(prob, s2))
    mom = rigid_moments(g, 0.5 * s2 + K)
    scale = np.abs(rigid_moments(g, np.abs(s2))).max()
    assert np.abs(mom).max() < 1e-8 * scale


def test_discrepancy_is_consistent():
    """Sec. 6.1/6.2 remark: W^T (g0 - g) = 0 (zero net force and zero net flux),
    even though W^T g alone is not zero when F != 0 (P11)."""
    prob = op.make_problem(W.random_ellipses(5, 0.3, seed=4, nodes=64, skew=0.3))
    g = prob.geom
    s2 = np.random.default_rng(5).standard_normal((g.N, 2))
    f = near.forces(g, s2)
    F = f.sum(0)
    d = periodizer.discrepancy(g, prob.W, f, prob.cfg.mu)
    Wt = periodizer.consistency_W(g, prob.W)
    dt = periodizer.g0_vector(g, prob.W, F) - d
    assert np.abs(Wt @ dt).max() < 1e-12 * np.abs(F).max()
    assert np.abs(Wt @ d).max() > 1e-3 * np.abs(F).max()
    # the same functionals annihilate Q (up to the MFS discretisation)
    assert np.abs(Wt @ prob.Q).max() < 1e-6 * np.abs(prob.Q).max()


def test_extended_proxy_data():
    """The extended-precision g0 - g (the test reference for the rounding of the FP64
    sums) equals the FP64 evaluation up to FP64 rounding, satisfies the consistency
    conditions W^T (g0 - g) = 0 far more tightly, and does not depend on the order of
    the sources."""
    prob = op.make_problem(W.random_ellipses(5, 0.3, seed=4, nodes=64, skew=0.3))
    g = prob.geom
    f = near.forces(g, 30.0 * np.random.default_rng(5).standard_normal((g.N, 2)))
    F = f.sum(0)
    v64 = periodizer.g0_vector(g, prob.W, F) - periodizer.discrepancy(g, prob.W, f, prob.cfg.mu)
    vx = periodizer.proxy_data_extended(g, prob.W, f, prob.cfg.mu)
    assert vx.dtype == np.longdouble
    assert np.abs(v64 - vx.astype(float)).max() < 1e-13 * np.abs(v64).max()
    Wt = periodizer.consistency_W(g, prob.W)
    assert float(np.abs(Wt.astype(np.longdouble) @ vx).max()) < 1e-15 * np.abs(F).max()
    perm = np.random.default_rng(1).permutation(g.N)

    class _Perm:
        e1, e2, x = g.e1, g.e2, g.x[perm]
    vp = periodizer.proxy_data_extended(_Perm, prob.W, f[perm], prob.cfg.mu)
    assert float(np.abs(vp - vx).max()) < 1e-16 * np.abs(v64).max()


class _Cell:
    def __init__(self, e2):
        self.e1 = np.array([1.0, 0.0])
        self.e2 = np.asarray(e2, float)
        self.cU = np.zeros(2)


@pytest.mark.parametrize("e2", [(0.0, 1.0), (np.cos(np.pi / 4), np.sin(np.pi / 4))])
def test_empty_box_known_solution(e2):
    """Sec. 6.1 Example 1 (P3): mu = 0.7, Stokeslet f0 = (0.3, -0.6) at
    y0 = 1.5 (cos .1, sin .1); jumps of the exact field on the walls are the EBVP
    data; the MFS solution matches on a 100 x 100 grid up to a constant, and the
    error falls geometrically with the number of proxies. y0 lies on the R = 1.5
    circle, so the proxies sit at R = 1.2 here (between the cell and y0).""" 
    mu = 0.7
    cell = _Cell(e2)
    y0 = 1.5 * np.array([np.cos(0.1), np.sin(0.1)])
    f0 = np.array([0.3, -0.6])
    from oracle.kernels import stokeslet_apply, traction_apply
    t = (np.arange(100) + 0.5) / 100 - 0.5
    grid = (t[:, None, None] * cell.e1 + t[None, :, None] * cell.e2).reshape(-1, 2)
    exact = stokeslet_apply(grid - y0, f0[None], mu)
    errs = []
    for M in (16, 32, 48):
        Wl = periodizer.walls(cell, 40)
        P = periodizer.proxies(cell, M, 1.2)
        Q = periodizer.build_Q(cell, Wl, P, mu)
        rows = []
        for (x, sh, nrm) in ((Wl["xL"], cell.e1, Wl["nL"]), (Wl["xD"], cell.e2, Wl["nD"])):
            du = stokeslet_apply(x + sh - y0, f0[None], mu) - stokeslet_apply(x - y0, f0[None], mu)
            dtr = traction_apply(x + sh - y0, nrm[None], f0[None]) - traction_apply(x - y0, nrm[None], f0[None])
            rows += [np.concatenate([du[:, 0], du[:, 1]]), np.concatenate([dtr[:, 0], dtr[:, 1]])]
        d = np.concatenate(rows)
        xi = periodizer.pinv_gauge_truncated(Q) @ d
        u = periodizer.correction_velocity(P, xi, grid, mu)
        e = (u - u[0]) - (exact - exact[0])
        errs.append(np.abs(e).max() / np.abs(exact).max())
    assert errs[2] < 2e-6
    assert errs[1] < 0.03 * errs[0] and errs[2] < 0.03 * errs[1]


def test_single_ellipse_symmetry_and_lu():
    """One centred ellipse in a square cell is point-symmetric: v = 0 and sigma is
    odd under t -> t + pi (P5); GMRES agrees with dense LU (P6)."""
    prob = op.make_problem(W.single_ellipse())
    x, info = op.solve(prob, tol=1e-12)
    xl, _ = op.solve(prob, method="lu")
    assert np.abs(x - xl).max() < 1e-10 * np.abs(xl).max()
    s2 = op.to2(xl)
    assert np.abs(s2[:64] + s2[64:]).max() < 1e-10 * np.abs(s2).max()
    v, om = readout.velocities(prob, xl)
    assert np.abs(v).max() < 1e-12


def test_dilute_disk_einstein_2d():
    """2-D dilute limit (P7): (mu_eff - 1)/phi -> 2 for a disk lattice; the residual
    falls with phi (about 2 - 1.2 phi at these sizes)."""
    slopes = []
    for rho in (0.02, 0.05):
        wl = W.single_ellipse(n_nodes=64, a=rho, b=rho)
        prob = op.make_problem(wl)
        x, _ = op.solve(prob, tol=1e-12)
        phi = np.pi * rho ** 2
        slopes.append((readout.mu_eff(prob, x) - 1.0) / phi)
        _, om = readout.velocities(prob, x)
        assert abs(om[0] + 0.5) < 1e-3        # a free disk spins with the fluid: omega = -gamma/2
    assert abs(slopes[0] - 2.0) < 5e-3
    assert abs(slopes[0] - 2.0) < abs(slopes[1] - 2.0)


def test_jeffery_rate_dilute():
    """Isolated ellipse in shear (P8): omega -> -gamma (a^2 sin^2 th + b^2 cos^2 th)/(a^2 + b^2)
    as the area fraction -> 0, with an O(phi) error."""
    th, ar = 0.6, 2.0
    errs = []
    for a in (0.1, 0.05):
        b = a / ar
        prob = op.make_problem(W.single_ellipse(n_nodes=96, a=a, b=b, theta=th))
        x, _ = op.solve(prob, tol=1e-12)
        _, om = readout.velocities(prob, x)
        jeff = -(a ** 2 * np.sin(th) ** 2 + b ** 2 * np.cos(th) ** 2) / (a ** 2 + b ** 2)
        errs.append(abs(om[0] - jeff))
    assert errs[1] < 2e-3
    assert errs[1] < 0.5 * errs[0]


def _fine_plain_traction(a, b, th, c, coeffs, N_fine, xt, nt):
    """Plain trapezoid sum on a much finer discretisation of the same curve, with the
    band-limited density evaluated exactly at the fine nodes."""
    x, xp, tau, n, w, kappa = geometry.ellipse_nodes(c, th, a, b, N_fine)
    t = 2 * np.pi * np.arange(N_fine) / N_fine
    sig = np.stack([sum(cf[k] * np.cos(k * t) + cf[k + 6] * np.sin(k * t) for k in range(6)) for cf in coeffs], 1)
    from oracle.kernels import traction_apply
    r = xt[:, None, :] - x[None]
    return traction_apply(r, nt[:, None, :], (w[:, None] * sig)[None]).sum(1)


@pytest.mark.parametrize("gap", [0.3, 1e-2, 1e-3])
def test_close_evaluation_accuracy(gap):
    """Sec. 6.3 (P10): the barycentric traction equals the plain rule far away and a
    64x-refined plain rule close to the curve, where the plain rule itself is O(1) wrong."""
    a, b, th, c = 0.2, 0.1, 0.3, np.array([0.05, -0.02])
    N = 128
    wl = {"skew": 0.0, "centers": c[None], "theta": np.array([th]), "a": np.array([a]), "b": np.array([b]),
          "n_nodes": np.array([N])}
    g = geometry.build_geometry(wl)
    rng = np.random.default_rng(9)
    coeffs = rng.standard_normal((2, 12))
    t = 2 * np.pi * np.arange(N) / N
    s2 = np.stack([sum(cf[k] * np.cos(k * t) + cf[k + 6] * np.sin(k * t) for k in range(6)) for cf in coeffs], 1)
    # targets at distance `gap` outside the curve, normal along the curve normal
    ts = np.array([0.1, 1.3, 2.9, 4.4])
    ct, st = np.cos(th), np.sin(th)
    base = np.stack([c[0] + ct * a * np.cos(ts) - st * b * np.sin(ts), c[1] + st * a * np.cos(ts) + ct * b * np.sin(ts)], 1)
    dxp = np.stack([-ct * a * np.sin(ts) - st * b * np.cos(ts), -st * a * np.sin(ts) + ct * b * np.cos(ts)], 1)
    nrm = np.stack([dxp[:, 1], -dxp[:, 0]], 1) / np.linalg.norm(dxp, axis=1)[:, None]
    xt = base + gap * nrm
    nt = np.stack([np.cos(ts + 0.4), np.sin(ts + 0.4)], 1)
    vp = close.curve_vplus(g, 0, s2)
    Tb = close.traction_bary(g, 0, vp, xt, nt)
    Tp = close.plain_traction(g, 0, s2, xt, nt)
    Tf = _fine_plain_traction(a, b, th, c, coeffs, 64 * N, xt, nt)
    scale = np.abs(Tf).max()
    err_b = np.abs(Tb - Tf).max() / scale
    err_p = np.abs(Tp - Tf).max() / scale
    if gap > 0.1:
        assert np.abs(Tb - Tp).max() < 1e-13 * scale
    else:
        assert err_b < 1e-12      # spectral: ~1e-14 at N = 128 for gaps 1e-2 and 1e-3
        assert err_p > 1e-2       # the plain rule is O(1e-2 .. 1) wrong here


def test_stresslet_equals_wall_integral():
    """eq. (mueff) evaluated on D equals the particle-stresslet form when D is clear (P12)."""
    prob = op.make_problem(W.single_ellipse(skew=0.2))
    x, _ = op.solve(prob, tol=1e-12)
    assert abs(readout.mu_eff(prob, x) - readout.mu_eff_wall(prob, x)) < 1e-6


def test_periodizer_convergence():
    """3x3 images / R = 1.5 / M = 32 against 5x5 images / R = 2.5 / M = 96 (P16)."""
    res = []
    for kw in (dict(), dict(image_range=2, R=2.5, M=96, m=64)):
        prob = op.make_problem(W.single_ellipse(), **kw)
        x, _ = op.solve(prob, tol=1e-12)
        _, om = readout.velocities(prob, x)
        res.append((om[0], readout.mu_eff(prob, x)))
    assert abs(res[0][0] - res[1][0]) < 2e-6
    assert abs(res[0][1] - res[1][1]) < 3e-7


@pytest.mark.parametrize("kw,tol", [(dict(), 3e-6), (dict(M=40, m=40, R=1.3), 2e-7)])
def test_translation_invariance(kw, tol):
    """Moving every particle by delta relative to the cell/proxies changes nothing
    physical: omega, mu_eff and differences of the disturbance velocity are invariant (P15). The residual is the MFS
    discretisation error: ~1.5e-6 in omega at M = 32, R = 1.5; ~6e-8 at M = 40, R = 1.3."""
    wl = W.random_ellipses(3, 0.2, seed=21, nodes=96, skew=0.15)
    out = []
    for delta in (np.zeros(2), np.array([0.13, -0.21])):
        w2 = dict(wl, centers=wl["centers"] + delta)
        prob = op.make_problem(w2, **kw)
        x, _ = op.solve(prob, tol=1e-12)
        v, om = readout.velocities(prob, x)
        # disturbance velocity u(c_i) = v_i - u0(c_i) at the wrapped centres is periodic
        dist = v - np.stack([w2["gamma"] * prob.geom.centers[:, 1], 0 * v[:, 1]], 1)
        out.append((dist, om, readout.mu_eff(prob, x)))
    assert np.abs(out[0][1] - out[1][1]).max() < tol
    assert abs(out[0][2] - out[1][2]) < tol
    dv0 = out[0][0] - out[0][0][0]
    dv1 = out[1][0] - out[1][0][0]
    assert np.abs(dv0 - dv1).max() < 3 * tol
    # the velocity gauge (zero area-weighted mean disturbance) does not depend on where the
    # particles sit in the cell: the disturbance velocities themselves are invariant
    assert np.abs(out[0][0] - out[1][0]).max() < 3 * tol


@pytest.mark.parametrize("skew", [0.0, 0.25, 0.5])
def test_pinv_drops_exactly_the_gauge_modes(skew):
    """Theorem EBVP: the empty-box problem determines u and p up to a constant velocity and a
    constant pressure, nothing else. The singular modes of Q (32 circle proxies, m = 24) that the
    oracle's pseudo-inverse leaves out of its range are read off from Q+ Q itself, not from its
    rule. There are three of them; the proxy field of each is constant across the cell to 1e-5 of
    its size; their constants span both velocity gauges and the pressure gauge; and every mode
    kept is further from a constant field than any mode dropped (a truncation that dropped a real
    mode, or kept a gauge mode, fails one of these)."""
    from oracle.kernels import pressure_apply
    cell = _Cell((skew, 1.0))
    Wl = periodizer.walls(cell, 24)
    P = periodizer.proxies(cell, 32, 1.5)
    Q = periodizer.build_Q(cell, Wl, P, 1.0)
    _, s, Vt = np.linalg.svd(Q, full_matrices=False)
    kept = np.linalg.norm(periodizer.pinv_gauge_truncated(Q) @ Q @ Vt.T, axis=0)
    assert np.all((kept > 1 - 1e-6) | (kept < 1e-6))
    drop = kept < 0.5
    assert drop.sum() == 3
    t = (np.arange(12) + 0.5) / 12 - 0.5
    X = (t[:, None, None] * cell.e1 + t[None, :, None] * cell.e2).reshape(-1, 2)
    res, const = np.zeros(len(s)), np.zeros((len(s), 3))
    for k in range(len(s)):
        u = periodizer.correction_velocity(P, Vt[k], X, 1.0)
        p = pressure_apply(X[:, None, :] - P[None], periodizer.xi_to_forces(Vt[k])[None]).sum(1)
        z = np.stack([u[:, 0], u[:, 1], p], axis=1)
        const[k] = z.mean(0)
        res[k] = np.linalg.norm(z - const[k]) / np.linalg.norm(z)
    print(f"[skew {skew}] dropped: nonconstant part <= {res[drop].max():.1e}; kept: >= {res[~drop].min():.1e}")
    assert res[drop].max() < 1e-5
    assert np.linalg.cond(const[drop]) < 100
    assert res[~drop].min() > res[drop].max()


def test_operator_nullspace_structure():
    """1/2 I + K has a 3 N_o-dimensional near-null space (Sec. 5); the completion L
    removes it (P9)."""
    prob = op.make_problem(W.random_ellipses(2, 0.1, seed=3, nodes=32))
    n2 = 2 * prob.N
    A = op.dense_matrix(prob)
    B = np.zeros((n2, n2))
    e = np.zeros(n2)
    for k in range(n2):
        e[k] = 1.0
        B[:, k] = 0.5 * e + op.to1(op.pin(prob, op.apply_K(prob, op.to2(e))))
        e[k] = 0.0
    sB = np.linalg.svd(B, compute_uv=False)
    sA = np.linalg.svd(A, compute_uv=False)
    assert sB[-6:].max() < 1e-6 * sB[0]
    assert sB[-7] > 1e-3 * sB[0]
    assert sA[-1] > 1e-3 * sA[0]


@pytest.mark.parametrize("case", ["two_ellipses_gap1e-3_skew", "star_ellipse_gap5e-3", "six_ellipses_skewed"])
def test_apply_rows_equals_full_product(case):
    """apply_rows evaluates the operator of Sec. 5 (eq. BIEPerturbed) at selected targets
    only: its own self term, close pairs picked by target, the pin through node 0 (Sec. 6.2
    remark). Every selected row must equal the same row of the full product, for row sets
    with and without node 0, unsorted and with repeats."""
    if case == "two_ellipses_gap1e-3_skew":
        wl = W.two_ellipses(1e-3, n_nodes=128, skew=0.3)
    elif case == "star_ellipse_gap5e-3":
        wl = W.star_and_ellipse(gap=5e-3, n_star=192, n_ellipse=128, skew=0.2)
    else:
        wl = W.random_ellipses(6, 0.3, 3, nodes=64)
    prob = op.make_problem(wl)
    assert len(prob.pairs) > 0
    rng = np.random.default_rng(11)
    sigma = rng.standard_normal(2 * prob.N)
    full = op.to2(op.apply(prob, sigma))
    scale = np.abs(full).max()
    close_targets = np.unique(prob.pairs[:, 0])
    row_sets = [
        np.array([0, 1, prob.N - 1]),
        np.sort(rng.choice(np.arange(1, prob.N), 40, replace=False)),       # without node 0
        np.concatenate([close_targets[:30], [0], close_targets[:5]]),       # close targets, repeats
        rng.permutation(prob.N)[:25],                                        # unsorted
    ]
    for rows in row_sets:
        got = op.apply_rows(prob, sigma, rows)
        assert got.shape == (len(rows), 2)
        assert np.abs(got - full[rows]).max() <= 1e-14 * scale, (case, rows[:5])
