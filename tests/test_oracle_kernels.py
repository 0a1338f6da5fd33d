"""Pins of the oracle's kernels and quadrature against facts fixed by the paper
and by the mathematics (not by retyping the oracle's formulas)."""
import numpy as np
import pytest
import scipy.special

from oracle import _clib, geometry, kernels, near
from paper_1912_04501_amd import workloads as W

MU = 0.7


def _u(x, y, f, mu=MU):
    return kernels.stokeslet_apply(np.asarray(x) - np.asarray(y), np.asarray(f), mu)


def _p(x, y, f):
    return kernels.pressure_apply(np.asarray(x) - np.asarray(y), np.asarray(f))


def _grad_u(x, y, f, h=1e-5):
    x = np.asarray(x, float)
    J = np.zeros((2, 2))
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        J[:, k] = (_u(x + e, y, f) - _u(x - e, y, f)) / (2 * h)
    return J  # J[i, k] = d u_i / d x_k


def test_traction_kernel_is_stress_of_stokeslet():
    """eq. (Gt): G^t f equals sigma(G f, G^p f) n, built here by finite differences
    of the Stokeslet velocity and the pressure kernel (P4)."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        x, y, f = rng.standard_normal(2), rng.standard_normal(2), rng.standard_normal(2)
        n = rng.standard_normal(2)
        n /= np.linalg.norm(n)
        J = _grad_u(x, y, f)
        sig = -_p(x, y, f) * np.eye(2) + MU * (J + J.T)
        T_fd = sig @ n
        T = kernels.traction_apply(x - y, n, f)
        assert np.allclose(T, T_fd, rtol=1e-6, atol=1e-7 * np.abs(T_fd).max())


def test_stokeslet_solves_stokes_and_carries_unit_force():
    """(G, G^p) solve Stokes away from the source (-mu Lap u + grad p = 0, div u = 0),
    and the traction flux through a circle around the source is -f (force balance,
    which fixes the 1/(4 pi mu) normalisation of eq. Gv)."""
    y = np.array([0.1, -0.2])
    f = np.array([0.3, -0.6])
    x = np.array([0.7, 0.4])
    h = 1e-3
    lap = np.zeros(2)
    gp = np.zeros(2)
    div = 0.0
    for k in range(2):
        e = np.zeros(2)
        e[k] = h
        lap += (_u(x + e, y, f) - 2 * _u(x, y, f) + _u(x - e, y, f)) / h ** 2
        gp[k] = (_p(x + e, y, f) - _p(x - e, y, f)) / (2 * h)
        div += (_u(x + e, y, f)[k] - _u(x - e, y, f)[k]) / (2 * h)
    assert np.allclose(-MU * lap + gp, 0, atol=1e-5)
    assert abs(div) < 1e-6 * np.abs(_u(x, y, f)).max() / 0.5
    t = np.linspace(0, 2 * np.pi, 200, endpoint=False)
    n = np.stack([np.cos(t), np.sin(t)], 1)
    pts = y + 0.37 * n
    T = kernels.traction_apply(pts - y, n, f[None, :])
    flux = T.sum(0) * (2 * np.pi * 0.37 / 200)
    assert np.allclose(flux, -f, atol=1e-12)


def test_vorticity_matches_finite_differences():
    rng = np.random.default_rng(1)
    for _ in range(10):
        x, y, f = rng.standard_normal(2), rng.standard_normal(2), rng.standard_normal(2)
        J = _grad_u(x, y, f)
        assert np.isclose(kernels.vorticity_apply(x - y, f, MU), J[1, 0] - J[0, 1], rtol=1e-7)


@pytest.mark.parametrize("a,b,theta", [(0.2, 0.1, 0.0), (0.3, 0.1, 0.7), (0.05, 0.04, 2.0)])
def test_trapezoid_rule_spectral(a, b, theta):
    """Sec. 6 periodic trapezoid rule (P1): int n ds = 0, int x.n ds = 2 * area = 2 pi a b,
    perimeter = 4 a E(1 - b^2/a^2) (complete elliptic integral), geometric convergence."""
    per = 4 * a * scipy.special.ellipe(1 - (b / a) ** 2)
    errs = []
    for N in (8, 16, 32, 64, 128):
        x, xp, tau, n, w, kappa = geometry.ellipse_nodes(np.array([0.3, -0.1]), theta, a, b, N)
        assert np.abs((w[:, None] * n).sum(0)).max() < 1e-15
        area2 = (w * ((x - [0.3, -0.1]) * n).sum(1)).sum()
        errs.append(max(abs(w.sum() - per) / per, abs(area2 - 2 * np.pi * a * b) / (2 * np.pi * a * b)))
    assert errs[-1] < 1e-14
    assert errs[1] < errs[0] and errs[2] < errs[1]


def test_skew_reduction_and_wrap():
    assert geometry.reduce_skew(0.7) == pytest.approx(-0.3)
    assert geometry.reduce_skew(0.5) == pytest.approx(-0.5)
    e1, e2 = geometry.lattice(0.2)
    c = geometry.wrap_centers(np.array([[0.9, 0.1], [0.0, 0.75]]), e1, e2)
    B = np.stack([e1, e2], 1)
    ab = np.linalg.solve(B, c.T).T
    assert np.all(ab >= -0.5) and np.all(ab < 0.5)
    # the same lattice point modulo e1, e2
    d = np.linalg.solve(B, (np.array([[0.9, 0.1], [0.0, 0.75]]) - c).T).T
    assert np.allclose(d, np.round(d))


def test_c_near_sum_equals_python_loops():
    """The plain-C near sum against a pure-Python loop over the same pairs."""
    wl = W.random_ellipses(3, 0.2, seed=3, nodes=16)
    g = geometry.build_geometry(wl)
    s2 = np.random.default_rng(0).standard_normal((g.N, 2))
    a = near.near_traction(g, s2)
    b = near.near_traction_bruteforce(g, s2)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


def test_self_term_is_limit_of_kernel():
    """The diagonal of K: G^t(x, y; n_x) w sigma -> -(kappa/2pi) tau tau^T as y -> x along Gamma."""
    a, b, th = 0.2, 0.1, 0.4
    x0, _, tau0, n0, _, k0 = geometry.ellipse_nodes(np.zeros(2), th, a, b, 8)
    for h in (1e-3, 1e-4):
        # point at parameter t = h on the same curve
        ct, st = np.cos(th), np.sin(th)
        y = np.array([ct * a * np.cos(h) - st * b * np.sin(h), st * a * np.cos(h) + ct * b * np.sin(h)])
        sig = np.array([0.3, -0.8])
        lim = -(k0[0] / (2 * np.pi)) * tau0[0] * (tau0[0] @ sig)
        val = kernels.traction_apply(x0[0] - y, n0[0], sig)
        assert np.allclose(val, lim, atol=5 * h * np.abs(lim).max())
