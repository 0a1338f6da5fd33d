"""Pins of the oracle's block preconditioner and learned warm start (features, Fourier
targets, MLP, Adam) against identities of the BIE and closed forms."""
import numpy as np
import pytest

from oracle import geometry, learned, near, precond
from oracle import operator as op
from paper_1912_04501_amd import workloads as W


def _one_ellipse(a, b, n, theta=0.0, c=(0.0, 0.0)):
    return geometry.build_geometry({"skew": 0.0, "centers": [list(c)], "theta": [theta], "a": [a], "b": [b],
                                    "n_nodes": [n]})


def _rigid_moments(x, w, v1, v2):
    return np.array([(w * v1).sum(), (w * v2).sum(), (w * (-x[:, 1] * v1 + x[:, 0] * v2)).sum()])


@pytest.mark.parametrize("a,b,n", [(0.2, 0.1, 64), (0.09, 0.03, 128)])
def test_self_block_normal_is_eigenvector(a, b, n):
    """The single layer with density n is a pure pressure field, so K n = n/2 on the
    curve (Sec. 4.1); n carries no net force or torque, so L n = 0: B n = n."""
    x, tau, nrm, w, kap = precond.body_nodes(a, b, n)
    B = precond.self_block(a, b, n)
    v = np.concatenate([nrm[:, 0], nrm[:, 1]])
    assert np.abs(B @ v - v).max() < 1e-12


def test_self_block_interior_gauss_law():
    """The interior traction 1/2 sigma + K sigma has no net force or torque (P2)."""
    a, b, n = 0.15, 0.06, 96
    x, tau, nrm, w, kap = precond.body_nodes(a, b, n)
    B0 = precond.self_block(a, b, n, complete=False)
    t = 2 * np.pi * np.arange(n) / n
    rng = np.random.default_rng(4)
    s1 = sum(rng.standard_normal() * np.cos(k * t + rng.uniform(0, 6)) for k in range(6))
    s2 = sum(rng.standard_normal() * np.cos(k * t + rng.uniform(0, 6)) for k in range(6))
    y = B0 @ np.concatenate([s1, s2])
    mom = _rigid_moments(x, w, y[:n], y[n:])
    scale = np.abs(_rigid_moments(x, w, np.abs(s1), np.abs(s2))).max()
    assert np.abs(mom).max() < 1e-12 * max(scale, 1.0)


def test_self_block_equals_matrix_free_free_space_operator():
    """Rows of the assembled block equal the matrix-free free-space Nystrom sum
    (near sum without images + diagonal limit) plus the completion, on one ellipse."""
    a, b, n = 0.2, 0.07, 80
    g = _one_ellipse(a, b, n)
    rng = np.random.default_rng(1)
    s2 = rng.standard_normal((n, 2))
    K = near.near_traction(g, s2, rng=0) + near.self_term(g, s2)
    F = (g.w[:, None] * s2).sum(0)
    perp = np.stack([-g.x[:, 1], g.x[:, 0]], 1)
    tq = (g.w * (perp * s2).sum(1)).sum()
    ref = 0.5 * s2 + K + F[None, :] + perp * tq
    y = precond.self_block(a, b, n) @ np.concatenate([s2[:, 0], s2[:, 1]])
    assert np.abs(y[:n] - ref[:, 0]).max() < 1e-13 * np.abs(ref).max()
    assert np.abs(y[n:] - ref[:, 1]).max() < 1e-13 * np.abs(ref).max()


def test_block_inverse_undoes_rotated_operator():
    """P^{-1} (lab-frame isolated operator) v = v for a rotated, translated ellipse:
    the body-frame block with the node rotations inverts the lab-frame operator."""
    a, b, n, th = 0.12, 0.05, 64, 1.1
    g = _one_ellipse(a, b, n, th, c=(0.2, -0.3))
    rng = np.random.default_rng(2)
    s2 = rng.standard_normal((n, 2))
    K = near.near_traction(g, s2, rng=0) + near.self_term(g, s2)
    F = (g.w[:, None] * s2).sum(0)
    rel = g.x - g.centers[0]
    perp = np.stack([-rel[:, 1], rel[:, 0]], 1)
    tq = (g.w * (perp * s2).sum(1)).sum()
    Bv = 0.5 * s2 + K + F[None, :] + perp * tq
    back = precond.apply_inverse(g, np.concatenate([Bv[:, 0], Bv[:, 1]]))
    assert np.abs(back - np.concatenate([s2[:, 0], s2[:, 1]])).max() < 1e-10


def test_self_block_is_invertible():
    s = np.linalg.svd(precond.self_block(0.2, 0.1, 64), compute_uv=False)
    assert s.min() > 1e-3 and s.max() < 2.0


# ---------------------------------------------------------------- learned warm start

def _band_limited(n, rng, mmax=32):
    t = 2 * np.pi * np.arange(n) / n
    ms = np.arange(-mmax, mmax)
    c = rng.standard_normal(len(ms)) + 1j * rng.standard_normal(len(ms))
    return c, np.exp(1j * np.outer(t, ms)) @ c


@pytest.mark.parametrize("n", [64, 128])
def test_modes_and_decode_are_exact_dft(n):
    """For a body-frame density with modes in -32..31 the coefficients are recovered
    exactly and decoding returns the density (discrete orthogonality of exp(i m t_k))."""
    rng = np.random.default_rng(n)
    th = 0.7
    g = _one_ellipse(0.2, 0.1, n, th)
    c, s = _band_limited(n, rng)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    mu, gam = 0.8, 1.3
    sig = mu * gam * (np.stack([s.real, s.imag], 1) @ R.T)
    md = learned.modes(g, sig, mu, gam)
    assert np.abs(md[0, :64] - c.real).max() < 1e-12
    assert np.abs(md[0, 64:] - c.imag).max() < 1e-12
    assert np.abs(learned.decode(g, md, mu, gam) - sig).max() < 1e-11


def test_single_mode_target():
    """sigma = mu gamma R(theta) (cos t, sin t): only c_1 = 1."""
    n, th = 96, -0.4
    g = _one_ellipse(0.2, 0.1, n, th)
    t = 2 * np.pi * np.arange(n) / n
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    sig = np.stack([np.cos(t), np.sin(t)], 1) @ R.T
    md = learned.modes(g, sig)
    want = np.zeros(128)
    want[32 + 1] = 1.0
    assert np.abs(md[0] - want).max() < 1e-13


def test_offset_removal():
    g = geometry.build_geometry(W.random_ellipses(3, 0.2, seed=5, nodes=64))
    rng = np.random.default_rng(0)
    s = rng.standard_normal((g.N, 2))
    r = learned.remove_offset(g, s)
    assert abs((r * g.n).sum()) < 1e-12 * np.abs(s).sum()
    assert np.abs(learned.remove_offset(g, s + 3.7 * g.n) - r).max() < 1e-12


def test_completed_operator_maps_normal_to_half_normal():
    """K n = n/2, the pin subtracts n/2 . n0 = 1/2 times n and L n = 0, so A n = n/2:
    the offset direction is an exact eigenvector (basis of the residual offset fit)."""
    prob = op.make_problem(W.random_ellipses(4, 0.25, seed=3, nodes=96))
    nv = op.to1(prob.geom.n)
    assert np.abs(op.apply(prob, nv) - 0.5 * nv).max() < 1e-9


def test_warm_start_from_exact_modes_recovers_solution():
    """With the exact (offset-free) targets as network output, decode + residual
    offset fit returns the solution itself."""
    prob = op.make_problem(W.random_ellipses(3, 0.2, seed=7, nodes=64))
    sig, info = op.solve(prob, tol=1e-12)
    g = prob.geom
    tg = learned.targets(g, op.to2(sig))
    x0 = learned.warm_start_from_modes(prob, tg)
    assert np.linalg.norm(x0 - sig) < 1e-9 * np.linalg.norm(sig)


def test_features_single_particle_square_lattice():
    """One ellipse per unit square cell: its 8 nearest images are the lattice
    neighbours at distance 1 (shifts (-1,0), (0,-1), (0,1), (1,0) in shift order) and
    sqrt 2; the neighbours are copies of itself, so cos 2dtheta = 1, sin = 0."""
    a, b, th = 0.2, 0.1, np.pi / 2
    g = _one_ellipse(a, b, 64, th, c=(0.1, 0.2))
    f = learned.features(g)[0]
    lab = [(-1, 0), (0, -1), (0, 1), (1, 0), (-1, -1), (-1, 1), (1, -1), (1, 1)]
    for k, (dx, dy) in enumerate(lab):
        # body frame of theta = pi/2: (dx, dy) -> (dy, -dx)
        assert np.allclose(f[4 * k:4 * k + 4], [dy / a, -dx / a, 1.0, 0.0], atol=1e-14)
    assert f[-1] == pytest.approx(a / b)


def test_features_two_particles():
    wl = {"skew": 0.0, "centers": [[0.0, 0.0], [0.3, 0.0]], "theta": [0.0, 0.5], "a": [0.1, 0.1],
          "b": [0.05, 0.04], "n_nodes": [64, 64]}
    g = geometry.build_geometry(wl)
    f = learned.features(g)
    # particle 0: nearest is particle 1 at (0.3, 0), then particle 1's image at (-0.7, 0)
    assert np.allclose(f[0, 0:4], [3.0, 0.0, np.cos(1.0), np.sin(1.0)], atol=1e-13)
    assert np.allclose(f[0, 4:8], [-7.0, 0.0, np.cos(1.0), np.sin(1.0)], atol=1e-13)
    # particle 1 (theta 0.5): nearest is particle 0 at (-0.3, 0) in the lab frame
    d = np.array([-0.3, 0.0])
    bx = (np.cos(0.5) * d[0] + np.sin(0.5) * d[1]) / 0.1
    by = (-np.sin(0.5) * d[0] + np.cos(0.5) * d[1]) / 0.1
    assert np.allclose(f[1, 0:4], [bx, by, np.cos(-1.0), np.sin(-1.0)], atol=1e-13)
    assert f[1, -1] == pytest.approx(0.1 / 0.04)


def test_mlp_gradients_match_central_differences():
    """Back-propagation of the oracle MLP against central differences of its loss (P17)."""
    layers = (5, 7, 6, 3)
    params = learned.init_params(3, layers)
    for W_, b_ in params:
        b_ += 0.1 * np.random.default_rng(9).standard_normal(b_.shape)
    rng = np.random.default_rng(1)
    x, t = rng.standard_normal((11, 5)), rng.standard_normal((11, 3))
    loss, grads = learned.loss_and_grads(params, x, t)
    h = 1e-6
    for li in range(len(params)):
        for k in range(2):
            p = params[li][k]
            num = np.zeros_like(p)
            it = np.nditer(p, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = p[idx]
                p[idx] = old + h
                lp, _ = learned.loss_and_grads(params, x, t)
                p[idx] = old - h
                lm, _ = learned.loss_and_grads(params, x, t)
                p[idx] = old
                num[idx] = (lp - lm) / (2 * h)
            assert np.abs(num - grads[li][k]).max() < 1e-7 * max(1.0, np.abs(num).max())


def test_mlp_forward_hand_network():
    """Weights chosen by hand: relu(W0 x + b0) then W1 h + b1."""
    params = [[np.array([[1.0, -1.0], [2.0, 0.5]]), np.array([0.0, -1.0])],
              [np.array([[1.0, 3.0]]), np.array([0.25])]]
    y, _ = learned.forward(params, np.array([[1.0, 2.0], [3.0, 1.0]]))
    # x=(1,2): z0 = (-1, 2) -> (0, 2); y = 6 + 0.25. x=(3,1): z0 = (2, 5.5) -> y = 2 + 16.5 + 0.25
    assert np.allclose(y[:, 0], [6.25, 18.75], atol=0)


def test_adam_first_step_closed_form():
    """With bias correction, the first step moves every parameter by -lr g / (|g| + eps)."""
    params = [[np.array([[1.0, -2.0]]), np.array([0.5])]]
    grads = [[np.array([[0.3, -4.0]]), np.array([1e-3])]]
    lr = 0.01
    learned.adam_step(params, grads, {}, lr)
    g = np.array([0.3, -4.0, 1e-3])
    want = np.array([1.0, -2.0, 0.5]) - lr * g / (np.abs(g) + 1e-8)
    got = np.array([params[0][0][0, 0], params[0][0][0, 1], params[0][1][0]])
    assert np.abs(got - want).max() < 1e-15


def test_round_bf16():
    """Nearest-even rounding to 8 significand bits: representable values are kept,
    halfway cases go to the even neighbour, others to the nearest."""
    u = 2.0 ** -7   # spacing of bfloat16 in [1, 2)
    vals = np.array([1.0, -3.5, 1 + u, 1 + u / 2, 1 + 3 * u / 2, 1 + 0.7 * u, 2.0 ** -130, 0.0])
    want = np.array([1.0, -3.5, 1 + u, 1.0, 1 + 2 * u, 1 + u, 2.0 ** -130, 0.0])
    assert np.array_equal(OL_round(vals), want)


def OL_round(v):
    return learned.round_bf16(v)


def test_bf16_rounded_network_is_close_to_exact():
    """With bf16 operands the forward pass stays within a few bf16 units of the exact one."""
    params = learned.init_params(1)
    x = np.random.default_rng(2).standard_normal((50, learned.N_FEAT))
    y, _ = learned.forward(params, x)
    yb, _ = learned.forward(params, x, rounding="bf16")
    assert 1e-4 < np.abs(yb - y).max() / np.abs(y).max() < 3e-2


def test_warm_start_fit_is_never_worse_than_zero():
    """The (alpha, beta) fit contains the zero guess, so any decoded density, even
    noise, leaves a residual no larger than |b|; and it is the plane's minimiser:
    perturbing alpha or beta raises the residual."""
    prob = op.make_problem(W.random_ellipses(3, 0.2, seed=7, nodes=64))
    g = prob.geom
    b = op.rhs(prob)
    noise = 50.0 * np.random.default_rng(0).standard_normal((g.No, learned.N_OUT))
    x0 = learned.warm_start_from_modes(prob, noise)
    r0 = np.linalg.norm(b - op.apply(prob, x0))
    assert r0 <= np.linalg.norm(b) * (1 + 1e-12)
    nv = op.to1(g.n)
    for dx in (1e-3 * x0, 1e-3 * np.linalg.norm(x0) / np.linalg.norm(nv) * nv):
        assert np.linalg.norm(b - op.apply(prob, x0 + dx)) > r0


def test_mlp_backward_of_upstream_gradient_matches_central_differences():
    """Back-propagation of an arbitrary upstream gradient dy: the derivative of the scalar
    sum(dy * y) with respect to every weight and bias against central differences (the
    chain rule written out, checked independently of the loss it is usually fed)."""
    layers = (4, 6, 5, 3)
    params = learned.init_params(7, layers)
    rng = np.random.default_rng(21)
    for W_, b_ in params:
        b_ += 0.1 * rng.standard_normal(b_.shape)
    x = rng.standard_normal((9, 4))
    dy = rng.standard_normal((9, 3))
    _, acts = learned.forward(params, x)
    grads = learned.backward(params, acts, dy)

    def scalar():
        y, _ = learned.forward(params, x)
        return float((dy * y).sum())

    h = 1e-6
    for li in range(len(params)):
        for k in range(2):
            p = params[li][k]
            num = np.zeros_like(p)
            it = np.nditer(p, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = p[idx]
                p[idx] = old + h
                fp = scalar()
                p[idx] = old - h
                fm = scalar()
                p[idx] = old
                num[idx] = (fp - fm) / (2 * h)
            assert np.abs(num - grads[li][k]).max() < 1e-7 * max(1.0, np.abs(num).max())
