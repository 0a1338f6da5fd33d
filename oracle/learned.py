"""Learned warm start: features, Fourier targets and a plain FP64 MLP (test infrastructure).

The network maps each particle's neighbourhood to its traction density, which then
serves as the initial guess of GMRES (its only role: the solver still runs to the
same FP64 residual, so the network changes cost, never the answer).

* features (33 per particle): the 8 nearest other particles (all 3x3 lattice images,
  the particle's own images included), sorted by centre distance; for each, the
  offset of its centre in the particle's body frame in units of the particle's
  semi-major axis, R(-theta_i)(c_j + s - c_i)/a_i, and (cos 2(theta_j - theta_i),
  sin 2(theta_j - theta_i)) (ellipses are symmetric under a half turn); then a_i/b_i.
* offset: the completed operator maps the normal field n to n/2 (the single layer
  with density n is a pure pressure, so K n = n/2 on every curve, the pin removes
  the value at the first node and L n = 0). A solution is therefore determined by the
  geometry only up to a cell-wide multiple beta n that no local feature can predict:
  the target density is sigma - beta* n with beta* = <sigma, n> / <n, n> over the
  cell's nodes.
* warm start: the decoded density g is scaled and given its offset by the least
  squares fit min over (alpha, beta) of |b - alpha A g - beta n / 2|, i.e. the
  guess alpha g + beta n with the smallest residual in that plane (never worse than
  the zero guess, which the plane contains).
* targets (128 per particle): the body-frame density s_k = R(-theta_i) sigma'_k / (mu gamma)
  of sigma' = sigma - beta* n at the nodes t_k = 2 pi k / N_i as a complex sequence
  s1 + i s2, its discrete Fourier coefficients c_m = (1/N_i) sum_k s_k exp(-i m t_k)
  for m = -32..31; real parts then imaginary parts.
* decode: sigma_k = mu gamma R(theta_i) sum_m c_m exp(i m t_k) (exact for densities
  whose modes lie in -32..31 when N_i >= 64).
* MLP: 33 -> 256 -> 256 -> 256 -> 128, ReLU on the hidden layers, loss
  (1/(2B)) sum_b |y_b - t_b|^2, Adam with bias correction.
"""
from __future__ import annotations

import numpy as np

N_NEIGH = 8
N_FEAT = 4 * N_NEIGH + 1
N_MODES = 64
N_OUT = 2 * N_MODES
LAYERS = (N_FEAT, 256, 256, 256, N_OUT)


def features(geom):
    c = geom.centers
    sh = geom.shifts(1)
    zero = int(np.argmin((sh ** 2).sum(1)))
    out = np.zeros((geom.No, N_FEAT))
    for i in range(geom.No):
        cand = []
        for j in range(geom.No):
            for si, s in enumerate(sh):
                if j == i and si == zero:
                    continue
                d = c[j] + s - c[i]
                cand.append((float(d[0] * d[0] + d[1] * d[1]), j, si, d))
        cand.sort(key=lambda t: (t[0], t[1], t[2]))
        ct, st = np.cos(geom.theta[i]), np.sin(geom.theta[i])
        for k in range(N_NEIGH):
            _, j, _, d = cand[k]
            bx = (ct * d[0] + st * d[1]) / geom.a[i]
            by = (-st * d[0] + ct * d[1]) / geom.a[i]
            dth = 2.0 * (geom.theta[j] - geom.theta[i])
            out[i, 4 * k:4 * k + 4] = (bx, by, np.cos(dth), np.sin(dth))
        out[i, -1] = geom.a[i] / geom.b[i]
    return out


def _mode_index():
    return np.arange(-N_MODES // 2, N_MODES // 2)


def remove_offset(geom, sigma2):
    """sigma - beta* n with beta* = <sigma, n> / <n, n> over all nodes of the cell."""
    beta = (sigma2 * geom.n).sum() / (geom.n * geom.n).sum()
    return sigma2 - beta * geom.n


def targets(geom, sigma2, mu=1.0, gamma=1.0):
    return modes(geom, remove_offset(geom, sigma2), mu, gamma)


def modes(geom, sigma2, mu=1.0, gamma=1.0):
    """Body-frame Fourier coefficients c_m, m = -32..31, of every particle's density."""
    out = np.zeros((geom.No, N_OUT))
    m = _mode_index()
    for i in range(geom.No):
        sl = geom.particle_slice(i)
        n = geom.n_nodes[i]
        ct, st = np.cos(geom.theta[i]), np.sin(geom.theta[i])
        s1 = (ct * sigma2[sl, 0] + st * sigma2[sl, 1]) / (mu * gamma)
        s2 = (-st * sigma2[sl, 0] + ct * sigma2[sl, 1]) / (mu * gamma)
        t = 2.0 * np.pi * np.arange(n) / n
        coef = (np.exp(-1j * np.outer(m, t)) @ (s1 + 1j * s2)) / n
        out[i, :N_MODES] = coef.real
        out[i, N_MODES:] = coef.imag
    return out


def decode(geom, modes, mu=1.0, gamma=1.0):
    sig = np.zeros((geom.N, 2))
    m = _mode_index()
    for i in range(geom.No):
        sl = geom.particle_slice(i)
        n = geom.n_nodes[i]
        t = 2.0 * np.pi * np.arange(n) / n
        coef = modes[i, :N_MODES] + 1j * modes[i, N_MODES:]
        s = np.exp(1j * np.outer(t, m)) @ coef
        ct, st = np.cos(geom.theta[i]), np.sin(geom.theta[i])
        sig[sl, 0] = mu * gamma * (ct * s.real - st * s.imag)
        sig[sl, 1] = mu * gamma * (st * s.real + ct * s.imag)
    return sig


def init_params(seed=0, layers=LAYERS):
    """He-normal weights, zero biases; W has shape (out, in)."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(layers[:-1], layers[1:]):
        params.append([rng.standard_normal((fo, fi)) * np.sqrt(2.0 / fi), np.zeros(fo)])
    return params


def round_bf16(a):
    """Round to bfloat16 through FP32, nearest even (the matrix-core operand format)."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _op(a, rounding):
    return a if rounding is None else round_bf16(a)


def forward(params, x, rounding=None):
    """rounding="bf16" rounds both operands of every layer product to bfloat16 (the
    products and sums stay FP64): the arithmetic of a bf16 x bf16 -> fp32 matrix unit
    up to the order and precision of accumulation."""
    acts = [x]
    h = x
    for li, (W, b) in enumerate(params):
        z = _op(h, rounding) @ _op(W, rounding).T + b
        h = np.maximum(z, 0.0) if li < len(params) - 1 else z
        acts.append(h)
    return h, acts


def backward(params, acts, dy, rounding=None):
    """Gradients of sum_b dy_b . y_b with respect to every (W, b), for the activations of
    one forward pass (acts) and an upstream gradient dy = dL/dy of shape (B, out): the
    chain rule through each affine layer (dW = d^T h_in, db = sum_b d) and through ReLU
    (d <- (d W) * [h > 0])."""
    d = dy
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        h_in = acts[li]
        grads[li] = [_op(d, rounding).T @ _op(h_in, rounding), d.sum(0)]
        if li > 0:
            d = (_op(d, rounding) @ _op(W, rounding)) * (acts[li] > 0)
    return grads


def loss_and_grads(params, x, t, rounding=None):
    """Loss (1/(2B)) sum |y - t|^2 and its gradients: backward with dy = (y - t) / B."""
    y, acts = forward(params, x, rounding)
    B = x.shape[0]
    loss = 0.5 * ((y - t) ** 2).sum() / B
    return loss, backward(params, acts, (y - t) / B, rounding)


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """state: {"t": int, "m": [...], "v": [...]} (created when empty)."""
    if not state:
        state["t"] = 0
        state["m"] = [[np.zeros_like(p) for p in layer] for layer in params]
        state["v"] = [[np.zeros_like(p) for p in layer] for layer in params]
    state["t"] += 1
    t = state["t"]
    for li, layer in enumerate(params):
        for k in range(2):
            g = grads[li][k]
            state["m"][li][k] = b1 * state["m"][li][k] + (1 - b1) * g
            state["v"][li][k] = b2 * state["v"][li][k] + (1 - b2) * g * g
            mh = state["m"][li][k] / (1 - b1 ** t)
            vh = state["v"][li][k] / (1 - b2 ** t)
            layer[k] = layer[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def warm_start_from_modes(prob, modes_):
    """x0 = alpha g + beta n, g = decode(modes), (alpha, beta) minimising
    |b - alpha A g - beta n / 2| (A n = n / 2)."""
    from .operator import apply, rhs, to1
    geo = prob.geom
    g = to1(decode(geo, modes_, prob.cfg.mu, prob.cfg.gamma))
    b = rhs(prob)
    z = apply(prob, g)
    h = 0.5 * to1(geo.n)
    M = np.array([[z @ z, z @ h], [z @ h, h @ h]])
    alpha, beta = np.linalg.solve(M, np.array([b @ z, b @ h]))
    return alpha * g + beta * to1(geo.n)


def learned_guess(prob, params):
    """The network's warm start: features -> MLP -> decode -> offset fit."""
    y, _ = forward(params, features(prob.geom))
    return warm_start_from_modes(prob, y)
