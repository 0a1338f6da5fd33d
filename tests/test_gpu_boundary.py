"""Boundary calls through the C ABI: an ensemble set and solved in one call (lattices, cell
centres and CSR particle arrays in the call), node counts by the perimeter rule, bfloat16
features, and the network's set-weights / backward / Adam-step calls, each against the
FP64 oracle (or, for the cell centre, against the library's own single-cell handle whose
lattice is centred there)."""
import math

import numpy as np
import pytest

from oracle import learned as OL
from oracle import operator as op
from oracle import readout as ro
from oracle.geometry import build_geometry
from paper_1912_04501_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _spm():
    from paper_1912_04501_amd import spm
    return spm


def _n(t):
    return t.detach().cpu().numpy()


def _t(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


CENTRES = [(0.0, 0.0), (0.3, -0.7), (-1.2, 2.5)]


def _cells():
    return [W.random_ellipses(5, 0.3, 41, target_total=420),
            W.random_ellipses(7, 0.25, 42, target_total=560),
            W.random_ellipses(4, 0.3, 43, target_total=300)]


def _batch_args(cells, centres):
    lat, cen = [], []
    for c, (cx, cy) in zip(cells, centres):
        lat.append([1.0, 0.0, c["skew"], 1.0, cx, cy])
        cen.append(np.asarray(c["centers"], float) + np.array([cx, cy]))
    off = np.concatenate([[0], np.cumsum([len(c["theta"]) for c in cells])]).astype(np.int32)
    cat = lambda k: np.concatenate([np.asarray(c[k], float) for c in cells])  # noqa: E731
    nn = np.concatenate([np.asarray(c["n_nodes"]) for c in cells]).astype(np.int32)
    return np.array(lat), off, np.concatenate(cen), cat("theta"), cat("a"), cat("b"), nn


def test_solve_batch_one_call_matches_oracle():
    """Cells centred away from the origin, solved in one call: omega and mu_eff are those of
    the oracle's solve of each cell about the origin, and the velocities differ from it by
    u0 = (gamma y, 0) of the cell centre (the method is translation invariant, u0 is not)."""
    spm = _spm()
    cells = _cells()
    lat, off, cen, th, a, b, nn = _batch_args(cells, CENTRES)
    s = spm.Solver("cuda:0", precond=spm.SPM_PRECOND_BLOCK, precision=spm.SPM_FP32_RELAXED)
    r = s.solve_batch(lat, off, cen, th, a, b, nn)
    vel, om, mu = _n(r["vel"]), _n(r["omega"]), _n(r["mu_eff"])
    for c, wl in enumerate(cells):
        assert r["infos"][c]["rel_residual"] <= 1e-10
        prob = op.make_problem(wl)
        x, _ = op.solve(prob, tol=1e-12)
        v_ref, om_ref = ro.velocities(prob, x)
        mu_ref = ro.mu_eff(prob, x)
        sl = slice(off[c], off[c + 1])
        v_ref = v_ref + np.array([CENTRES[c][1], 0.0])
        sc_v = math.hypot(wl["skew"], 1.0)
        print(f"[solve_batch cell {c}] omega {np.abs(om[sl] - om_ref).max():.2e} "
              f"v {np.abs(vel[sl] - v_ref).max():.2e} mu {abs(mu[c] - mu_ref):.2e}")
        # relaxed FP32 with the block preconditioner stops at the FP64 residual 1e-10
        assert np.abs(om[sl] - om_ref).max() <= 1e-7 * max(1.0, np.abs(om_ref).max())
        assert np.abs(vel[sl] - v_ref).max() <= 1e-7 * sc_v
        assert abs(mu[c] - mu_ref) <= 1e-7 * mu_ref


def test_solve_batch_centre_matches_centred_single_cell():
    """A cell centred at c in the one-call ensemble gives the same readouts as a single-cell
    handle whose lattice (walls, proxies, wrapping) is centred at c natively (FP64 solves)."""
    spm = _spm()
    cells = _cells()
    lat, off, cen, th, a, b, nn = _batch_args(cells, CENTRES)
    r = spm.Solver("cuda:0").solve_batch(lat, off, cen, th, a, b, nn)
    for c, wl in enumerate(cells):
        one = spm.Solver("cuda:0")
        one.set_lattice(wl["skew"], center=CENTRES[c])
        sl = slice(off[c], off[c + 1])
        one.set_ellipses(cen[sl], th[sl], a[sl], b[sl], nn[sl])
        q = one.solve()
        scale = math.hypot(wl["skew"], 1.0)
        assert np.abs(_n(r["vel"])[sl] - _n(q["vel"])).max() <= 1e-9 * scale
        assert np.abs(_n(r["omega"])[sl] - _n(q["omega"])).max() <= 1e-9
        assert abs(float(_n(r["mu_eff"])[c]) - float(q["mu_eff"].item())) <= 1e-9


def test_solve_batch_rejects_bad_lattice():
    spm = _spm()
    cells = _cells()[:1]
    lat, off, cen, th, a, b, nn = _batch_args(cells, CENTRES[:1])
    lat[0, 0] = 1.5
    with pytest.raises(spm.SpmError):
        spm.Solver("cuda:0").solve_batch(lat, off, cen, th, a, b, nn)


def test_perimeter_rule_node_counts():
    """n_nodes NULL: the library's node counts are clamp(8 ceil(P / (8 h)), 64, 256) with the
    configured spacing; the nodes then coincide with the oracle's geometry built from the
    input generator's own implementation of that rule (Ramanujan's perimeter)."""
    spm = _spm()
    wl = W.ellipses_25()
    h = W.c1_h_star()
    want = W.node_rule(wl["a"], wl["b"], h)
    s = spm.Solver("cuda:0", node_spacing=h)
    s.set_lattice(wl["skew"])
    s.set_ellipses(wl["centers"], wl["theta"], wl["a"], wl["b"], None)
    assert s.N == int(want.sum())
    g = build_geometry({**wl, "n_nodes": want})
    x, y = (_n(t) for t in s.nodes()[:2])
    assert np.abs(x - g.x[:, 0]).max() <= 1e-14 and np.abs(y - g.x[:, 1]).max() <= 1e-14
    # default spacing is the same value
    d = spm.Solver("cuda:0")
    d.set_lattice(wl["skew"])
    d.set_ellipses(wl["centers"], wl["theta"], wl["a"], wl["b"], None)
    assert d.N == s.N


def test_perimeter_rule_star():
    """Stars: the perimeter by the trapezoid rule on |x'(t)| (here with 4,096 points)."""
    spm = _spm()
    wl = W.star_and_ellipse(gap=2e-2)
    h = 4e-3
    k = np.asarray(wl["kind"])
    prm = np.asarray(wl["params"], float).reshape(-1, 4)
    want = []
    for kind, p in zip(k, prm):
        if kind == 0:
            P = W._ellipse_perimeter(p[0], p[1])
        else:
            t = 2 * np.pi * np.arange(4096) / 4096
            r = p[0] * (1 + p[1] * np.cos(p[2] * t + p[3]))
            rp = -p[0] * p[1] * p[2] * np.sin(p[2] * t + p[3])
            P = np.sqrt(r * r + rp * rp).mean() * 2 * np.pi
        want.append(min(256, max(64, 8 * math.ceil(P / (8 * h)))))
    s = spm.Solver("cuda:0", node_spacing=h)
    s.set_cells([{**wl, "n_nodes": None}])
    assert s.N == sum(want)


def test_features_bf16_is_rounded_fp32():
    spm = _spm()
    s = spm.Solver("cuda:0").set_workload(W.ellipses_25())
    f32 = _n(s.features())
    f16 = s.features_bf16().float().cpu().numpy()
    assert np.array_equal(f16, OL.round_bf16(f32).astype(np.float32))


def _params(seed):
    p = OL.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    for W_, b_ in p:
        b_ += 0.05 * rng.standard_normal(b_.shape)
    flat = np.concatenate([np.concatenate([W_.ravel(), b_.ravel()]) for W_, b_ in p]).astype(np.float32)
    return flat


def _unpack(flat):
    out, o = [], 0
    for fi, fo in zip(OL.LAYERS[:-1], OL.LAYERS[1:]):
        W_ = flat[o:o + fo * fi].reshape(fo, fi).astype(np.float64)
        o += fo * fi
        b_ = flat[o:o + fo].astype(np.float64)
        o += fo
        out.append([W_, b_])
    return out


def _pack(params):
    return np.concatenate([np.concatenate([W_.ravel(), b_.ravel()]) for W_, b_ in params])


@pytest.mark.parametrize("batch", [1, 77, 300])
def test_mlp_backward_upstream_gradient(batch):
    """grad = d(sum dy . y)/d params for a random dy: FP32 matrix-core mode within 1e-5 of the
    oracle's back-propagation, BF16 mode within 1e-4 of the oracle with bf16-rounded operands
    (Frobenius-norm relative errors)."""
    spm = _spm()
    flat = _params(4)
    params = _unpack(flat)
    rng = np.random.default_rng(batch + 7)
    x = rng.standard_normal((batch, OL.N_FEAT)).astype(np.float32).astype(np.float64)
    dy = rng.standard_normal((batch, OL.N_OUT)).astype(np.float32).astype(np.float64)
    net = spm.MLP("cuda:0")
    net.set_params(_t(flat, torch.float32))
    for mode, rounding, tol in ((spm.SPM_MLP_FP32, None, 1e-5), (spm.SPM_MLP_BF16, "bf16", 1e-4)):
        _, acts = OL.forward(params, x, rounding)
        ref = _pack(OL.backward(params, acts, dy, rounding))
        g = _n(net.backward(_t(x, torch.float32), _t(dy, torch.float32), mode)).astype(np.float64)
        err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
        print(f"[backward B={batch} mode={mode}] {err:.2e}")
        assert err <= tol


def test_mlp_adam_step_matches_oracle():
    """Two single Adam steps with caller-chosen hyper-parameters against the oracle's Adam."""
    spm = _spm()
    flat = _params(5)
    params = _unpack(flat)
    rng = np.random.default_rng(3)
    grads = [rng.standard_normal(flat.size).astype(np.float32) for _ in range(2)]
    net = spm.MLP("cuda:0")
    net.set_params(_t(flat, torch.float32))
    lr, b1, b2, eps = 2e-3, 0.8, 0.99, 1e-6
    state = {}
    for k, g in enumerate(grads):
        net.adam_step(_t(g, torch.float32), lr, b1, b2, eps, step=k + 1)
        OL.adam_step(params, _unpack(g), state, lr, b1, b2, eps)
    got = _n(net.get_params()).astype(np.float64)
    want = _pack(params)
    print(f"[adam_step] max diff {np.abs(got - want).max():.2e}")
    assert np.abs(got - want).max() <= 1e-6
    with pytest.raises(spm.SpmError):
        net.adam_step(_t(grads[0], torch.float32), lr, step=0)


def test_mlp_set_weights():
    """bfloat16 weights alone set the master to their exact FP32 values (and BF16-mode
    outputs are then those of set_params with the widened values); a consistent pair sets
    the master (outputs as set_params of the master: biases are added in FP32, only the
    product operands are rounded); an inconsistent pair is rejected."""
    spm = _spm()
    flat = _params(6)
    bf = OL.round_bf16(flat).astype(np.float32)
    net = spm.MLP("cuda:0")
    net.set_weights(params_bf16=_t(bf, torch.float32).to(torch.bfloat16))
    assert np.array_equal(_n(net.get_params()), bf)
    x = _t(np.random.default_rng(1).standard_normal((50, OL.N_FEAT)), torch.float32)
    ref = spm.MLP("cuda:0")
    for mode in (spm.SPM_MLP_BF16, spm.SPM_MLP_FP32):
        ref.set_params(_t(bf, torch.float32))
        assert np.array_equal(_n(net.forward(x, mode)), _n(ref.forward(x, mode)))
    net.set_weights(params_bf16=_t(bf, torch.float32).to(torch.bfloat16), master=_t(flat, torch.float32))
    assert np.array_equal(_n(net.get_params()), flat)
    ref.set_params(_t(flat, torch.float32))
    assert np.array_equal(_n(net.forward(x, spm.SPM_MLP_BF16)), _n(ref.forward(x, spm.SPM_MLP_BF16)))
    wrong = bf.copy()
    wrong[17] = np.float32(wrong[17] * 2 + 1)
    with pytest.raises(spm.SpmError):
        net.set_weights(params_bf16=_t(wrong, torch.float32).to(torch.bfloat16), master=_t(flat, torch.float32))
