"""Star-shaped particles (Sec. 8, the jamming examples) on the HIP path: the
preconditioner's self blocks, time stepping, and the shape checks at set-up. The
stage-by-stage parity of star cells runs with the ellipse cases in test_gpu_parity."""
import numpy as np
import pytest

from oracle import precond as OP
from oracle import step as ostep
from oracle.geometry import build_geometry
from paper_1912_04501_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _spm():
    from paper_1912_04501_amd import spm
    return spm


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda:0")


def _n(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("wl", [W.two_stars(n_nodes=128), W.star_and_ellipse()], ids=lambda w: w["name"])
def test_precond_apply_stars(wl):
    """Block inverses of star self blocks (FP32 storage: bound 1e-5 relative)."""
    g = build_geometry(wl)
    s = _spm().Solver("cuda:0").set_workload(wl)
    v = np.random.default_rng(3).standard_normal(2 * g.N)
    out = _n(s.precond_apply(_t(v)))
    ref = OP.apply_inverse(g, v)
    e = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"[precond {wl['name']}] rel err {e:.2e}", flush=True)
    assert e <= 1e-5


def _ragged_segments():
    wl = W.random_ellipses(3, 0.2, seed=4, nodes=64)
    return dict(wl, n_nodes=np.array([66, 130, 258], dtype=np.int32), name="ellipses_66_130_258")


@pytest.mark.parametrize("wl", [dict(W.single_ellipse(n_nodes=130), name="single_ellipse_130"), _ragged_segments()],
                         ids=lambda w: w["name"])
def test_precond_apply_ragged_segments(wl):
    """The inverses are stored and applied in eight row segments per particle here (a handful of
    particles); with 130 nodes the last segment holds 4 nodes, with 66 nodes the eighth segment is
    empty. Against the oracle's per-particle solves (FP32 storage: bound 1e-5 relative)."""
    g = build_geometry(wl)
    s = _spm().Solver("cuda:0").set_workload(wl)
    v = np.random.default_rng(5).standard_normal(2 * g.N)
    out = _n(s.precond_apply(_t(v)))
    ref = OP.apply_inverse(g, v)
    e = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"[precond ragged {wl.get('name')}] rel err {e:.2e}", flush=True)
    assert e <= 1e-5


def test_preconditioned_star_solve():
    spm = _spm()
    wl = W.star_and_ellipse()
    plain = spm.Solver("cuda:0").set_workload(wl).solve()
    pc = spm.Solver("cuda:0", precond=spm.SPM_PRECOND_BLOCK).set_workload(wl).solve()
    print(f"[star precond] its {pc['info']['iterations']} (plain {plain['info']['iterations']})", flush=True)
    assert pc["info"]["rel_residual"] <= 1e-10
    assert np.abs(_n(pc["omega"]) - _n(plain["omega"])).max() <= 1e-8
    assert abs(float(pc["mu_eff"].item()) - float(plain["mu_eff"].item())) <= 1e-9 * float(plain["mu_eff"].item())


def test_star_time_stepping_matches_oracle():
    """Forward Euler (Sec. 7) of two three-armed stars and an ellipse."""
    wl = W.star_and_ellipse(gap=5e-2, n_star=128, n_ellipse=96)
    dt, n = 0.02, 3
    c_ref, th_ref, mu_ref = ostep.euler(wl, dt, n, tol=1e-12)
    s = _spm().Solver("cuda:0").set_workload(wl)
    out = s.step(dt, n, 0.0, wl["centers"], wl["theta"])
    print(f"[star step] mu {out['mu_eff']} ref {mu_ref}", flush=True)
    assert np.abs(out["mu_eff"] - mu_ref).max() < 1e-9
    assert np.abs(out["theta"] - th_ref).max() < 1e-9
    e2 = np.array([wl["skew"] - np.floor(wl["skew"] + 0.5) + n * dt, 1.0])
    B = np.array([[1.0, e2[0]], [0.0, 1.0]])
    d = np.linalg.solve(B, (out["centers"] - c_ref).T).T
    assert np.abs(d - np.round(d)).max() < 1e-9


def test_star_shape_checks():
    spm = _spm()
    base = W.two_stars(n_nodes=64)
    for bad in ({"A": 1.0}, {"omega": 2.5}, {"s": -0.1}, {"s": 0.35}):
        wl = dict(base)
        prm = np.array(base["params"], dtype=float)
        col = {"s": 0, "A": 1, "omega": 2}[next(iter(bad))]
        prm[:, col] = next(iter(bad.values()))
        wl["params"] = prm
        with pytest.raises(spm.SpmError) as e:
            spm.Solver("cuda:0").set_workload(wl)
        assert e.value.code == spm.SPM_EINVAL, bad
    # arms that reach into each other: overlap
    wl = W.two_stars(s=0.25, A=0.5, omega=1.0, second_theta=np.pi, n_nodes=64)
    wl = dict(wl, centers=np.array([[-0.2, 0.0], [0.2, 0.0]]))
    with pytest.raises(spm.SpmError) as e:
        spm.Solver("cuda:0").set_workload(wl)
    assert e.value.code == spm.SPM_EOVERLAP


def test_star_cells_in_one_ensemble():
    """Cells of stars, of ellipses and of both kinds solved together (one launch per
    product, per-cell convergence) against the oracle solving each cell alone."""
    from oracle import operator as op
    from oracle import readout as ro
    spm = _spm()
    cells = [W.two_stars(n_nodes=128), W.star_and_ellipse(), W.random_ellipses(5, 0.3, seed=1004, nodes=64),
             W.stars([[0.1, -0.2]], 0.2, 0.3, 3, theta=0.4, n_nodes=96, skew=-0.3)]
    s = spm.Solver("cuda:0").set_cells(cells)
    r = s.solve_cells()
    vel, om, mu = _n(r["vel"]), _n(r["omega"]), _n(r["mu_eff"])
    off = s.part_off
    for k, wl in enumerate(cells):
        prob = op.make_problem(wl)
        x, _ = op.solve(prob, tol=1e-12)
        v, o = ro.velocities(prob, x)
        m = ro.mu_eff(prob, x)
        sl = slice(off[k], off[k + 1])
        sc_v = max(np.abs(v).max(), np.hypot(*prob.geom.e2))
        print(f"[star ensemble] cell {k}: its {r['infos'][k]['iterations']} omega err {np.abs(om[sl] - o).max():.1e} "
              f"mu err {abs(mu[k] - m):.1e}", flush=True)
        assert r["infos"][k]["rel_residual"] <= 1e-10
        assert np.abs(om[sl] - o).max() <= 1e-9 * max(1.0, np.abs(o).max())
        assert np.abs(vel[sl] - v).max() <= 1e-9 * sc_v
        assert abs(mu[k] - m) <= 1e-9 * m
