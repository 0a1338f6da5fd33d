"""Effective viscosity by contour deformation (spm_effective_viscosity_contour) against the
oracle's contour form on the device's own density: particles across D, a 25-ellipse cell,
the jamming stars and an ensemble of cells with different skews. With the device's proxy
strengths both sides evaluate the same sums (FP64, different order): 1e-12. With the
oracle's own proxy strengths the difference is the proxy solve's rounding (xi agrees to
1e-9 of its largest entry), carried to mu_eff through the correction traction on D."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import periodizer
from oracle import readout as ro
from paper_1912_04501_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "single_ellipse_across_D_skew0.2": lambda: W.single_ellipse(skew=0.2, theta=0.7, center=(0.0, -0.45)),
    "random_25_phi0.3_seed1": lambda: W.random_ellipses(25, 0.3, seed=1),
    "two_stars_s0.25_A0.5_w4": lambda: W.two_stars(omega=4.0),
}


def _n(t):
    return t.detach().cpu().numpy()


def _xi_bound(prob, xi):
    """|d mu_eff| for a change of 1e-9 max|xi| in every proxy strength (correction on D)."""
    _, _, _, xD, nD, wD = ro.contour_points(prob.geom, 16)
    r = xD[:, None, :] - prob.P[None]
    rr = (r * r).sum(-1)
    rn = np.abs((r * nD[:, None, :]).sum(-1))
    sens = (wD[:, None] * np.abs(r[..., 0]) * rn * np.sqrt(rr) / (np.pi * rr * rr)).sum() * 2.0
    return 1e-9 * np.abs(xi).max() * sens / prob.cfg.gamma


def _check_cell(prob, sig, xi_dev, mu_dev, tag):
    a = ro.mu_eff_contour(prob, sig, xi=xi_dev)
    b = ro.mu_eff_contour(prob, sig)
    st = ro.mu_eff(prob, sig)
    bound = 1e-12 + _xi_bound(prob, xi_dev)
    print(f"[contour {tag}] device {mu_dev:.15f} same-xi err {abs(mu_dev - a):.1e} oracle-xi err "
          f"{abs(mu_dev - b):.1e} (bound {bound:.1e}) stresslet diff {abs(mu_dev - st):.1e}", flush=True)
    assert abs(mu_dev - a) < 1e-12
    assert abs(mu_dev - b) < bound
    assert abs(mu_dev - st) < 1e-6                      # the two forms of eq. (mueff), MFS error


@pytest.mark.parametrize("name", list(CASES))
def test_contour_matches_oracle(name):
    from paper_1912_04501_amd import spm
    wl = CASES[name]()
    prob = op.make_problem(wl)
    s = spm.Solver("cuda:0").set_workload(wl)
    print(f"[contour {name}] N {prob.N}", flush=True)
    sig = s.solve()["sigma"]
    mu = _n(s.effective_viscosity_contour(sig))
    xi = _n(s.proxy_strengths(sig))
    _check_cell(prob, _n(sig), xi, mu[0], name)


def test_contour_ensemble_cells():
    from paper_1912_04501_amd import spm
    h = W.c1_h_star()
    cells = [W.random_ellipses(n, 0.3, seed=1000 + k, h_star=h, name=f"cell{k}") for k, n in enumerate((4, 9, 6))]
    cells.append(W.single_ellipse(n_nodes=96, skew=0.37, center=(0.2, 0.44)))
    s = spm.Solver("cuda:0").set_cells(cells)
    sig = _n(s.solve_cells()["sigma"])
    dev = s.proxy_strengths(torch.as_tensor(sig, device="cuda:0"))
    mu = _n(s.effective_viscosity_contour(torch.as_tensor(sig, device="cuda:0")))
    xi = _n(dev)
    M = s.cfg.M
    N = s.N
    n0 = 0
    for k, wl in enumerate(cells):
        prob = op.make_problem(wl)
        n1 = n0 + prob.N
        sk = np.concatenate([sig[n0:n1], sig[N + n0:N + n1]])
        _check_cell(prob, sk, xi[2 * M * k:2 * M * (k + 1)], mu[k], f"cell{k}")
        n0 = n1


def test_contour_quadrature_argument():
    from paper_1912_04501_amd import spm
    wl = W.single_ellipse(n_nodes=64, center=(0.1, 0.47))
    s = spm.Solver("cuda:0").set_workload(wl)
    sig = s.solve()["sigma"]
    a = _n(s.effective_viscosity_contour(sig))[0]
    b = _n(s.effective_viscosity_contour(sig, m=16))[0]
    c = _n(s.effective_viscosity_contour(sig, m=40))[0]
    assert a == b and abs(a - c) < 1e-13
    for bad in (3, 129, -1):
        with pytest.raises(spm.SpmError) as err:
            s.effective_viscosity_contour(sig, m=bad)
        assert err.value.code == spm.SPM_EINVAL


def test_contour_200_ellipses():
    """The bench's 200-ellipse cell (N = 51,200; particles across D) in the bench's solver
    configuration, against the oracle's contour sums on the device's density and strengths."""
    from paper_1912_04501_amd import spm
    wl = W.ellipses_200()
    s = spm.Solver("cuda:0", precision=spm.SPM_FP32_IR, precond=spm.SPM_PRECOND_BLOCK).set_workload(wl)
    r = s.solve()
    sig = r["sigma"]
    mu = _n(s.effective_viscosity_contour(sig))[0]
    xi = _n(s.proxy_strengths(sig))
    prob = op.make_problem(wl)
    a = ro.mu_eff_contour(prob, _n(sig), xi=xi)
    st = _n(r["mu_eff"])[0]
    print(f"[contour 200 ellipses] device {mu:.15f} oracle (same xi) err {abs(mu - a):.1e} stresslet diff "
          f"{abs(mu - st):.1e}", flush=True)
    assert abs(mu - a) < 1e-12
    assert abs(mu - st) < 1e-6
