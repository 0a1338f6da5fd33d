"""End-to-end pins of the oracle solver: spectral convergence in N for two close
ellipses (Sec. 8 Example 1), GMRES against LU with close pairs, and first-order
convergence of forward Euler (Sec. 7; Sec. 8 Example 3 table)."""
import numpy as np
import pytest

from oracle import operator as op
from oracle import readout, step
from paper_1912_04501_amd import workloads as W


def _solve(wl, **kw):
    prob = op.make_problem(wl, **kw)
    x, info = op.solve(prob, tol=1e-13, maxiter=400)
    v, om = readout.velocities(prob, x)
    return prob, x, v, om


@pytest.mark.parametrize("d,Ns,Nref,tol", [(1e-1, (24, 48, 72), 160, 1e-10), (1e-2, (64, 128, 256), 384, 1e-12)])
def test_two_ellipse_spectral_convergence(d, Ns, Nref, tol):
    """Two ellipses (0.25, 0.125) and (0.125, 0.25) at gap d: the angular velocities
    and the velocity difference converge spectrally in the nodes per ellipse,
    with the onset moving to larger N as d shrinks."""
    ref = _solve(W.two_ellipses(d, n_nodes=Nref))
    errs = []
    for N in Ns:
        r = _solve(W.two_ellipses(d, n_nodes=N))
        e_om = np.abs(r[3] - ref[3]).max()
        e_v = np.abs((r[2][1] - r[2][0]) - (ref[2][1] - ref[2][0])).max()
        errs.append(max(e_om, e_v))
    assert errs[-1] < tol
    assert all(errs[k + 1] < 0.01 * errs[k] for k in range(len(errs) - 1))  # onset ~1/sqrt(d)


def test_gmres_matches_lu_with_close_pairs():
    wl = W.two_ellipses(3e-2, n_nodes=128)     # resolved: gap 3e-2 < 10 h, so close pairs are active
    prob = op.make_problem(wl)
    assert len(prob.pairs) > 0
    x, info = op.solve(prob, tol=1e-13)
    xl, _ = op.solve(prob, method="lu")
    assert np.abs(x - xl).max() < 1e-10 * np.abs(xl).max()
    # the solution satisfies the force- and torque-free constraints (Sec. 5, eqs. BIEconstraint)
    g = prob.geom
    s2 = op.to2(xl)
    for i in range(g.No):
        sl = g.particle_slice(i)
        rel = g.x[sl] - g.centers[i]
        F = (g.w[sl, None] * s2[sl]).sum(0)
        tq = (g.w[sl] * (-rel[:, 1] * s2[sl, 0] + rel[:, 0] * s2[sl, 1])).sum()
        assert np.abs(F).max() < 1e-10 and abs(tq) < 1e-10


def test_euler_first_order():
    """Forward Euler self-convergence of mu_eff(t) (Sec. 7; the paper's Table on
    mu_eff shows order 1.00 on [0, 1]): successive differences halve with dt."""
    wl = W.random_ellipses(3, 0.12, seed=8, nodes=64, skew=0.0)   # min gap 0.02: resolved
    T = 0.4
    finals = []
    for n in (4, 8, 16):
        _, _, mus = step.euler(wl, T / n, n + 1)
        finals.append(mus[-1])
    d1 = abs(finals[1] - finals[0])
    d2 = abs(finals[2] - finals[1])
    order = np.log2(d1 / d2)
    assert 0.9 < order < 1.15     # observed 1.03
