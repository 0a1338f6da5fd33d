"""Forward Euler time stepping of particle centres and angles (Sec. 7).

State s = (centres, angles). At t_n = n dt (computed, not accumulated) the lattice
is e1 = (1, 0), e2 = (s0 + gamma t_n, 1), reduced to skew in [-1/2, 1/2) by the
nearest-integer shift of Sec. 7 (ties by floor(x + 1/2)); centres are wrapped into
the cell, the mobility problem is solved, and

    c_i <- c_i + dt v_i,    theta_i <- theta_i + dt omega_i.

mu_eff(t_n) is recorded for every step.
"""
from __future__ import annotations

import numpy as np

from .operator import make_problem, solve
from .readout import mu_eff, velocities


def euler(wl, dt, n_steps, tol=1e-10, **cfg):
    centers = np.array(wl["centers"], dtype=float)
    theta = np.array(wl["theta"], dtype=float)
    s0 = float(wl["skew"])
    gamma = float(wl.get("gamma", 1.0))
    series = []
    x_prev = None
    for n in range(n_steps):
        t = n * dt
        w = dict(wl, centers=centers, theta=theta, skew=s0 + gamma * t)
        prob = make_problem(w, **cfg)
        x, info = solve(prob, tol=tol, x0=x_prev)
        v, om = velocities(prob, x)
        series.append(mu_eff(prob, x))
        centers = prob.geom.centers + dt * v
        theta = theta + dt * om
        x_prev = x
    return centers, theta, np.array(series)
