"""Seeded synthetic workloads: ellipse suspensions in a sheared unit cell.

This module only *generates inputs* (particle tables, lattice skews, random
densities). It holds none of the method's arithmetic: no kernels, no
quadrature, no solver. Both the HIP path and the CPU oracle take their inputs
from here, so the two never share numerical code.

A workload is a dict::

    {"name": str, "skew": float,            # e2 = (skew, 1), e1 = (1, 0), cell centre (0, 0)
     "centers": (No, 2) float64, "theta": (No,), "a": (No,), "b": (No,),
     "n_nodes": (No,) int32, "mu": float, "gamma": float}

Geometry conventions follow the paper's setup (Sec. 2): lattice vectors
e1 = (1, 0), e2 = (gamma t, 1); an ellipse is x(t) = c + R(theta) (a cos t, b sin t).

Recipes:

* ``single_ellipse``: one ellipse a=0.2, b=0.1, theta=0 at the cell centre,
  skew 0, N=128 nodes.
* ``random_ellipses(n, phi, seed, ...)``: n ellipses of equal area phi/n,
  aspect ratio AR ~ U[ar_lo, ar_hi], a = sqrt(area*AR/pi), b = a/AR,
  theta ~ U[0, pi), skew ~ U[0, 1) (reduced later by the library/oracle to
  [-1/2, 1/2), which is the same lattice), centres uniform in lattice
  coordinates, random sequential placement rejecting any candidate whose
  periodic gap to an already placed ellipse is below ``min_gap``.
  Node counts: fixed ``nodes`` if given, else the perimeter rule
  N_i = clamp(8*ceil(P_i / (8 h)), 64, 256) with h = sum(P_i) / target_total.
* ``two_ellipses(d)``: two ellipses with semi-axes (0.25, 0.125) and
  (0.125, 0.25) on a horizontal line, boundary gap d (the paper's two-ellipse
  convergence example, Sec. 8 Example 1).
"""
from __future__ import annotations

import math

import numpy as np

# node density of the 25-ellipse, 5,000-node workload (used by ensembles and
# time stepping, whose cells draw their node counts from the same density)
_C1_TARGET_TOTAL = 5000


def _ellipse_perimeter(a: float, b: float) -> float:
    """Ramanujan's second approximation (rel. error < 1e-9 for AR <= 3); only
    used to pick node counts, never inside the method."""
    h = ((a - b) / (a + b)) ** 2
    return math.pi * (a + b) * (1 + 3 * h / (10 + math.sqrt(4 - 3 * h)))


def node_rule(a, b, h_star, lo=64, hi=256):
    """N_i = clamp(8 ceil(P_i / (8 h*)), lo, hi)."""
    out = []
    for ai, bi in zip(a, b):
        p = _ellipse_perimeter(float(ai), float(bi))
        n = 8 * int(math.ceil(p / (8.0 * h_star)))
        out.append(min(max(n, lo), hi))
    return np.asarray(out, dtype=np.int32)


# ---------------------------------------------------------------------------
# periodic gap test used only by the placement loop
# ---------------------------------------------------------------------------

def _boundary(c, th, a, b, t):
    ct, st = math.cos(th), math.sin(th)
    px = a * np.cos(t)
    py = b * np.sin(t)
    return np.stack([c[0] + ct * px - st * py, c[1] + st * px + ct * py], axis=-1)


def _inside(p, c, th, a, b):
    ct, st = math.cos(th), math.sin(th)
    dx = p[..., 0] - c[0]
    dy = p[..., 1] - c[1]
    u = ct * dx + st * dy
    v = -st * dx + ct * dy
    return (u / a) ** 2 + (v / b) ** 2 < 1.0


def _pair_gap(c1, th1, a1, b1, c2, th2, a2, b2, ns=256):
    """Minimum distance between two ellipse boundaries (<= 0 if they overlap)."""
    t = np.arange(ns) * (2 * math.pi / ns)
    p1 = _boundary(c1, th1, a1, b1, t)
    p2 = _boundary(c2, th2, a2, b2, t)
    if _inside(p1, c2, th2, a2, b2).any() or _inside(p2, c1, th1, a1, b1).any():
        return -1.0
    d2 = ((p1[:, None, :] - p2[None, :, :]) ** 2).sum(-1)
    k = np.unravel_index(np.argmin(d2), d2.shape)
    t1, t2 = t[k[0]], t[k[1]]
    step = 2 * math.pi / ns
    best = math.sqrt(d2[k])
    for _ in range(3):  # local refinement around the best pair
        s = np.linspace(-2 * step, 2 * step, 41)
        q1 = _boundary(c1, th1, a1, b1, t1 + s)
        q2 = _boundary(c2, th2, a2, b2, t2 + s)
        dd = ((q1[:, None, :] - q2[None, :, :]) ** 2).sum(-1)
        kk = np.unravel_index(np.argmin(dd), dd.shape)
        t1, t2 = t1 + s[kk[0]], t2 + s[kk[1]]
        best = min(best, math.sqrt(dd[kk]))
        step = step / 10
    return best


def periodic_min_gap(wl) -> float:
    """Smallest boundary gap over all pairs and the 3x3 lattice images."""
    c, th, a, b = wl["centers"], wl["theta"], wl["a"], wl["b"]
    e1 = np.array([1.0, 0.0])
    e2 = np.array([wl["skew"], 1.0])
    n = len(a)
    g = math.inf
    for i in range(n):
        for j in range(i, n):
            for m in (-1, 0, 1):
                for k in (-1, 0, 1):
                    if i == j and m == 0 and k == 0:
                        continue
                    cj = c[j] + m * e1 + k * e2
                    if np.linalg.norm(c[i] - cj) > a[i] + a[j] + 0.05:
                        continue
                    g = min(g, _pair_gap(c[i], th[i], a[i], b[i], cj, th[j], a[j], b[j]))
    return g


def _place(rng, area, n, ar_lo, ar_hi, skew, min_gap, max_tries=100000):
    e1 = np.array([1.0, 0.0])
    e2 = np.array([skew, 1.0])
    centers, thetas, aa, bb = [], [], [], []
    for _ in range(n):
        ar = rng.uniform(ar_lo, ar_hi)
        a = math.sqrt(area * ar / math.pi)
        b = a / ar
        for _try in range(max_tries):
            al, be = rng.uniform(-0.5, 0.5, size=2)
            c = al * e1 + be * e2
            th = rng.uniform(0.0, math.pi)
            ok = True
            for j in range(len(centers)):
                for m in (-1, 0, 1):
                    for k in (-1, 0, 1):
                        cj = centers[j] + m * e1 + k * e2
                        dist = float(np.linalg.norm(c - cj))
                        if dist > a + aa[j] + min_gap:
                            continue
                        if dist < b + bb[j] + min_gap:
                            ok = False
                            break
                        if _pair_gap(c, th, a, b, cj, thetas[j], aa[j], bb[j]) < min_gap:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                # the ellipse must also clear its own periodic images
                for m in (-1, 0, 1):
                    for k in (-1, 0, 1):
                        if m == 0 and k == 0:
                            continue
                        cj = c + m * e1 + k * e2
                        if float(np.linalg.norm(c - cj)) < 2 * a + min_gap:
                            if _pair_gap(c, th, a, b, cj, th, a, b) < min_gap:
                                ok = False
            if ok:
                centers.append(c)
                thetas.append(th)
                aa.append(a)
                bb.append(b)
                break
        else:
            return None
    return (np.array(centers), np.array(thetas), np.array(aa), np.array(bb))


def random_ellipses(n, phi, seed, ar_lo=1.5, ar_hi=3.0, min_gap=1e-3, nodes=None,
                    target_total=_C1_TARGET_TOTAL, h_star=None, skew=None, name=None,
                    mu=1.0, gamma=1.0):
    rng = np.random.default_rng(seed)
    sk = float(rng.uniform(0.0, 1.0)) if skew is None else float(skew)
    area = phi / n
    for attempt in range(20):
        placed = _place(rng, area, n, ar_lo, ar_hi, sk, min_gap)
        if placed is not None:
            break
    else:  # pragma: no cover - reseeding never needed for the shipped recipes
        raise RuntimeError("random sequential placement failed")
    c, th, a, b = placed
    if nodes is not None:
        nn = np.full(n, int(nodes), dtype=np.int32)
    else:
        if h_star is None:
            per = sum(_ellipse_perimeter(x, y) for x, y in zip(a, b))
            h_star = per / float(target_total)
        nn = node_rule(a, b, h_star)
    return {"name": name or f"random_{n}_phi{phi}_seed{seed}", "skew": sk, "centers": c,
            "theta": th, "a": a, "b": b, "n_nodes": nn, "mu": mu, "gamma": gamma}


def c1_h_star(seed=1):
    """Node spacing of the 25-ellipse, ~5,000-node workload (reused by other recipes)."""
    wl = random_ellipses(25, 0.3, seed, nodes=64)
    per = sum(_ellipse_perimeter(x, y) for x, y in zip(wl["a"], wl["b"]))
    return per / float(_C1_TARGET_TOTAL)


# ---------------------------------------------------------------------------
# named recipes
# ---------------------------------------------------------------------------

def single_ellipse(n_nodes=128, a=0.2, b=0.1, theta=0.0, skew=0.0, center=(0.0, 0.0), mu=1.0, gamma=1.0):
    return {"name": "single_ellipse_128", "skew": float(skew), "centers": np.array([center], dtype=float),
            "theta": np.array([theta], dtype=float), "a": np.array([a], dtype=float),
            "b": np.array([b], dtype=float), "n_nodes": np.array([n_nodes], dtype=np.int32),
            "mu": mu, "gamma": gamma}


def ellipses_25(seed=1):
    """25 ellipses, area fraction 0.3, AR in [1.5, 3], ~5,000 nodes, min gap 1e-3."""
    wl = random_ellipses(25, 0.3, seed, name="ellipses_25_phi0.3")
    return wl


def ellipses_200(seed=2):
    """200 ellipses, area fraction 0.4, 256 nodes each (N = 51,200)."""
    return random_ellipses(200, 0.4, seed, nodes=256, name="ellipses_200_phi0.4_N51200")


def ensemble_cells(n_cells=64, base_seed=1000, h_star=None, lo=4, hi=50, phi=0.3):
    """Independent cells for the batched ensemble: cell c uses seed base_seed + c,
    particle count ~ U{lo..hi}, area fraction phi, node counts from the
    25-ellipse node density."""
    if h_star is None:
        h_star = c1_h_star()
    cells = []
    for c in range(n_cells):
        rng = np.random.default_rng(base_seed + c)
        n = int(rng.integers(lo, hi + 1))
        cells.append(random_ellipses(n, phi, base_seed + c, h_star=h_star, name=f"cell{c}"))
    return cells


def trajectory_cell(seed, lo=25, hi=100, phi=0.3, h_star=None):
    """Initial state of a time-stepping run: n ~ U{lo..hi} ellipses (from the seed) at
    area fraction phi in an unskewed cell (s(0) = 0), node counts from the 25-ellipse
    node density."""
    if h_star is None:
        h_star = c1_h_star()
    n = int(np.random.default_rng(seed).integers(lo, hi + 1))
    return random_ellipses(n, phi, seed, h_star=h_star, skew=0.0, name=f"trajectory{seed}")


def two_ellipses(d, n_nodes=64, skew=0.0):
    """Semi-axes (0.25, 0.125) and (0.125, 0.25) with boundary gap d along x."""
    sep = d + 0.375
    c = np.array([[-sep / 2, 0.0], [sep / 2, 0.0]])
    return {"name": f"two_ellipses_d{d:g}", "skew": float(skew), "centers": c,
            "theta": np.array([0.0, 0.0]), "a": np.array([0.25, 0.125]), "b": np.array([0.125, 0.25]),
            "n_nodes": np.array([n_nodes, n_nodes], dtype=np.int32), "mu": 1.0, "gamma": 1.0}


def stars(centers, s, A, omega, phase=None, theta=None, n_nodes=256, skew=0.0, name="stars"):
    """Smooth star-shaped particles r(t) = s (1 + A cos(omega t + phase)) in the body frame,
    x = c + R(theta) r(t) (cos t, sin t)."""
    c = np.asarray(centers, dtype=float).reshape(-1, 2)
    n = len(c)
    bc = lambda v: np.broadcast_to(np.asarray(v, dtype=float), (n,)).copy()  # noqa: E731
    params = np.stack([bc(s), bc(A), bc(omega), bc(0.0 if phase is None else phase)], axis=1)
    th = bc(0.0 if theta is None else theta)
    return {"name": name, "skew": float(skew), "centers": c, "theta": th, "kind": np.ones(n, dtype=np.int32),
            "params": params, "a": params[:, 0] * (1 + np.abs(params[:, 1])),
            "b": params[:, 0] * (1 - np.abs(params[:, 1])),
            "n_nodes": np.broadcast_to(np.asarray(n_nodes, dtype=np.int32), (n,)).copy(), "mu": 1.0, "gamma": 1.0}


def two_stars(s=0.25, A=0.5, omega=1.0, second_theta=0.0, n_nodes=256):
    """Two star-shaped particles of the Sec. 8 jamming examples, centred at (1/4, 1/4) and
    (3/4, 3/4) of the unit square (here relative to the cell centre), the second turned by
    second_theta."""
    return stars([[-0.25, -0.25], [0.25, 0.25]], s, A, omega, theta=[0.0, second_theta], n_nodes=n_nodes,
                 name=f"two_stars_s{s}_A{A}_w{omega:g}")


def star_and_ellipse(gap=2e-2, s=0.15, A=0.3, omega=3.0, n_star=192, n_ellipse=128, skew=0.2):
    """A three-armed star (r = s (1 + A cos(omega t))) beside an ellipse with semi-axes
    (0.2, 0.1), boundary gap `gap` along x between the star's arm tip and the ellipse's
    vertex: a cell that mixes both particle kinds."""
    rmax = s * (1.0 + abs(A))
    sep = rmax + 0.2 + gap
    c = np.array([[-sep / 2, 0.05], [sep / 2, 0.05]])
    return {"name": f"star_and_ellipse_d{gap:g}", "skew": float(skew), "centers": c,
            "theta": np.array([0.0, 0.0]), "kind": np.array([1, 0], dtype=np.int32),
            "params": np.array([[s, A, omega, 0.0], [0.2, 0.1, 0.0, 0.0]]),
            "a": np.array([rmax, 0.2]), "b": np.array([s * (1.0 - abs(A)), 0.1]),
            "n_nodes": np.array([n_star, n_ellipse], dtype=np.int32), "mu": 1.0, "gamma": 1.0}


def random_stars(n, phi, seed, n_nodes=350, A=0.3, omega=5, min_gap=None, skew=0.0, name=None):
    """n star-shaped "islands" r(t) = s (1 + A cos(omega t + phase)) of one size at area
    fraction phi (area pi s^2 (1 + A^2/2) each), random centres, turns and phases, n_nodes
    nodes each (Sec. 8 Example 2 uses 350). Centres are placed by random sequential addition
    with bounding circles of radius s (1 + A) kept min_gap apart (default s/5) over the 3x3
    periodic images."""
    rng = np.random.default_rng(seed)
    s_ = math.sqrt(phi / (n * math.pi * (1.0 + 0.5 * A * A)))
    R = s_ * (1.0 + A)
    gap = 0.2 * s_ if min_gap is None else min_gap
    e1, e2 = np.array([1.0, 0.0]), np.array([skew, 1.0])
    shifts = np.array([m * e1 + k * e2 for m in (-1, 0, 1) for k in (-1, 0, 1)])
    cs = np.zeros((0, 2))
    for _ in range(n):
        for _try in range(200000):
            al, be = rng.uniform(-0.5, 0.5, size=2)
            c = al * e1 + be * e2
            if len(cs):
                d = np.linalg.norm((cs[:, None, :] + shifts[None]) - c, axis=2).min()
                if d < 2 * R + gap:
                    continue
            if np.linalg.norm(shifts[[0, 1, 2, 3, 5, 6, 7, 8]], axis=1).min() < 2 * R + gap:
                raise ValueError("islands larger than the cell")
            cs = np.vstack([cs, c])
            break
        else:
            raise ValueError("could not place the islands")
    return stars(cs, s_, A, omega, phase=rng.uniform(0, 2 * math.pi, n), theta=rng.uniform(0, 2 * math.pi, n),
                 n_nodes=n_nodes, skew=skew, name=name or f"islands_{n}_phi{phi}_N{n * n_nodes}")


def random_density(n_total, seed=7):
    """sigma ~ N(0, 1), SoA [sigma_1(0..N-1), sigma_2(0..N-1)]."""
    return np.random.default_rng(seed).standard_normal(2 * int(n_total))


def total_nodes(wl) -> int:
    return int(np.sum(wl["n_nodes"]))
