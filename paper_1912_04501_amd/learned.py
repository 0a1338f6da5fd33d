"""Training and use of the learned warm start (orchestration over the C ABI).

Data: forward-Euler trajectories run by the solver itself (spm_step_record) store,
for every particle at every step, its neighbour features and the body-frame Fourier
coefficients of its solved density. Training: minibatch Adam in the library's
matrix-core kernels (spm_mlp_train); the minibatch order is drawn here from a
seeded generator and passed in. Use: spm_set_network + cfg.x0 = SPM_X0_NETWORK.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import spm as S
from . import workloads as W


def init_params(seed=0):
    """He-normal weights, zero biases, packed as the library expects (FP32)."""
    rng = np.random.default_rng(seed)
    parts = []
    layers = (S.SPM_MLP_IN, S.SPM_MLP_HIDDEN, S.SPM_MLP_HIDDEN, S.SPM_MLP_HIDDEN, S.SPM_MLP_OUT)
    for fi, fo in zip(layers[:-1], layers[1:]):
        parts.append((rng.standard_normal((fo, fi)) * np.sqrt(2.0 / fi)).ravel())
        parts.append(np.zeros(fo))
    return torch.as_tensor(np.concatenate(parts), dtype=torch.float32)


def record_trajectory(wl, steps, dt=0.01, device="cuda:0", **cfg):
    """Run up to `steps` Euler steps from workload wl and return the recorded
    (features [k*n, 33], targets [k*n, 128], completed steps k, infos). A collision
    (SPM_EOVERLAP) ends the trajectory early; the steps before it are kept."""
    s = S.Solver(device, **cfg).set_workload(wl)
    n = s.No
    feat = torch.empty(steps, n, S.SPM_MLP_IN, dtype=torch.float32, device=s.device)
    tgt = torch.empty(steps, n, S.SPM_MLP_OUT, dtype=torch.float32, device=s.device)
    t_io = np.zeros(1)
    c = np.ascontiguousarray(np.asarray(wl["centers"], float).reshape(-1)).copy()
    th = np.ascontiguousarray(wl["theta"], float).copy()
    mus = np.zeros(steps)
    infos = (S.spm_solve_info * steps)()
    rc = S.lib().spm_step_record(s.h, float(dt), int(steps), S._dp(t_io), S._dp(c), S._dp(th), S._dp(mus), infos,
                                 S._fptr(feat), S._fptr(tgt))
    done = steps if rc == 0 else int(round(t_io[0] / dt))
    if rc not in (0, S.SPM_EOVERLAP):
        raise S.SpmError(rc, S.lib().spm_last_error(s.h).decode())
    s.close()
    return (feat[:done].reshape(-1, S.SPM_MLP_IN).clone(), tgt[:done].reshape(-1, S.SPM_MLP_OUT).clone(), done,
            [infos[k].as_dict() for k in range(done)])


def generate(seeds, steps, dt=0.01, device="cuda:0", log=None, lo=25, hi=100, **cfg):
    """Training data from one trajectory per seed (W.trajectory_cell with lo..hi ellipses)."""
    X, T, total = [], [], 0
    for sd in seeds:
        t0 = time.perf_counter()
        f, t, done, _ = record_trajectory(W.trajectory_cell(sd, lo=lo, hi=hi), steps, dt, device, **cfg)
        X.append(f)
        T.append(t)
        total += done
        if log:
            log(f"[learned] trajectory seed {sd}: {done} steps, {f.shape[0]} samples, "
                f"{time.perf_counter() - t0:.1f} s")
    return torch.cat(X), torch.cat(T), total


def train(net, X, T, epochs, batch=256, lr=1e-3, seed=0, mode=S.SPM_MLP_BF16, lr_final=None, log=None):
    """Adam over `epochs` shuffled passes (seeded permutations); a cosine decay to
    lr_final when given. Returns the per-minibatch losses (host)."""
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    nb = n // batch
    out = []
    for e in range(epochs):
        perm = rng.permutation(n)[:nb * batch].astype(np.int32)
        idx = torch.as_tensor(perm, device=X.device)
        cur = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * e / max(1, epochs)))
        losses = net.train(X, T, idx, batch, cur, mode).cpu().numpy()
        out.append(losses)
        if log:
            log(f"[learned] epoch {e}: lr {cur:.2e} loss {losses.mean():.4e}")
    return np.concatenate(out)
