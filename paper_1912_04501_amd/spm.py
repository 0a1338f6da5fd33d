"""Thin Python binding of libspm.so (the C ABI in include/spm.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels. PyTorch provides device memory (through the allocator callbacks given to
``spm_create``, so the library's workspace lives in torch's caching allocator) and
the stream (torch's current stream). The binding fails loudly if the library is
missing; there is no CPU fallback.

Function names mirror the C ABI; ``Solver`` wraps a handle for convenience.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspm.so")

SPM_OK, SPM_EINVAL, SPM_EOVERLAP, SPM_ENOCONV, SPM_EHIP, SPM_ENOMEM, SPM_ESTATE = 0, -1, -2, -3, -4, -5, -6
SPM_FP64, SPM_FP32, SPM_FP32_IR, SPM_FP32_RELAXED = 0, 1, 2, 3
SPM_X0_ZERO, SPM_X0_PREVIOUS, SPM_X0_NETWORK = 0, 1, 2
SPM_PRECOND_NONE, SPM_PRECOND_BLOCK = 0, 1
SPM_NEAR_DIRECT, SPM_NEAR_FMM = 0, 1
SPM_NEAR_SET_3X3, SPM_NEAR_SET_DILATED = 0, 1
SPM_MLP_IN, SPM_MLP_HIDDEN, SPM_MLP_OUT, SPM_MLP_NPARAMS = 33, 256, 128, 173184
SPM_MLP_BF16, SPM_MLP_FP32 = 0, 1
_ERRNAMES = {-1: "SPM_EINVAL", -2: "SPM_EOVERLAP", -3: "SPM_ENOCONV", -4: "SPM_EHIP", -5: "SPM_ENOMEM",
             -6: "SPM_ESTATE"}


class spm_config(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("gamma", ctypes.c_double), ("M", ctypes.c_int32),
                ("R_proxy", ctypes.c_double), ("m_wall", ctypes.c_int32), ("close_factor", ctypes.c_double),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("min_gap", ctypes.c_double), ("rcond", ctypes.c_double),
                ("use_graph", ctypes.c_int32), ("poll_every", ctypes.c_int32), ("x0", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("learned_max_iter", ctypes.c_int32), ("relax_tol", ctypes.c_double),
                ("near_method", ctypes.c_int32), ("fmm_order", ctypes.c_int32),
                ("node_spacing", ctypes.c_double), ("relax_safety", ctypes.c_double),
                ("learned_accept", ctypes.c_double), ("near_set", ctypes.c_int32)]


class spm_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("fp64_matvecs", ctypes.c_int32),
                ("fp32_matvecs", ctypes.c_int32), ("n_close_pairs", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("seconds_setup", ctypes.c_double), ("seconds_solve", ctypes.c_double),
                ("seconds_readout", ctypes.c_double), ("fallback", ctypes.c_int32),
                ("first_iterations", ctypes.c_int32), ("min_gap", ctypes.c_double),
                ("guess_rejected", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


class SpmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load libspm.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run paper_1912_04501_amd.build.build() (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    d = ctypes.POINTER(ctypes.c_double)
    i32 = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "spm_default_config": (None, [ctypes.POINTER(spm_config)]),
        "spm_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.POINTER(spm_config), P, ALLOC_FN, FREE_FN, P]),
        "spm_destroy": (None, [P]),
        "spm_last_error": (ctypes.c_char_p, [P]),
        "spm_set_lattice": (ctypes.c_int, [P, d, d, d]),
        "spm_set_ellipses": (ctypes.c_int, [P, ctypes.c_int32, d, d, d, d, i32]),
        "spm_num_nodes": (ctypes.c_int, [P, i64]),
        "spm_num_particles": (ctypes.c_int, [P, i32]),
        "spm_get_nodes": (ctypes.c_int, [P, P, P, P, P, P]),
        "spm_get_centers": (ctypes.c_int, [P, d]),
        "spm_apply": (ctypes.c_int, [P, P, P, ctypes.c_int32]),
        "spm_rhs": (ctypes.c_int, [P, P]),
        "spm_solve": (ctypes.c_int, [P, P, P, P, P, P, ctypes.POINTER(spm_solve_info)]),
        "spm_velocities": (ctypes.c_int, [P, P, P, P]),
        "spm_effective_viscosity": (ctypes.c_int, [P, P, P]),
        "spm_effective_viscosity_contour": (ctypes.c_int, [P, P, ctypes.c_int32, P]),
        "spm_fmm_stats": (ctypes.c_int, [P, P, P, P, P]),
        "spm_step": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_int32, d, d, d, d,
                                    ctypes.POINTER(spm_solve_info)]),
        "spm_near_traction": (ctypes.c_int, [P, P, P, ctypes.c_int32]),
        "spm_close_correction": (ctypes.c_int, [P, P, P, ctypes.c_int32]),
        "spm_proxy_strengths": (ctypes.c_int, [P, P, P]),
        "spm_close_pairs": (ctypes.c_int, [P, i64, i32, i32, i32, ctypes.c_int64]),
        "spm_proxy_pinv": (ctypes.c_int, [P, d]),
        "spm_proxy_svd": (ctypes.c_int, [P, d, d, i32]),
        "spm_set_cells": (ctypes.c_int, [P, ctypes.c_int32, d, i32, d, d, d, d, i32]),
        "spm_set_cells_shapes": (ctypes.c_int, [P, ctypes.c_int32, d, i32, d, d, i32, d, i32]),
        "spm_eval_field": (ctypes.c_int, [P, P, ctypes.c_int64, P, P, P, P]),
        "spm_num_cells": (ctypes.c_int, [P, i32]),
        "spm_solve_cells": (ctypes.c_int, [P, P, P, P, P, P, ctypes.POINTER(spm_solve_info), d]),
        "spm_solve_batch": (ctypes.c_int, [P, ctypes.c_int32, d, i32, d, d, d, d, i32, P, P, P,
                                           ctypes.POINTER(spm_solve_info), d]),
        "spm_autotune": (ctypes.c_int, [P, ctypes.c_char_p, d]),
        "spm_get_launch": (ctypes.c_int, [P, ctypes.c_int32, i32]),
        "spm_set_launch": (ctypes.c_int, [P, ctypes.c_int32, i32]),
        "spm_profile": (ctypes.c_int, [P, ctypes.c_int32]),
        "spm_profile_read": (ctypes.c_int, [P, ctypes.c_int32, d, i64, d]),
        "spm_precond_apply": (ctypes.c_int, [P, P, P]),
        "spm_features": (ctypes.c_int, [P, P]),
        "spm_features_f32": (ctypes.c_int, [P, P]),
        "spm_density_modes": (ctypes.c_int, [P, P, P]),
        "spm_warm_start": (ctypes.c_int, [P, P, P]),
        "spm_set_network": (ctypes.c_int, [P, P]),
        "spm_learned_guess": (ctypes.c_int, [P, P]),
        "spm_step_record": (ctypes.c_int, [P, ctypes.c_double, ctypes.c_int32, d, d, d, d,
                                           ctypes.POINTER(spm_solve_info), P, P]),
        "spm_mlp_create": (ctypes.c_int, [ctypes.POINTER(P), P, ALLOC_FN, FREE_FN, P]),
        "spm_mlp_destroy": (None, [P]),
        "spm_mlp_last_error": (ctypes.c_char_p, [P]),
        "spm_mlp_set_params": (ctypes.c_int, [P, P]),
        "spm_mlp_get_params": (ctypes.c_int, [P, P]),
        "spm_mlp_forward": (ctypes.c_int, [P, P, ctypes.c_int64, P, ctypes.c_int32]),
        "spm_mlp_loss_grad": (ctypes.c_int, [P, P, P, ctypes.c_int64, ctypes.c_int32, P, d]),
        "spm_mlp_train": (ctypes.c_int, [P, P, P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_float, ctypes.c_int32, P]),
        "spm_mlp_set_weights": (ctypes.c_int, [P, P, P, ctypes.c_int64]),
        "spm_near_traction_noalloc": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_double, P, P, P, P, P, P,
                                                     ctypes.c_int32, P]),
        "spm_mlp_backward": (ctypes.c_int, [P, P, P, ctypes.c_int64, P, ctypes.c_int32]),
        "spm_mlp_adam_step": (ctypes.c_int, [P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                             ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def default_config(**kw) -> spm_config:
    c = spm_config()
    lib().spm_default_config(ctypes.byref(c))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ptr(t, dtype=torch.float64):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _fptr(t):
    return _ptr(t, torch.float32)


def _iptr(t):
    return _ptr(t, torch.int32)


class _TorchAlloc:
    """Allocator callbacks backed by torch's caching allocator."""

    def __init__(self, device):
        self.device = device
        self.blocks = {}

        def _alloc(nbytes, stream, ctx):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, stream, ctx):
            self.blocks.pop(ptr, None)

        self.alloc_cb = ALLOC_FN(_alloc)
        self.free_cb = FREE_FN(_free)


SPM_NOALLOC_MAX_N = 131072


def near_traction_noalloc(x, y, nx, ny, w, sigma, skew, precision=SPM_FP64, out=None):
    """spm_near_traction_noalloc on torch's current stream: the near-image traction sum of one
    cell from its node arrays (device FP64 tensors [n], sigma [2n]) without any allocation in
    the library. Returns out [2n] (allocated here by torch when not given)."""
    n = x.numel()
    if out is None:
        out = torch.empty(2 * n, dtype=torch.float64, device=x.device)
    st = torch.cuda.current_stream(x.device)
    rc = lib().spm_near_traction_noalloc(ctypes.c_void_p(st.cuda_stream), n, float(skew), _ptr(x), _ptr(y),
                                         _ptr(nx), _ptr(ny), _ptr(w), _ptr(sigma), int(precision), _ptr(out))
    if rc != 0:
        raise SpmError(rc, "spm_near_traction_noalloc failed")
    return out


class MLP:
    """The warm-start network (spm_mlp_*): parameters, forward, gradients, Adam training."""

    def __init__(self, device="cuda"):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required (no CPU fallback)")
        self.device = torch.device(device)
        self._mem = _TorchAlloc(self.device)
        self._stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = lib().spm_mlp_create(ctypes.byref(h), ctypes.c_void_p(self._stream.cuda_stream), self._mem.alloc_cb,
                                  self._mem.free_cb, None)
        if rc != 0:
            raise SpmError(rc, "spm_mlp_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().spm_mlp_destroy(self.h)
            self.h = None
            self._mem.blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise SpmError(rc, lib().spm_mlp_last_error(self.h).decode())

    def set_params(self, params):
        p = params.to(device=self.device, dtype=torch.float32).contiguous()
        if p.numel() != SPM_MLP_NPARAMS:
            raise ValueError("wrong parameter count")
        self._check(lib().spm_mlp_set_params(self.h, _fptr(p)))

    def get_params(self):
        p = torch.empty(SPM_MLP_NPARAMS, dtype=torch.float32, device=self.device)
        self._check(lib().spm_mlp_get_params(self.h, _fptr(p)))
        return p

    def forward(self, x, mode=SPM_MLP_BF16):
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        y = torch.empty(x.shape[0], SPM_MLP_OUT, dtype=torch.float32, device=self.device)
        self._check(lib().spm_mlp_forward(self.h, _fptr(x), x.shape[0], _fptr(y), int(mode)))
        return y

    def loss_grad(self, x, t, mode=SPM_MLP_BF16):
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        t = t.to(device=self.device, dtype=torch.float32).contiguous()
        g = torch.empty(SPM_MLP_NPARAMS, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        self._check(lib().spm_mlp_loss_grad(self.h, _fptr(x), _fptr(t), x.shape[0], int(mode), _fptr(g),
                                            ctypes.byref(loss)))
        return loss.value, g

    def set_weights(self, params_bf16=None, master=None):
        """spm_mlp_set_weights: bfloat16 weights (a torch.bfloat16 tensor) and/or the FP32 master."""
        pb = None if params_bf16 is None else params_bf16.to(device=self.device).contiguous()
        pm = None if master is None else master.to(device=self.device, dtype=torch.float32).contiguous()
        if pb is not None and pb.dtype != torch.bfloat16:
            raise TypeError("params_bf16 must be a torch.bfloat16 tensor")
        self._check(lib().spm_mlp_set_weights(self.h, None if pb is None else ctypes.c_void_p(pb.data_ptr()),
                                              None if pm is None else _fptr(pm), SPM_MLP_NPARAMS))

    def backward(self, x, dy, mode=SPM_MLP_BF16):
        """Gradient of sum(dy * MLP(x)) with respect to the packed parameters."""
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        dy = dy.to(device=self.device, dtype=torch.float32).contiguous()
        g = torch.empty(SPM_MLP_NPARAMS, dtype=torch.float32, device=self.device)
        self._check(lib().spm_mlp_backward(self.h, _fptr(x), _fptr(dy), x.shape[0], _fptr(g), int(mode)))
        return g

    def adam_step(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
        g = grad.to(device=self.device, dtype=torch.float32).contiguous()
        self._check(lib().spm_mlp_adam_step(self.h, _fptr(g), float(lr), float(beta1), float(beta2), float(eps),
                                            int(step)))

    def train(self, x, t, idx, batch, lr, mode=SPM_MLP_BF16):
        """Adam steps over the minibatches idx.view(-1, batch) (device int32)."""
        nb = idx.numel() // batch
        losses = torch.empty(nb, dtype=torch.float32, device=self.device)
        self._check(lib().spm_mlp_train(self.h, _fptr(x), _fptr(t), x.shape[0], _iptr(idx), nb, int(batch),
                                        float(lr), int(mode), _fptr(losses)))
        return losses


class Solver:
    """One handle of the C ABI; device memory from torch, kernels on torch's current stream."""

    def __init__(self, device="cuda", **cfg):
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required (no CPU fallback)")
        self.device = torch.device(device)
        self.cfg = default_config(**cfg)
        self._mem = _TorchAlloc(self.device)
        self._stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = lib().spm_create(ctypes.byref(h), ctypes.byref(self.cfg), ctypes.c_void_p(self._stream.cuda_stream),
                              self._mem.alloc_cb, self._mem.free_cb, None)
        if rc != 0:
            raise SpmError(rc, "spm_create failed (bad config?)")
        self.h = h
        self.N = 0
        self.No = 0
        self.C = 0

    def close(self):
        if getattr(self, "h", None):
            lib().spm_destroy(self.h)
            self.h = None
            self._mem.blocks.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=()):
        if rc != 0 and rc not in allow:
            raise SpmError(rc, lib().spm_last_error(self.h).decode())
        return rc

    # --- setup -------------------------------------------------------------
    def set_lattice(self, skew, center=(0.0, 0.0)):
        e1 = np.array([1.0, 0.0])
        e2 = np.array([float(skew), 1.0])
        c = np.array(center, dtype=float)
        self._check(lib().spm_set_lattice(self.h, _dp(e1), _dp(e2), _dp(c)))

    def set_ellipses(self, centers, theta, a, b, n_nodes=None):
        """n_nodes None: the library's perimeter rule."""
        c = np.ascontiguousarray(np.asarray(centers, dtype=float).reshape(-1))
        th = np.ascontiguousarray(theta, dtype=float)
        aa = np.ascontiguousarray(a, dtype=float)
        bb = np.ascontiguousarray(b, dtype=float)
        nn = None if n_nodes is None else np.ascontiguousarray(n_nodes, dtype=np.int32)
        self._check(lib().spm_set_ellipses(self.h, len(th), _dp(c), _dp(th), _dp(aa), _dp(bb),
                                           None if nn is None else nn.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        self.C = 1
        self._refresh_sizes()

    def _refresh_sizes(self):
        n = ctypes.c_int64()
        self._check(lib().spm_num_nodes(self.h, ctypes.byref(n)))
        self.N = int(n.value)
        k = ctypes.c_int32()
        self._check(lib().spm_num_particles(self.h, ctypes.byref(k)))
        self.No = int(k.value)

    def set_workload(self, wl):
        if "kind" in wl:
            self.set_cells([wl])
            return self
        self.set_lattice(wl["skew"])
        self.set_ellipses(wl["centers"], wl["theta"], wl["a"], wl["b"], wl["n_nodes"])
        return self

    @staticmethod
    def _shape_arrays(c):
        """(kind, params [n, 4]) of one workload: stars carry their own, ellipses (a, b, 0, 0)."""
        n = len(c["theta"])
        if "kind" in c:
            return np.asarray(c["kind"], np.int32), np.asarray(c["params"], float).reshape(n, 4)
        prm = np.zeros((n, 4))
        prm[:, 0] = c["a"]
        prm[:, 1] = c["b"]
        return np.zeros(n, np.int32), prm

    def set_cells(self, cells):
        """An ensemble: a list of workload dicts, one per independent cell (n_nodes None in
        every cell: the library's perimeter rule)."""
        skews = np.array([float(c["skew"]) for c in cells])
        counts = [len(c["theta"]) for c in cells]
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
        cen = np.ascontiguousarray(np.concatenate([np.asarray(c["centers"], float) for c in cells]).reshape(-1))
        th = np.ascontiguousarray(np.concatenate([np.asarray(c["theta"], float) for c in cells]))
        if all(c.get("n_nodes") is None for c in cells):
            nn = None
        else:
            nn = np.ascontiguousarray(np.concatenate([np.asarray(c["n_nodes"]) for c in cells]).astype(np.int32))
        ip = lambda a: None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
        if any("kind" in c for c in cells):
            shapes = [self._shape_arrays(c) for c in cells]
            kind = np.ascontiguousarray(np.concatenate([k for k, _ in shapes]).astype(np.int32))
            prm = np.ascontiguousarray(np.concatenate([p for _, p in shapes]).reshape(-1))
            self._check(lib().spm_set_cells_shapes(self.h, len(cells), _dp(skews), ip(off), _dp(cen), _dp(th),
                                                   ip(kind), _dp(prm), ip(nn)))
        else:
            aa = np.ascontiguousarray(np.concatenate([np.asarray(c["a"], float) for c in cells]))
            bb = np.ascontiguousarray(np.concatenate([np.asarray(c["b"], float) for c in cells]))
            self._check(lib().spm_set_cells(self.h, len(cells), _dp(skews), ip(off), _dp(cen), _dp(th), _dp(aa),
                                            _dp(bb), ip(nn)))
        n = ctypes.c_int64()
        self._check(lib().spm_num_nodes(self.h, ctypes.byref(n)))
        self.N = int(n.value)
        self.No = int(off[-1])
        self.C = len(cells)
        self.part_off = off
        return self

    def solve_cells(self, sigma0=None, allow_noconv=False):
        """Solve the cells set by set_cells (spm_solve_cells)."""
        C = getattr(self, "C", 1)
        sig = self._vec(2 * self.N)
        vel = self._vec(2 * self.No)
        om = self._vec(self.No)
        mu = self._vec(C)
        infos = (spm_solve_info * C)()
        lat = np.zeros(C)
        rc = lib().spm_solve_cells(self.h, _ptr(sigma0), _ptr(sig), _ptr(vel), _ptr(om), _ptr(mu), infos, _dp(lat))
        self._check(rc, allow=(SPM_ENOCONV,) if allow_noconv else ())
        return {"sigma": sig, "vel": vel.view(-1, 2), "omega": om, "mu_eff": mu,
                "infos": [i.as_dict() for i in infos], "latency_s": lat}

    def solve_batch(self, lattices, part_offsets, centers, theta, a, b, n_nodes=None, allow_noconv=False):
        """One call: set and solve an ensemble of ellipse cells (spm_solve_batch). lattices
        [C, 6] = e1, e2, cell centre per cell; part_offsets [C + 1]; n_nodes None: the
        perimeter rule."""
        lat = np.ascontiguousarray(np.asarray(lattices, dtype=np.float64).reshape(-1))
        off = np.ascontiguousarray(np.asarray(part_offsets, dtype=np.int32))
        C = len(off) - 1
        n = int(off[-1])
        cen = np.ascontiguousarray(np.asarray(centers, dtype=np.float64).reshape(-1))
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        aa = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
        bb = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
        nn = None if n_nodes is None else np.ascontiguousarray(np.asarray(n_nodes, dtype=np.int32))
        ip = lambda v: None if v is None else v.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
        vel = self._vec(2 * n)
        om = self._vec(n)
        mu = self._vec(C)
        infos = (spm_solve_info * C)()
        latency = np.zeros(C)
        rc = lib().spm_solve_batch(self.h, C, _dp(lat), ip(off), _dp(cen), _dp(th), _dp(aa), _dp(bb), ip(nn),
                                   _ptr(vel), _ptr(om), _ptr(mu), infos, _dp(latency))
        self._check(rc, allow=(SPM_ENOCONV,) if allow_noconv else ())
        self.C = C
        self._refresh_sizes()
        return {"vel": vel.view(-1, 2), "omega": om, "mu_eff": mu, "infos": [i.as_dict() for i in infos],
                "latency_s": latency}

    def _vec(self, n):
        return torch.empty(int(n), dtype=torch.float64, device=self.device)

    # --- calls ---------------------------------------------------------------
    def nodes(self):
        out = [self._vec(self.N) for _ in range(5)]
        self._check(lib().spm_get_nodes(self.h, *[_ptr(t) for t in out]))
        return out

    def centers(self):
        c = np.zeros(2 * self.No)
        self._check(lib().spm_get_centers(self.h, _dp(c)))
        return c.reshape(-1, 2)

    def apply(self, sigma, precision=SPM_FP64, out=None):
        out = self._vec(2 * self.N) if out is None else out
        self._check(lib().spm_apply(self.h, _ptr(sigma), _ptr(out), precision))
        return out

    def rhs(self):
        out = self._vec(2 * self.N)
        self._check(lib().spm_rhs(self.h, _ptr(out)))
        return out

    def solve(self, sigma0=None, allow_noconv=False):
        sig = self._vec(2 * self.N)
        vel = self._vec(2 * self.No)
        om = self._vec(self.No)
        mu = self._vec(getattr(self, "C", 1))
        info = spm_solve_info()
        rc = lib().spm_solve(self.h, _ptr(sigma0), _ptr(sig), _ptr(vel), _ptr(om), _ptr(mu), ctypes.byref(info))
        self._check(rc, allow=(SPM_ENOCONV,) if allow_noconv else ())
        return {"sigma": sig, "vel": vel.view(-1, 2), "omega": om, "mu_eff": mu, "info": info.as_dict()}

    def velocities(self, sigma):
        vel = self._vec(2 * self.No)
        om = self._vec(self.No)
        self._check(lib().spm_velocities(self.h, _ptr(sigma), _ptr(vel), _ptr(om)))
        return vel.view(-1, 2), om

    def eval_field(self, sigma, targets):
        """Flow velocity [n, 2] and pressure [n] at targets [n, 2] (array-like) for a solved density."""
        pts = torch.as_tensor(np.ascontiguousarray(np.asarray(targets, dtype=np.float64).reshape(-1, 2)),
                              device=self.device)
        xt = pts[:, 0].contiguous()
        yt = pts[:, 1].contiguous()
        n = int(xt.numel())
        u = self._vec(2 * n)
        p = self._vec(n)
        self._check(lib().spm_eval_field(self.h, _ptr(sigma), n, _ptr(xt), _ptr(yt), _ptr(u), _ptr(p)))
        return torch.stack([u[:n], u[n:]], dim=1), p

    def effective_viscosity(self, sigma):
        mu = self._vec(self.C)
        self._check(lib().spm_effective_viscosity(self.h, _ptr(sigma), _ptr(mu)))
        return mu

    def fmm_stats(self):
        """Quadtree of the FMM near sum: levels, expansion terms, direct pairs, M2L translations."""
        lv, od = ctypes.c_int32(), ctypes.c_int32()
        pp, ml = ctypes.c_double(), ctypes.c_double()
        self._check(lib().spm_fmm_stats(self.h, ctypes.byref(lv), ctypes.byref(od), ctypes.byref(pp), ctypes.byref(ml)))
        return {"levels": lv.value, "order": od.value, "p2p_pairs": pp.value, "m2l": ml.value}

    def effective_viscosity_contour(self, sigma, m=0):
        """mu_eff of every cell by contour deformation; m Gauss-Legendre nodes per cell edge (0: 16)."""
        mu = self._vec(self.C)
        self._check(lib().spm_effective_viscosity_contour(self.h, _ptr(sigma), int(m), _ptr(mu)))
        return mu

    def step(self, dt, n_steps, t, centers, theta, record=False):
        t_io = np.array([float(t)])
        c = np.ascontiguousarray(np.asarray(centers, dtype=float).reshape(-1)).copy()
        th = np.ascontiguousarray(theta, dtype=float).copy()
        mus = np.zeros(int(n_steps))
        infos = (spm_solve_info * int(n_steps))()
        feat = tgt = None
        if record:
            feat = torch.empty(int(n_steps), self.No, SPM_MLP_IN, dtype=torch.float32, device=self.device)
            tgt = torch.empty(int(n_steps), self.No, SPM_MLP_OUT, dtype=torch.float32, device=self.device)
        self._check(lib().spm_step_record(self.h, float(dt), int(n_steps), _dp(t_io), _dp(c), _dp(th), _dp(mus),
                                          infos, _fptr(feat), _fptr(tgt)))
        out = {"t": float(t_io[0]), "centers": c.reshape(-1, 2), "theta": th, "mu_eff": mus,
               "infos": [i.as_dict() for i in infos]}
        if record:
            out["features"] = feat
            out["targets"] = tgt
        return out

    # --- block preconditioner and learned warm start ----------------------------
    def precond_apply(self, v):
        out = self._vec(2 * self.N)
        self._check(lib().spm_precond_apply(self.h, _ptr(v), _ptr(out)))
        return out

    def features(self):
        f = torch.empty(self.No, SPM_MLP_IN, dtype=torch.float32, device=self.device)
        self._check(lib().spm_features_f32(self.h, _fptr(f)))
        return f

    def features_bf16(self):
        f = torch.empty(self.No, SPM_MLP_IN, dtype=torch.bfloat16, device=self.device)
        self._check(lib().spm_features(self.h, ctypes.c_void_p(f.data_ptr())))
        return f

    def density_modes(self, sigma):
        m = torch.empty(self.No, SPM_MLP_OUT, dtype=torch.float32, device=self.device)
        self._check(lib().spm_density_modes(self.h, _ptr(sigma), _fptr(m)))
        return m

    def warm_start(self, modes):
        out = self._vec(2 * self.N)
        m = modes.to(device=self.device, dtype=torch.float32).contiguous()
        self._check(lib().spm_warm_start(self.h, _fptr(m), _ptr(out)))
        return out

    def set_network(self, net):
        self._net = net
        self._check(lib().spm_set_network(self.h, None if net is None else net.h))

    def learned_guess(self):
        out = self._vec(2 * self.N)
        self._check(lib().spm_learned_guess(self.h, _ptr(out)))
        return out

    # --- stage entry points ----------------------------------------------------
    def near_traction(self, sigma, precision=SPM_FP64):
        out = self._vec(2 * self.N)
        self._check(lib().spm_near_traction(self.h, _ptr(sigma), _ptr(out), precision))
        return out

    def close_correction(self, sigma, precision=SPM_FP64):
        out = self._vec(2 * self.N)
        self._check(lib().spm_close_correction(self.h, _ptr(sigma), _ptr(out), precision))
        return out

    def proxy_strengths(self, sigma):
        out = self._vec(2 * self.cfg.M * getattr(self, "C", 1))
        self._check(lib().spm_proxy_strengths(self.h, _ptr(sigma), _ptr(out)))
        return out

    def close_pairs(self):
        n = ctypes.c_int64()
        self._check(lib().spm_close_pairs(self.h, ctypes.byref(n), None, None, None, 0))
        k = int(n.value)
        t = np.zeros(max(k, 1), dtype=np.int32)
        q = np.zeros(max(k, 1), dtype=np.int32)
        s = np.zeros(max(k, 1), dtype=np.int32)
        ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))  # noqa: E731
        self._check(lib().spm_close_pairs(self.h, ctypes.byref(n), ip(t), ip(q), ip(s), max(k, 1)))
        return np.stack([t[:k], q[:k], s[:k]], axis=1).astype(np.int64)

    def autotune(self, cache_path=None):
        ms = np.zeros(2)
        p = None if cache_path is None else str(cache_path).encode()
        self._check(lib().spm_autotune(self.h, p, _dp(ms)))
        return {"fp64_ms": float(ms[0]), "fp32_ms": float(ms[1]),
                "fp64": self.get_launch(SPM_FP64), "fp32": self.get_launch(SPM_FP32)}

    def get_launch(self, precision):
        c = np.zeros(4, dtype=np.int32)
        self._check(lib().spm_get_launch(self.h, int(precision), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return {"block": int(c[0]), "tpt": int(c[1]), "tile": int(c[2]), "wg_per_cu": int(c[3])}

    def set_launch(self, precision, block, tpt, tile, wg_per_cu=0):
        c = np.array([block, tpt, tile, wg_per_cu], dtype=np.int32)
        self._check(lib().spm_set_launch(self.h, int(precision), c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))

    def profile(self, enable=True):
        self._check(lib().spm_profile(self.h, 1 if enable else 0))

    def profile_read(self, kernel):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        pairs = ctypes.c_double()
        self._check(lib().spm_profile_read(self.h, int(kernel), ctypes.byref(ms), ctypes.byref(n),
                                           ctypes.byref(pairs)))
        return {"ms": ms.value, "launches": int(n.value), "pairs": pairs.value}

    def proxy_svd(self):
        M, m, C = self.cfg.M, self.cfg.m_wall, getattr(self, "C", 1)
        Q = np.zeros(C * 2 * M * 8 * m)
        sv = np.zeros(C * 2 * M)
        sw = np.zeros(C, dtype=np.int32)
        self._check(lib().spm_proxy_svd(self.h, _dp(Q), _dp(sv), sw.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return Q.reshape(C, 8 * m, 2 * M), sv.reshape(C, 2 * M), sw

    def proxy_pinv(self):
        M, m, C = self.cfg.M, self.cfg.m_wall, getattr(self, "C", 1)
        out = np.zeros(C * 2 * M * 8 * m)
        self._check(lib().spm_proxy_pinv(self.h, _dp(out)))
        return out.reshape(C, 2 * M, 8 * m)
