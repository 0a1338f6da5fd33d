"""The allocation-free near sum (spm_near_traction_noalloc) against the handle-based
spm_near_traction on the same nodes and density: two calls in a row, the second on a smaller
cell, in FP64 and FP32; sizes beyond the maximum are rejected."""
import numpy as np
import pytest

from paper_1912_04501_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _check(spm, wl, seed):
    s = spm.Solver("cuda:0")
    s.set_workload(wl)
    x, y, nx, ny, w = s.nodes()
    sigma = torch.as_tensor(W.random_density(s.N, seed=seed), device="cuda:0")
    for prec in (spm.SPM_FP64, spm.SPM_FP32):
        ref = s.near_traction(sigma, precision=prec).cpu().numpy()
        got = spm.near_traction_noalloc(x, y, nx, ny, w, sigma, wl["skew"], precision=prec).cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(f"[noalloc N={s.N} precision={prec}] max rel diff {err:.2e}", flush=True)
        # same pair arithmetic and tiles; only the FP64 grouping of the tile sums differs
        assert err <= 1e-12
    s.close()


def test_noalloc_near_sum_matches_handle_entry_point():
    from paper_1912_04501_amd import spm
    _check(spm, W.ellipses_200(), 7)     # N = 51,200
    _check(spm, W.ellipses_25(), 8)      # then a smaller cell: the shared array is reused


def test_noalloc_rejects_oversize():
    from paper_1912_04501_amd import spm
    n = spm.SPM_NOALLOC_MAX_N + 1
    z = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(spm.SpmError):
        spm.near_traction_noalloc(z, z, z, z, z, torch.zeros(2 * n, dtype=torch.float64, device="cuda:0"), 0.0)
