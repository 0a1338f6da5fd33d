"""The C ABI library loads and exports every function include/spm.h declares
(no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "spm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(spm_[a-z_0-9]+)\s*\(", src)))


# The calls of the method's boundary: create / destroy a handle, lattice and particles
# (Sec. 2, Sec. 6), the operator (Sec. 5) and its solve with the readouts (Sec. 3), time
# stepping (Sec. 7), ensembles in one call, and the network calls of the learned warm start.
BOUNDARY = ("spm_create", "spm_destroy", "spm_last_error", "spm_set_lattice", "spm_set_ellipses", "spm_num_nodes",
            "spm_get_nodes", "spm_apply", "spm_solve", "spm_effective_viscosity", "spm_step", "spm_solve_batch",
            "spm_features", "spm_mlp_set_weights", "spm_mlp_forward", "spm_mlp_backward", "spm_mlp_adam_step",
            "spm_autotune")


def test_header_declares_the_boundary():
    names = _declared()
    missing = [n for n in BOUNDARY if n not in names]
    assert not missing, missing


def test_boundary_signatures():
    """Argument lists of the boundary calls whose layout the callers depend on."""
    src = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "spm.h")).read(), flags=re.S)

    def args(name):
        m = re.search(name + r"\s*\(([^)]*)\)", src)
        return [a.strip() for a in m.group(1).split(",")]

    sb = args("spm_solve_batch")
    assert len(sb) == 14 and "int32_t n_cells" in sb[1] and "lattices" in sb[2] and "part_offsets" in sb[3]
    assert "n_nodes" in sb[8] and "cell_latency" in sb[13]
    assert "uint16_t" in args("spm_features")[1]
    sw = args("spm_mlp_set_weights")
    assert "uint16_t" in sw[1] and "float" in sw[2] and "int64_t" in sw[3]
    bw = args("spm_mlp_backward")
    assert "dy" in bw[2] and "grad" in bw[4]
    ad = args("spm_mlp_adam_step")
    assert [a.split()[-1] for a in ad[1:]] == ["grad", "lr", "beta1", "beta2", "eps", "step"]


def test_library_exports_every_declared_symbol():
    from paper_1912_04501_amd import spm
    lib = ctypes.CDLL(spm.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_default_config_without_device():
    from paper_1912_04501_amd import spm
    c = spm.default_config()
    assert c.M == 32 and c.m_wall == 24 and abs(c.R_proxy - 1.5) < 1e-15 and c.tol == 1e-10
    h = ctypes.c_void_p()
    bad = spm.default_config(M=2)
    assert spm.lib().spm_create(ctypes.byref(h), ctypes.byref(bad), None, spm.ALLOC_FN(0), spm.FREE_FN(0), None) \
        == spm.SPM_EINVAL
