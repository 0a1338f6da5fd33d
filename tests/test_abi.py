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


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("spm_create", "spm_set_lattice", "spm_set_ellipses", "spm_apply", "spm_solve", "spm_step",
                 "spm_effective_viscosity", "spm_autotune"):
        assert must in names


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
