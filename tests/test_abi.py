"""The C ABI library loads and exports every function include/mondpm.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mondpm.h")
LIB = os.path.join(ROOT, "paper_2312_02968_amd", "libmondpm.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\**([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_entry_points():
    names = declared_functions()
    for required in ("pm_deposit", "aqual_solve", "smooth_accel", "interp_push", "pm_step",
                     "pm_create", "pm_destroy", "pm_workspace_bytes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build the library first (python -m paper_2312_02968_amd.build)"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_side_argument_checks_without_gpu():
    from paper_2312_02968_amd import mondpm as M
    import workloads as W
    assert M.pm_spectrum_pitch(512) == 272 and M.pm_spectrum_pitch(16) == 16
    good = W.params(256)
    assert M.pm_workspace_bytes(good, 1 << 20) > 4 * 512 ** 3 * 4
    assert M.pm_workspace_bytes(dict(good, n_pad=500), 0) == 0     # not a power of two
    assert M.pm_workspace_bytes(dict(good, sigma=3.0), 0) == 0     # ball radius > 10 cells
    assert M.pm_workspace_bytes(dict(good, iters=0), 0) == 0


def test_net_parameter_layout_and_argument_checks_without_gpu():
    from paper_2312_02968_amd import mondpm as M
    from oracle import convnet as cn
    import ctypes as C
    assert M.pm_net_param_count() == sum(v.size for v in cn.init_params(0).values())
    h = C.c_void_p()
    L = M.lib()
    assert L.pm_net_create(12, 1, None, C.byref(h)) == M.PM_E_INVAL      # not a power of two
    assert L.pm_net_create(16, 0, None, C.byref(h)) == M.PM_E_INVAL      # no slots
    assert L.pm_net_create(4, 1, None, C.byref(h)) == M.PM_E_INVAL       # too small for 3 levels


def test_workspace_and_noalloc_argument_checks_without_gpu():
    import ctypes as C
    from paper_2312_02968_amd import mondpm as M
    import workloads as W
    L = M.lib()
    p = M.make_params(W.params(64))
    h = C.c_void_p()
    # a misaligned caller workspace is refused before any device call
    assert L.pm_create(C.byref(p), 0, C.c_void_p(0x1000 + 8), 1 << 30, None, C.byref(h)) == M.PM_E_INVAL
    assert L.pm_create(C.byref(p), -1, None, 0, None, C.byref(h)) == M.PM_E_INVAL
    assert M.pm_workspace_bytes(W.params(64), (1 << 30) + 1) == 0
    # the no-allocation deposit refuses inputs beyond its fixed scratch
    fake = C.c_void_p(0x1000)
    assert L.pm_deposit_noalloc(C.byref(p), fake, fake, (1 << 20) + 1, fake, None) == M.PM_E_INVAL
    big = M.make_params(W.params(512))                       # n_pad 1024
    assert L.pm_deposit_noalloc(C.byref(big), fake, fake, 10, fake, None) == M.PM_E_INVAL
    assert L.pm_deposit_noalloc(C.byref(p), None, None, 10, fake, None) == M.PM_E_INVAL
