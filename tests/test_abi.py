"""The C-ABI library loads and exports every entry point include/disco.h declares;
host-side argument checks that run before any device call return the documented codes.
No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "disco.h")
LIB = os.path.join(ROOT, "paper_1807_00467_amd", "libdisco.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_path_entry_points():
    names = declared_functions()
    for n in ("ngf_eval", "ngf_grad", "ngf_hessvec", "curvature_apply", "volchange_eval", "keypoint_penalty",
              "gn_pcg_step", "gn_hessvec", "disco_create", "disco_destroy", "disco_set_images",
              "disco_set_keypoints", "disco_set_reference", "disco_copy_buffer", "disco_profile",
              "disco_profile_read", "disco_status_string", "lbfgs_step", "lbfgs_reset"):
        assert n in names, n


def test_library_exports_every_declared_symbol(lib):
    for n in declared_functions():
        assert hasattr(lib, n), f"missing export {n}"


def test_binding_covers_every_declared_symbol():
    from paper_1807_00467_amd import disco
    assert sorted(disco.EXPORTS) == declared_functions()


class Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3)]


def test_host_validation_codes_without_device(lib):
    lib.disco_create.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    lib.disco_status_string.restype = ctypes.c_char_p
    out = ctypes.c_void_p(123)
    # null geometry / null out
    assert lib.disco_create(None, 0, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.disco_create(None, 0, None) == -1
    # a size that is not a multiple of 4
    g = Geom((ctypes.c_int32 * 3)(30, 32, 32), (ctypes.c_double * 3)(1.0, 1.0, 1.0))
    assert lib.disco_create(ctypes.byref(g), 0, ctypes.byref(out)) == -2
    # non-positive spacing, bad storage enum
    g = Geom((ctypes.c_int32 * 3)(32, 32, 32), (ctypes.c_double * 3)(1.0, 0.0, 1.0))
    assert lib.disco_create(ctypes.byref(g), 0, ctypes.byref(out)) == -4
    g = Geom((ctypes.c_int32 * 3)(32, 32, 32), (ctypes.c_double * 3)(1.0, 1.0, float("nan")))
    assert lib.disco_create(ctypes.byref(g), 0, ctypes.byref(out)) == -4
    g = Geom((ctypes.c_int32 * 3)(32, 32, 32), (ctypes.c_double * 3)(1.0, 1.0, 1.0))
    assert lib.disco_create(ctypes.byref(g), 7, ctypes.byref(out)) == -1
    # null context on every entry point
    V = ctypes.c_void_p
    lib.ngf_eval.argtypes = [V, ctypes.c_double, V, V, V]
    assert lib.ngf_eval(None, 10.0, None, None, None) == -1
    lib.ngf_hessvec.argtypes = [V, V, V, V]
    assert lib.ngf_hessvec(None, None, None, None) == -1
    lib.gn_pcg_step.argtypes = [V, V, V, V, V, V]
    assert lib.gn_pcg_step(None, None, None, None, None, None) == -1
    lib.lbfgs_step.argtypes = [V, V, V, V, V, V, V]
    assert lib.lbfgs_step(None, None, None, None, None, None, None) == -1
    lib.lbfgs_reset.argtypes = [V]
    assert lib.lbfgs_reset(None) == -1
    lib.objective_linearise.argtypes = [V, V, V, V, V, V, V]
    assert lib.objective_linearise(None, None, None, None, None, None, None) == -1
    lib.disco_set_masks.argtypes = [V, V, V, V]
    assert lib.disco_set_masks(None, None, None, None) == -1
    lib.multilevel_register.argtypes = [V] * 12
    assert lib.multilevel_register(*([None] * 12)) == -1
    lib.pyramid_downsample.argtypes = [V] * 6
    assert lib.pyramid_downsample(*([None] * 6)) == -1
    lib.pyramid_prolong.argtypes = [V] * 5
    assert lib.pyramid_prolong(*([None] * 5)) == -1
    # keypoint stage: argument checks before any device call
    lib.disco_kp_create.argtypes = [V, V, V]
    kp = ctypes.c_void_p(7)
    n3 = (ctypes.c_int32 * 3)(32, 32, 0)
    h3 = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert lib.disco_kp_create(n3, h3, ctypes.byref(kp)) == -2 and kp.value is None
    n3 = (ctypes.c_int32 * 3)(32, 32, 32)
    h3 = (ctypes.c_double * 3)(1.0, float("inf"), 1.0)
    assert lib.disco_kp_create(n3, h3, ctypes.byref(kp)) == -4
    assert lib.disco_kp_create(None, h3, ctypes.byref(kp)) == -1
    lib.disco_kp_cost.argtypes = [V, ctypes.c_int32, V, ctypes.c_int32, V, V]
    assert lib.disco_kp_cost(None, 1, None, 16, None, None) == -1
    lib.disco_kp_regularise.argtypes = [V, ctypes.c_int32, V, V, ctypes.c_int32, V, ctypes.c_double,
                                        ctypes.c_double, V, V, V, V]
    assert lib.disco_kp_regularise(None, 1, None, None, 16, None, 0.1, 150.0, None, None, None, None) == -1
    lib.disco_kp_destroy.argtypes = [V]
    lib.disco_kp_destroy(None)
    lib.disco_destroy.argtypes = [V]
    lib.disco_destroy(None)
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.disco_status_string(code)


def test_oracle_and_library_share_no_code():
    """The oracle never includes, links or imports the GPU library, and vice versa."""
    import glob
    for f in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if f.endswith((".c", ".py")):
            txt = open(f).read()
            assert "paper_1807_00467_amd" not in txt and "disco.h" not in txt and "kernels.hpp" not in txt, f
    for f in glob.glob(os.path.join(ROOT, "paper_1807_00467_amd", "**", "*"), recursive=True):
        if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            txt = open(f).read()
            assert "import oracle" not in txt and "disco_oracle" not in txt and "from oracle" not in txt, f
