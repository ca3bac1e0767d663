"""The C-ABI library loads and exports every entry point include/sf.h
declares; host-side validation runs without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sf_create", "sf_solve", "sf_get_log", "sf_destroy",
              "sf_params_default", "sf_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1610_07159_amd import sf
    lib = ctypes.CDLL(sf.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n


def test_params_default_is_paper_column():
    from paper_1610_07159_amd import sf
    p = sf.sf_params_default().as_dict()
    expect = dict(w_reg=0.5, w_photo=0.5, w_grad=5.0, w_epi=0.5, w_s=0.75,
                  w_m=0.5, w_d=0.01, m_s=0.5, m_m=10.0, m_d=100.0,
                  w_smooth=1.0, w_mag=1.0, eps=0.001, eps_p=0.2)
    for k, v in expect.items():
        assert p[k] == pytest.approx(v, rel=1e-6), k


def test_host_validation_without_gpu():
    from paper_1610_07159_amd import sf
    lib = sf.lib
    p = sf.sf_params_default()
    h = ctypes.c_void_p()
    assert lib.sf_create(None, 64, 48, ctypes.byref(p), None) == -1
    assert lib.sf_create(ctypes.byref(h), 64, 48, None, None) == -1
    assert h.value is None
    for field, bad in (("levels", 0), ("levels", 99), ("pcg_iters", 65),
                       ("grid_stride", 0), ("m_m", 0.0), ("w_photo", -1.0),
                       ("max_backtracks", 9), ("exec_mode", 3), ("tile_mode", 5),
                       ("init_mode", 2), ("apply_mode", 4), ("apply_mode", -1), ("temporal", 2), ("illum", 2),
                       ("occlusion", 2), ("occlusion", -1),
                       ("eps", float("nan"))):
        q = sf.sf_params_default(**{field: bad})
        assert lib.sf_create(ctypes.byref(h), 64, 48, ctypes.byref(q), None) == -1, field
    # video mode needs the zero initialisation of the first frame
    q = sf.sf_params_default(levels=5, init_mode=1, temporal=1)
    assert lib.sf_create(ctypes.byref(h), 640, 480, ctypes.byref(q), None) == -1
    # levels that would shrink below 8 x 8 pixels
    q = sf.sf_params_default(levels=4)
    assert lib.sf_create(ctypes.byref(h), 60, 40, ctypes.byref(q), None) == -2
    assert lib.sf_create(ctypes.byref(h), 7, 40, ctypes.byref(p), None) == -2
    assert lib.sf_solve(None, None, None, None, None, None, None, None, None,
                        None) == -1
    n = ctypes.c_int()
    assert lib.sf_get_log(None, None, 0, ctypes.byref(n)) == -1
    assert lib.sf_debug_size(None, 0, 0) == 0
    lib.sf_destroy(None)
    assert sf.sf_status_string(-3) == "HIP runtime error"


def test_batch_levels_rule_and_validation_without_gpu():
    from paper_1610_07159_amd import sf
    lib = sf.lib
    # the batched workload's resolutions give 4 / 5 / 5 / 6 levels
    assert [sf.sf_batch_levels(w, h, 6) for w, h in
            ((320, 240), (640, 480), (960, 540), (1280, 720))] == [4, 5, 5, 6]
    assert sf.sf_batch_levels(64, 48, 3) == 1
    assert sf.sf_batch_levels(160, 120, 3) == 3
    assert sf.sf_batch_levels(159, 120, 3) == 2
    assert sf.sf_batch_levels(640, 20, 6) == 2  # coarsest level stays >= 8 px
    assert sf.sf_batch_levels(4, 48, 3) == 0
    fr = (sf.sf_frame * 1)()
    p = sf.sf_params_default()
    assert lib.sf_solve_batch(None, 1, fr, ctypes.byref(p)) == -1
    n = ctypes.c_int()
    assert lib.sf_get_batch_log(None, 0, None, 0, ctypes.byref(n)) == -1
    ms = ctypes.c_float()
    assert lib.sf_time_batch_kernel(None, 0, 0, 1, ctypes.byref(ms)) == -1
    v = ctypes.c_int(-1)
    assert lib.sf_tile_variant(None, 0, 0, ctypes.byref(v)) == -1
