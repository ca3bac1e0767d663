"""ctypes binding of the C ABI in include/sf.h (argument marshalling only).

Every function here has the name of the C entry point it wraps and passes
plain integers (device addresses, a hipStream_t) and ctypes structs; all
computation happens in libsf.so on the GPU.  Importing this module fails
loudly if the library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsf.so")

SF_OK = 0
STATUS = {0: "SF_OK", -1: "SF_ERR_INVALID_ARG", -2: "SF_ERR_SIZE",
          -3: "SF_ERR_HIP", -4: "SF_ERR_OOM", -5: "SF_ERR_NUMERIC",
          -6: "SF_ERR_STATE"}

# debug / stage enums (include/sf.h)
SF_DBG_TEX, SF_DBG_CMASK, SF_DBG_WNODE, SF_DBG_BASE, SF_DBG_DELTA = 0, 1, 2, 3, 4
SF_DBG_DX, SF_DBG_R, SF_DBG_Z, SF_DBG_Q, SF_DBG_DIAG = 5, 6, 7, 8, 9
SF_DBG_REC, SF_DBG_P, SF_DBG_ENERGY, SF_DBG_OCC = 10, 11, 12, 13
SF_STAGE_LEVEL_INIT, SF_STAGE_LINEARIZE, SF_STAGE_APPLY = 0, 1, 2
SF_STAGE_PCG, SF_STAGE_GN, SF_STAGE_FINISH, SF_STAGE_MASKS, SF_STAGE_STEP = 3, 4, 5, 6, 7
SF_STAGE_OCC, SF_STAGE_SPEC_STEP = 8, 9
SF_KERNEL_APPLY, SF_KERNEL_LINEARIZE, SF_KERNEL_UPDATE, SF_KERNEL_RHS, SF_KERNEL_BLOCKS = 0, 1, 2, 3, 4
SF_KERNEL_PCG_TILE = 5
SF_CNN_PARAMS = 39910
SF_TR_INPUT, SF_TR_ACT, SF_TR_OUT, SF_TR_DOUT, SF_TR_DPRE, SF_TR_GRAD = 0, 1, 2, 3, 4, 5


class SfError(RuntimeError):
    def __init__(self, code, where):
        msg = f"{where} failed: {STATUS.get(code, code)}"
        if code in (-3, -4):
            detail = lib.sf_last_error().decode()
            if detail:
                msg += f" [{detail}]"
        super().__init__(msg)
        self.code = code


class sf_calib(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("baseline", ctypes.c_float), ("F", ctypes.c_float * 9)]


_PARAM_INTS = ("levels", "grid_stride", "gn_iters", "pcg_iters",
               "max_backtracks", "init_mode", "exec_mode", "tile_mode",
               "apply_mode", "temporal", "illum", "occlusion", "gn_fine")
_PARAM_FLOATS = ("w_reg", "w_photo", "w_grad", "w_epi", "w_smooth", "w_mag",
                 "w_s", "w_m", "w_d", "m_s", "m_m", "m_d", "eps", "eps_p",
                 "st_gamma", "st_tau")


class sf_params(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_int) for n in _PARAM_INTS]
                + [(n, ctypes.c_float) for n in _PARAM_FLOATS])

    def as_dict(self):
        return {n: getattr(self, n) for n in _PARAM_INTS + _PARAM_FLOATS}


class sf_iter_log(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int), ("gn_iter", ctypes.c_int),
                ("energy", ctypes.c_double), ("e_photo", ctypes.c_double),
                ("e_grad", ctypes.c_double), ("e_smooth", ctypes.c_double),
                ("e_epi", ctypes.c_double), ("e_mag", ctypes.c_double),
                ("energy_after", ctypes.c_double), ("tau", ctypes.c_float),
                ("pcg_iters", ctypes.c_int), ("pcg_res", ctypes.c_float * 64),
                ("n_valid", ctypes.c_int)]


class sf_frame(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p * 4), ("width", ctypes.c_int),
                ("height", ctypes.c_int), ("calib", sf_calib),
                ("depth", ctypes.c_void_p), ("flow3d", ctypes.c_void_p),
                ("flows", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime; loading it first makes libsf.so bind
    # to that same runtime, so device pointers and streams from torch are
    # valid here (two runtimes in one process do not share devices)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    lib.sf_params_default.argtypes = [ctypes.POINTER(sf_params)]
    lib.sf_create.argtypes = [ctypes.POINTER(P), I, I,
                              ctypes.POINTER(sf_params), P]
    lib.sf_solve.argtypes = [P, P, P, P, P, ctypes.POINTER(sf_calib),
                             ctypes.POINTER(sf_params), P, P, P]
    lib.sf_get_log.argtypes = [P, ctypes.POINTER(sf_iter_log), I,
                               ctypes.POINTER(I)]
    lib.sf_status_string.argtypes = [I]
    lib.sf_status_string.restype = ctypes.c_char_p
    lib.sf_last_error.argtypes = []
    lib.sf_last_error.restype = ctypes.c_char_p
    lib.sf_destroy.argtypes = [P]
    lib.sf_destroy.restype = None
    lib.sf_reset_sequence.argtypes = [P]
    lib.sf_debug_size.argtypes = [P, I, I]
    lib.sf_debug_size.restype = ctypes.c_size_t
    lib.sf_debug_read.argtypes = [P, I, I, P, ctypes.c_size_t]
    lib.sf_debug_write.argtypes = [P, I, I, P, ctypes.c_size_t]
    lib.sf_debug_set_images.argtypes = [P, P, P, P, P,
                                        ctypes.POINTER(sf_calib)]
    lib.sf_debug_run.argtypes = [P, I, I]
    lib.sf_time_kernel.argtypes = [P, I, I, I, ctypes.POINTER(ctypes.c_float)]
    lib.sf_time_batch_kernel.argtypes = [P, I, I, I, ctypes.POINTER(ctypes.c_float)]
    lib.sf_tile_variant.argtypes = [P, I, I, ctypes.POINTER(I)]
    lib.sf_batch_levels.argtypes = [I, I, I]
    lib.sf_solve_batch.argtypes = [P, I, ctypes.POINTER(sf_frame),
                                   ctypes.POINTER(sf_params)]
    lib.sf_get_batch_log.argtypes = [P, I, ctypes.POINTER(sf_iter_log), I,
                                     ctypes.POINTER(I)]
    lib.sf_solve_noalloc.argtypes = [I, I, P, P, P, P, ctypes.POINTER(sf_calib),
                                     ctypes.POINTER(sf_params), P, P, P, P]
    lib.sf_solve_noalloc.restype = I
    F = ctypes.c_float
    D = ctypes.c_double
    S = ctypes.c_size_t
    lib.sf_set_initializer.argtypes = [P, P, S]
    lib.sf_get_init_result.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(D),
                                       ctypes.POINTER(D)]
    lib.sf_get_batch_init_result.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(D),
                                             ctypes.POINTER(D)]
    lib.sf_trainer_create.argtypes = [ctypes.POINTER(P), I, I, I, P]
    lib.sf_trainer_set_params.argtypes = [P, P, S]
    lib.sf_trainer_get_params.argtypes = [P, P, S]
    lib.sf_trainer_forward.argtypes = [P, P, I, P]
    lib.sf_trainer_step.argtypes = [P, P, P, I, F, ctypes.POINTER(F)]
    lib.sf_trainer_size.argtypes = [P, I, I]
    lib.sf_trainer_size.restype = S
    lib.sf_trainer_read.argtypes = [P, I, I, P, S]
    lib.sf_trainer_destroy.argtypes = [P]
    lib.sf_trainer_destroy.restype = None
    for f in ("sf_set_initializer", "sf_get_init_result", "sf_get_batch_init_result",
              "sf_trainer_create",
              "sf_trainer_set_params", "sf_trainer_get_params", "sf_trainer_forward",
              "sf_trainer_step", "sf_trainer_read"):
        getattr(lib, f).restype = I
    for f in ("sf_params_default", "sf_create", "sf_solve", "sf_get_log",
              "sf_debug_read", "sf_debug_write", "sf_debug_set_images",
              "sf_debug_run", "sf_time_kernel", "sf_time_batch_kernel", "sf_tile_variant",
              "sf_batch_levels", "sf_solve_batch", "sf_get_batch_log"):
        getattr(lib, f).restype = I
    return lib


lib = _load()


def _check(code, where):
    if code != SF_OK:
        raise SfError(code, where)


# ---- the C entry points ---------------------------------------------------

def sf_params_default(**overrides) -> sf_params:
    p = sf_params()
    _check(lib.sf_params_default(ctypes.byref(p)), "sf_params_default")
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def make_calib(fx, fy, cx, cy, baseline, F) -> sf_calib:
    c = sf_calib()
    c.fx, c.fy, c.cx, c.cy, c.baseline = fx, fy, cx, cy, baseline
    F = np.asarray(F, np.float64).reshape(9)
    for i in range(9):
        c.F[i] = float(F[i])
    return c


def sf_create(width: int, height: int, params: sf_params, stream: int = 0):
    h = ctypes.c_void_p()
    _check(lib.sf_create(ctypes.byref(h), int(width), int(height),
                         ctypes.byref(params), ctypes.c_void_p(stream)),
           "sf_create")
    return h


def sf_solve(ctx, I_left_t: int, I_right_t: int, I_left_t1: int,
             I_right_t1: int, calib: sf_calib, params: sf_params | None,
             depth: int, flow3d: int, flows: int = 0):
    _check(lib.sf_solve(ctx, I_left_t, I_right_t, I_left_t1, I_right_t1,
                        ctypes.byref(calib),
                        ctypes.byref(params) if params is not None else None,
                        depth, flow3d, flows or None), "sf_solve")


def _log_records(buf, n):
    out = []
    for i in range(n.value):
        r = buf[i]
        out.append(dict(level=r.level, gn_iter=r.gn_iter, energy=r.energy,
                        terms=dict(photo=r.e_photo, grad=r.e_grad,
                                   smooth=r.e_smooth, epi=r.e_epi,
                                   mag=r.e_mag),
                        energy_after=r.energy_after, tau=r.tau,
                        pcg_res=list(r.pcg_res[:r.pcg_iters]),
                        n_valid=r.n_valid))
    return out


def sf_get_log(ctx, cap: int = 4096):
    buf = (sf_iter_log * cap)()
    n = ctypes.c_int()
    code = lib.sf_get_log(ctx, buf, cap, ctypes.byref(n))
    if code not in (SF_OK, -5):
        _check(code, "sf_get_log")
    return _log_records(buf, n), code


def sf_solve_noalloc(width, height, imgs, calib: sf_calib, params: sf_params, depth, flow3d,
                     flows=0, stream=0):
    """imgs: four device addresses; depth, flow3d, flows: device addresses
    (flows may be 0); stream: a hipStream_t as an integer."""
    _check(lib.sf_solve_noalloc(int(width), int(height), *[int(a) for a in imgs],
                                ctypes.byref(calib), ctypes.byref(params), int(depth),
                                int(flow3d), int(flows) or None, int(stream) or None),
           "sf_solve_noalloc")


def sf_batch_levels(width: int, height: int, max_levels: int) -> int:
    return lib.sf_batch_levels(int(width), int(height), int(max_levels))


def make_frame(imgs, width, height, calib: sf_calib, depth, flow3d, flows=0):
    """imgs: four device addresses (left t, right t, left t+1, right t+1)."""
    f = sf_frame()
    for k in range(4):
        f.img[k] = int(imgs[k])
    f.width, f.height, f.calib = int(width), int(height), calib
    f.depth, f.flow3d, f.flows = int(depth), int(flow3d), (int(flows) or None)
    return f


def sf_solve_batch(ctx, frames, params: sf_params | None = None):
    arr = (sf_frame * len(frames))(*frames)
    _check(lib.sf_solve_batch(ctx, len(frames), arr,
                              ctypes.byref(params) if params is not None else None),
           "sf_solve_batch")


def sf_get_batch_log(ctx, frame: int, cap: int = 4096):
    buf = (sf_iter_log * cap)()
    n = ctypes.c_int()
    code = lib.sf_get_batch_log(ctx, int(frame), buf, cap, ctypes.byref(n))
    if code not in (SF_OK, -5):
        _check(code, "sf_get_batch_log")
    return _log_records(buf, n), code


def sf_status_string(code: int) -> str:
    return lib.sf_status_string(code).decode()


def sf_destroy(ctx):
    lib.sf_destroy(ctx)


def sf_reset_sequence(ctx):
    _check(lib.sf_reset_sequence(ctx), "sf_reset_sequence")


def sf_debug_size(ctx, what, level) -> int:
    return lib.sf_debug_size(ctx, what, level)


_DTYPE = {SF_DBG_TEX: np.float32, SF_DBG_CMASK: np.uint8,
          SF_DBG_ENERGY: np.float64, SF_DBG_OCC: np.uint8}


def sf_debug_read(ctx, what, level) -> np.ndarray:
    n = lib.sf_debug_size(ctx, what, level)
    if n == 0:
        raise SfError(-1, "sf_debug_size")
    dt = _DTYPE.get(what, np.float32)
    arr = np.empty(n // np.dtype(dt).itemsize, dt)
    _check(lib.sf_debug_read(ctx, what, level, arr.ctypes.data, n),
           "sf_debug_read")
    return arr


def sf_debug_write(ctx, what, level, arr):
    dt = _DTYPE.get(what, np.float32)
    a = np.ascontiguousarray(arr, dt)
    _check(lib.sf_debug_write(ctx, what, level, a.ctypes.data, a.nbytes),
           "sf_debug_write")


def sf_debug_set_images(ctx, I_left_t, I_right_t, I_left_t1, I_right_t1,
                        calib: sf_calib):
    _check(lib.sf_debug_set_images(ctx, I_left_t, I_right_t, I_left_t1,
                                   I_right_t1, ctypes.byref(calib)),
           "sf_debug_set_images")


def sf_debug_run(ctx, stage, level):
    _check(lib.sf_debug_run(ctx, stage, level), "sf_debug_run")


def sf_time_kernel(ctx, kernel, level, reps) -> float:
    """Average milliseconds per launch of one solver kernel (HIP events on
    the context's stream)."""
    ms = ctypes.c_float()
    _check(lib.sf_time_kernel(ctx, kernel, level, reps, ctypes.byref(ms)),
           "sf_time_kernel")
    return ms.value


def sf_tile_variant(ctx, batched, level) -> int:
    """The PCG iteration kernel's tile variant V at `level` of the last
    solve (batched False) or batch (True)."""
    v = ctypes.c_int(-1)
    _check(lib.sf_tile_variant(ctx, 1 if batched else 0, level, ctypes.byref(v)),
           "sf_tile_variant")
    return v.value


def sf_time_batch_kernel(ctx, kernel, level, reps) -> float:
    """The same over every frame of the last batch (one launch)."""
    ms = ctypes.c_float()
    _check(lib.sf_time_batch_kernel(ctx, kernel, level, reps, ctypes.byref(ms)),
           "sf_time_batch_kernel")
    return ms.value


# ---- learned initialiser --------------------------------------------------

def bf16_bits(values) -> np.ndarray:
    """float values -> bfloat16 bit patterns (uint16), round to nearest even."""
    f = np.ascontiguousarray(values, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def sf_set_initializer(ctx, weights):
    """weights: SF_CNN_PARAMS values (float, rounded to bfloat16 here) or
    uint16 bfloat16 bit patterns."""
    w = np.asarray(weights)
    bits = w if w.dtype == np.uint16 else bf16_bits(w)
    bits = np.ascontiguousarray(bits)
    _check(lib.sf_set_initializer(ctx, bits.ctypes.data, bits.nbytes), "sf_set_initializer")


def sf_get_init_result(ctx):
    used, ep, ez = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(lib.sf_get_init_result(ctx, ctypes.byref(used), ctypes.byref(ep), ctypes.byref(ez)),
           "sf_get_init_result")
    return bool(used.value), ep.value, ez.value


def sf_get_batch_init_result(ctx, frame):
    """(used, e_pred, e_zero) of batch frame `frame`; used = -1 for a frame
    with too few levels for the network (it started from zero)."""
    used, ep, ez = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    _check(lib.sf_get_batch_init_result(ctx, int(frame), ctypes.byref(used), ctypes.byref(ep),
                                        ctypes.byref(ez)), "sf_get_batch_init_result")
    return used.value, ep.value, ez.value


def sf_trainer_create(max_batch, height, width, stream=0):
    h = ctypes.c_void_p()
    _check(lib.sf_trainer_create(ctypes.byref(h), int(max_batch), int(height), int(width),
                                 ctypes.c_void_p(stream)), "sf_trainer_create")
    return h


def sf_trainer_set_params(t, flat):
    a = np.ascontiguousarray(flat, np.float32)
    _check(lib.sf_trainer_set_params(t, a.ctypes.data, a.size), "sf_trainer_set_params")


def sf_trainer_get_params(t):
    a = np.empty(SF_CNN_PARAMS, np.float32)
    _check(lib.sf_trainer_get_params(t, a.ctypes.data, a.size), "sf_trainer_get_params")
    return a


def sf_trainer_forward(t, x, batch, out):
    _check(lib.sf_trainer_forward(t, x, int(batch), out), "sf_trainer_forward")


def sf_trainer_step(t, x, target, batch, lr, want_loss=True):
    loss = ctypes.c_float()
    _check(lib.sf_trainer_step(t, x, target, int(batch), float(lr),
                               ctypes.byref(loss) if want_loss else None), "sf_trainer_step")
    return loss.value if want_loss else None


_TR_DTYPE = {SF_TR_INPUT: np.uint16, SF_TR_ACT: np.uint16, SF_TR_OUT: np.float32,
             SF_TR_DOUT: np.uint16, SF_TR_DPRE: np.uint16, SF_TR_GRAD: np.float32}


def sf_trainer_read(t, what, layer=0):
    n = lib.sf_trainer_size(t, what, layer)
    if n == 0:
        raise SfError(-1, "sf_trainer_size")
    dt = _TR_DTYPE[what]
    a = np.empty(n // np.dtype(dt).itemsize, dt)
    _check(lib.sf_trainer_read(t, what, layer, a.ctypes.data, n), "sf_trainer_read")
    return a


def bf16_to_float(bits) -> np.ndarray:
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32)


def sf_trainer_destroy(t):
    lib.sf_trainer_destroy(t)
