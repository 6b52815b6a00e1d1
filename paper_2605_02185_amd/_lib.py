"""ctypes binding of liblbm.so (include/lbm.h).  Argument marshalling only.

Every step of the solver runs in the HIP kernels of liblbm.so; this module
converts Python arguments to the C ABI and C status codes to exceptions.  It
loads nothing else: if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

OK, ERR_INVALID_ARG, ERR_HIP, ERR_OOM, ERR_DIVERGED, ERR_RANGE, ERR_STATE = 0, -1, -2, -3, -4, -5, -6
WALL_FREE_SLIP, WALL_PERIODIC, WALL_NEBB, WALL_MOVING_BB = 0, 1, 2, 3
OUTLET_COPY_ALL, OUTLET_COPY_UNKNOWN = 0, 1
COLLISION_BGK, COLLISION_MRT = 0, 1
BOUNCE_HALFWAY, BOUNCE_INTERP, BOUNCE_FULLWAY = 0, 1, 2


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class DivergedError(LbmError):
    pass


class RangeError(LbmError):
    pass


class Params(ctypes.Structure):
    """Mirror of lbm_params."""

    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("diameter", ctypes.c_int32),
        ("cx2", ctypes.c_int32),
        ("cy2", ctypes.c_int32),
        ("u_in", ctypes.c_double),
        ("re", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("wall", ctypes.c_int32),
        ("outlet_mode", ctypes.c_int32),
        ("u_wall_top", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double),
        ("x_periodic", ctypes.c_int32),
        ("collision", ctypes.c_int32),
        ("perturb_amp", ctypes.c_double),
        ("hist_capacity", ctypes.c_int64),
        ("s_rates", ctypes.c_double * 9),
        ("bounce", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
    ]


class Shedding(ctypes.Structure):
    _fields_ = [("mean_cd", ctypes.c_double), ("cl_amp", ctypes.c_double),
                ("st", ctypes.c_double), ("period", ctypes.c_double)]


def _load():
    # torch links its own HIP runtime by the unversioned name libamdhip64.so;
    # loading it first makes liblbm.so's libamdhip64.so.7 resolve to that same
    # runtime (matching SONAME), so the process holds one HIP runtime and
    # torch's streams and device pointers are valid in the library.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')"
        )
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp, fp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    P = ctypes.POINTER(Params)
    sigs = {
        "lbm_params_init": (None, [P]),
        "lbm_validate_params": (i32, [P]),
        "lbm_params_tau": (ctypes.c_double, [P]),
        "lbm_geometry": (i32, [P, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "lbm_create": (i32, [P, vp, ctypes.POINTER(vp)]),
        "lbm_destroy": (None, [vp]),
        "lbm_step": (i32, [vp, i64]),
        "lbm_sync": (i32, [vp]),
        "lbm_get_step": (i32, [vp, ctypes.POINTER(i64)]),
        "lbm_diverged_step": (i32, [vp, ctypes.POINTER(i64)]),
        "lbm_forces": (i32, [vp, i64, i64, vp, vp, vp, vp]),
        "lbm_fields": (i32, [vp, vp, vp, vp, ctypes.c_int]),
        "lbm_get_populations": (i32, [vp, vp, ctypes.c_int, ctypes.c_int]),
        "lbm_set_populations": (i32, [vp, vp, ctypes.c_int, ctypes.c_int]),
        "lbm_shedding_stats": (i32, [dp, dp, i64, ctypes.c_double, ctypes.c_double, i32, ctypes.POINTER(Shedding)]),
        "lbm_num_variants": (i32, []),
        "lbm_set_variant": (i32, [vp, i32]),
        "lbm_get_variant": (i32, [vp]),
        "lbm_variant_name": (ctypes.c_char_p, [i32]),
        "lbm_set_graphs": (i32, [vp, ctypes.c_int]),
        "lbm_copy_probe": (i32, [vp, vp, i64, vp]),
        "lbm_autotune": (i32, [vp, i32, ctypes.c_char_p, ctypes.POINTER(i32)]),
        "lbm_batch_create": (i32, [P, ctypes.POINTER(i64), i32, vp, ctypes.c_char_p, ctypes.POINTER(vp)]),
        "lbm_batch_destroy": (None, [vp]),
        "lbm_batch_step": (i32, [vp, i64]),
        "lbm_batch_sync": (i32, [vp]),
        "lbm_batch_case_info": (i32, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "lbm_batch_forces": (i32, [vp, i32, i64, i64, vp, vp, vp, vp]),
        "lbm_batch_fields": (i32, [vp, i32, vp, vp, vp, ctypes.c_int]),
        "lbm_batch_get_populations": (i32, [vp, i32, vp, ctypes.c_int, ctypes.c_int]),
        "lbm_batch_set_populations": (i32, [vp, i32, vp, ctypes.c_int, ctypes.c_int]),
        "lbm_batch_variant": (i32, [vp]),
        "lbm_batch_set_variant": (i32, [vp, i32]),
        "lbm_mlp_create": (i32, [vp, vp, ctypes.POINTER(vp)]),
        "lbm_mlp_destroy": (None, [vp]),
        "lbm_mlp_get_params": (i32, [vp, vp]),
        "lbm_mlp_set_params": (i32, [vp, vp]),
        "lbm_mlp_forward": (i32, [vp, vp, i64, vp]),
        "lbm_mlp_set_norm": (i32, [vp, vp]),
        "lbm_mlp_set_noise": (i32, [vp, ctypes.c_float, ctypes.c_uint64]),
        "lbm_mlp_train_step": (i32, [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
        "lbm_mlp_gradient": (i32, [vp, vp, vp, i64, vp, ctypes.POINTER(ctypes.c_double)]),
        "lbm_column_moments": (i32, [vp, i64, i32, vp, vp, vp]),
        "lbm_column_moments_noalloc": (i32, [vp, i64, i32, vp, vp, vp]),
        "lbm_sample_boundary": (i32, [vp, i32, i32, i32, i32, vp, i64, vp, vp, vp]),
        "lbm_closure_set_bias": (i32, [vp, vp]),
        "lbm_closure_enable": (i32, [vp, vp, vp, i32]),
        "lbm_closure_set_interval": (i32, [vp, i32]),
        "lbm_closure_disable": (i32, [vp]),
        "lbm_closure_set_filter": (i32, [vp, ctypes.c_float, i32]),
        "lbm_closure_set_guard": (i32, [vp, ctypes.c_float, i32, i32]),
        "lbm_closure_residuals": (i32, [vp, vp]),
        "lbm_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int):
    if status == OK:
        return
    msg = lib.lbm_last_error().decode(errors="replace")
    if status == ERR_DIVERGED:
        raise DivergedError(status, msg)
    if status == ERR_RANGE:
        raise RangeError(status, msg)
    raise LbmError(status, msg)


def make_params(nx, ny, diameter=0, cx2=None, cy2=None, u_in=0.1, re=100.0, tau=0.0,
                wall=WALL_FREE_SLIP, outlet_mode=OUTLET_COPY_ALL, u_wall_top=math.nan,
                u_wall_bottom=math.nan, x_periodic=False, perturb_amp=1e-3,
                hist_capacity=1 << 20, collision=COLLISION_BGK, s_rates=None,
                bounce=BOUNCE_HALFWAY) -> Params:
    """lbm_params from keywords; s_rates (9 values, MRT) defaults to the
    rates of Sec. 2.1, with 0 for the shear rates meaning 1/tau."""
    p = Params()
    lib.lbm_params_init(ctypes.byref(p))
    p.nx, p.ny, p.diameter = nx, ny, diameter
    p.cx2 = 21 * diameter if cx2 is None else cx2
    p.cy2 = 21 * diameter if cy2 is None else cy2
    p.u_in, p.re, p.tau = u_in, re, tau
    p.wall, p.outlet_mode = wall, outlet_mode
    p.u_wall_top, p.u_wall_bottom = u_wall_top, u_wall_bottom
    p.x_periodic = 1 if x_periodic else 0
    p.perturb_amp = perturb_amp
    p.hist_capacity = hist_capacity
    p.collision = collision
    p.bounce = bounce
    if s_rates is not None:
        if len(s_rates) != 9:
            raise ValueError("s_rates needs 9 values")
        p.s_rates[:] = [float(v) for v in s_rates]
    return p
