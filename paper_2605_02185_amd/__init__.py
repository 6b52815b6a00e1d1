"""MI355X-native D2Q9 BGK lattice Boltzmann solver for unconfined flow past a
circular cylinder (arXiv 2605.02185), behind the C ABI of include/lbm.h.

``Lattice`` wraps one solver context.  PyTorch is used only to hand device
buffers and the current HIP stream to the library; all arithmetic runs in the
library's gfx950 kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (
    BOUNCE_HALFWAY,
    BOUNCE_INTERP,
    BOUNCE_FULLWAY,
    COLLISION_BGK,
    COLLISION_MRT,
    OUTLET_COPY_ALL,
    OUTLET_COPY_UNKNOWN,
    WALL_FREE_SLIP,
    WALL_MOVING_BB,
    WALL_NEBB,
    WALL_PERIODIC,
    DivergedError,
    LbmError,
    RangeError,
    check,
    make_params,
)

__all__ = [
    "Lattice", "Ensemble", "Mlp", "column_moments", "column_moments_noalloc", "make_params", "MLP_PARAMS", "validate", "tau_of", "geometry", "shedding_stats", "copy_probe",
    "num_variants", "variant_name", "LbmError", "DivergedError", "RangeError",
    "WALL_FREE_SLIP", "WALL_PERIODIC", "WALL_NEBB", "WALL_MOVING_BB",
    "OUTLET_COPY_ALL", "OUTLET_COPY_UNKNOWN", "COLLISION_BGK", "COLLISION_MRT", "BOUNCE_HALFWAY", "BOUNCE_INTERP", "BOUNCE_FULLWAY",
]


def validate(p: _lib.Params):
    check(_lib.lib.lbm_validate_params(ctypes.byref(p)))


def tau_of(p: _lib.Params) -> float:
    return _lib.lib.lbm_params_tau(ctypes.byref(p))


def geometry(p: _lib.Params):
    """(solid mask [ny][nx] uint8, n_solid, n_boundary_nodes, n_links); host only."""
    mask = np.zeros((p.ny, p.nx), dtype=np.uint8)
    ns, nb, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    check(_lib.lib.lbm_geometry(ctypes.byref(p), mask.ctypes.data, ctypes.byref(ns), ctypes.byref(nb),
                                ctypes.byref(nl)))
    return mask, ns.value, nb.value, nl.value


def shedding_stats(cd, cl, d, u, periods=5):
    cd = np.ascontiguousarray(cd, dtype=np.float64)
    cl = np.ascontiguousarray(cl, dtype=np.float64)
    out = _lib.Shedding()
    dp = ctypes.POINTER(ctypes.c_double)
    check(_lib.lib.lbm_shedding_stats(cd.ctypes.data_as(dp), cl.ctypes.data_as(dp), len(cd), d, u,
                                      periods, ctypes.byref(out)))
    return {"mean_cd": out.mean_cd, "cl_amp": out.cl_amp, "st": out.st, "period": out.period}


def copy_probe(dst, src, nbytes: int, stream=None):
    """Plain streaming copy of nbytes between two device tensors (bandwidth reference)."""
    for t, name in ((dst, "dst"), (src, "src")):
        if not getattr(t, "is_cuda", False) or not t.is_contiguous():
            raise LbmError(f"{name} must be a contiguous GPU tensor")
        if t.numel() * t.element_size() < nbytes:
            raise LbmError(f"{name} holds fewer than {nbytes} bytes")
    check(_lib.lib.lbm_copy_probe(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                  nbytes, _stream_handle(stream)))


def num_variants() -> int:
    return _lib.lib.lbm_num_variants()


def variant_name(v: int) -> str:
    return _lib.lib.lbm_variant_name(v).decode()


def _device_ptr(t, numel: int, dtypes=("torch.float32",), name: str = "tensor") -> ctypes.c_void_p:
    """The device address of a contiguous GPU tensor holding exactly `numel`
    elements of one of `dtypes`; raises instead of letting a kernel read or
    write past it."""
    if not getattr(t, "is_cuda", False):
        raise LbmError(f"{name} must be a GPU tensor")
    if str(t.dtype) not in dtypes:
        raise LbmError(f"{name} has dtype {t.dtype}; expected one of {', '.join(dtypes)}")
    if not t.is_contiguous():
        raise LbmError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise LbmError(f"{name} holds {t.numel()} elements; expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Lattice:
    """One solver context on the current device, ordered on `stream`
    (default: torch's current stream)."""

    def __init__(self, params: _lib.Params, stream=None):
        self.params = params
        self.nx, self.ny = params.nx, params.ny
        self._h = ctypes.c_void_p()
        check(_lib.lib.lbm_create(ctypes.byref(params), _stream_handle(stream), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _lib.lib.lbm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ steps
    def step(self, n: int = 1):
        check(_lib.lib.lbm_step(self._h, n))

    def sync(self):
        check(_lib.lib.lbm_sync(self._h))

    @property
    def t(self) -> int:
        s = ctypes.c_int64()
        check(_lib.lib.lbm_get_step(self._h, ctypes.byref(s)))
        return s.value

    def diverged_step(self) -> int:
        s = ctypes.c_int64()
        check(_lib.lib.lbm_diverged_step(self._h, ctypes.byref(s)))
        return s.value

    def set_variant(self, v: int):
        check(_lib.lib.lbm_set_variant(self._h, v))

    @property
    def variant(self) -> int:
        """Kernel variant in use (1-based, see variant_name)."""
        return _lib.lib.lbm_get_variant(self._h)

    def set_graphs(self, enable: bool):
        check(_lib.lib.lbm_set_graphs(self._h, 1 if enable else 0))

    # ------------------------------------------------------- learned closure
    def sample_boundary(self, ox, oy, wnx, wny, nodes, feat, target, bias=None):
        """Training samples of a wnx x wny window at (ox, oy); nodes (int32),
        feat [n][36], target [n][3] and the optional per-node bias [nb][3]
        subtracted from the targets are device tensors."""
        n = nodes.numel()
        pn = _device_ptr(nodes, n, ("torch.int32",), "nodes")
        pf = _device_ptr(feat, 36 * n, name="feat")
        pt = _device_ptr(target, 3 * n, name="target")
        pb = _device_ptr(bias, 3 * (2 * (wnx - 2) + (wny - 2)), name="bias") if bias is not None else None
        check(_lib.lib.lbm_sample_boundary(self._h, ox, oy, wnx, wny, pn, n, pb, pf, pt))

    def enable_closure(self, mlp: "Mlp", norm, boundaries: int = 7):
        """norm: 75 floats (feature mean[36], feature 1/std[36], output scale[3]);
        boundaries: bit mask 1 top, 2 bottom, 4 outlet."""
        a = np.ascontiguousarray(norm, dtype=np.float32)
        if a.size != 75:
            raise LbmError(f"norm needs 75 values; got {a.size}")
        self._mlp_ref = mlp
        check(_lib.lib.lbm_closure_enable(self._h, mlp._h, a.ctypes.data, boundaries))

    def set_closure_filter(self, beta: float = 1.0, taper: int = 0):
        check(_lib.lib.lbm_closure_set_filter(self._h, beta, taper))

    def set_closure_bias(self, bias):
        """Per-node fixed residual (host [nb][3]) added to the network's, or None."""
        if bias is None:
            check(_lib.lib.lbm_closure_set_bias(self._h, None))
            return
        nb = 2 * (self.nx - 2) + (self.ny - 2)
        a = np.ascontiguousarray(bias, dtype=np.float32)
        if a.size != 3 * nb:
            raise LbmError(f"bias needs {3 * nb} values; got {a.size}")
        check(_lib.lib.lbm_closure_set_bias(self._h, a.ctypes.data))

    def set_closure_guard(self, limit: float = 0.0, outlet_taper: int = 0, outlet_neutral: bool = False):
        """Clamp the network output to +-limit (units of the output scale; 0 =
        off), keep outlet nodes within outlet_taper of the rows plain and, with
        outlet_neutral, remove the mass the outlet residuals would add."""
        check(_lib.lib.lbm_closure_set_guard(self._h, limit, outlet_taper, 1 if outlet_neutral else 0))

    def set_closure_interval(self, interval: int = 1):
        """Evaluate the network every `interval` steps (a divisor of 96)."""
        check(_lib.lib.lbm_closure_set_interval(self._h, interval))

    def disable_closure(self):
        check(_lib.lib.lbm_closure_disable(self._h))
        self._mlp_ref = None

    def closure_residuals(self):
        nb = 2 * (self.nx - 2) + (self.ny - 2)
        out = np.empty((nb, 3), np.float32)
        check(_lib.lib.lbm_closure_residuals(self._h, out.ctypes.data))
        return out

    def autotune(self, steps: int = 20, cache: str | None = None) -> int:
        """Pick the fastest kernel variant (timed on a scratch copy); returns it."""
        best = ctypes.c_int32()
        check(_lib.lib.lbm_autotune(self._h, steps, cache.encode() if cache else None, ctypes.byref(best)))
        return best.value

    # ---------------------------------------------------------------- outputs
    def forces(self, first: int = 1, count: int | None = None):
        """(fx, fy, cd, cl) for steps [first, first+count); cd/cl None without a cylinder."""
        if count is None:
            count = self.t - first + 1
        fx, fy = np.zeros(count), np.zeros(count)
        coeff = self.params.diameter > 0 and self.params.u_in > 0
        cd = np.zeros(count) if coeff else None
        cl = np.zeros(count) if coeff else None
        check(_lib.lib.lbm_forces(self._h, first, count, fx.ctypes.data, fy.ctypes.data,
                                  cd.ctypes.data if coeff else None, cl.ctypes.data if coeff else None))
        return fx, fy, cd, cl

    def fields(self):
        """Host float32 arrays rho, ux, uy [ny][nx]."""
        shape = (self.ny, self.nx)
        rho, ux, uy = (np.empty(shape, np.float32) for _ in range(3))
        check(_lib.lib.lbm_fields(self._h, rho.ctypes.data, ux.ctypes.data, uy.ctypes.data, 0))
        return rho, ux, uy

    def fields_device(self, rho, ux, uy):
        """Fill caller-owned device tensors (float32, [ny][nx], contiguous)."""
        n = self.nx * self.ny
        ptr = [_device_ptr(t, n, name=nm) if t is not None else None
               for t, nm in ((rho, "rho"), (ux, "ux"), (uy, "uy"))]
        check(_lib.lib.lbm_fields(self._h, *ptr, 1))

    def get_populations(self, dtype=np.float32):
        dt = 0 if np.dtype(dtype) == np.float32 else 1
        out = np.empty((9, self.ny, self.nx), dtype=np.float32 if dt == 0 else np.float64)
        check(_lib.lib.lbm_get_populations(self._h, out.ctypes.data, dt, 0))
        return out

    def set_populations(self, f):
        f = np.asarray(f)
        dt = 0 if f.dtype == np.float32 else 1
        a = np.ascontiguousarray(f, dtype=np.float32 if dt == 0 else np.float64)
        if a.shape != (9, self.ny, self.nx):
            raise LbmError(f"populations must have shape (9, {self.ny}, {self.nx}); got {a.shape}")
        check(_lib.lib.lbm_set_populations(self._h, a.ctypes.data, dt, 0))

    def get_populations_device(self, t):
        """Copy the state into a device tensor [9][ny][nx] (float32 or float64)."""
        ptr = _device_ptr(t, 9 * self.nx * self.ny, ("torch.float32", "torch.float64"), "populations")
        dt = 0 if str(t.dtype) == "torch.float32" else 1
        check(_lib.lib.lbm_get_populations(self._h, ptr, dt, 1))

    def set_populations_device(self, t):
        """Load the state from a device tensor [9][ny][nx] (float32 or float64)."""
        ptr = _device_ptr(t, 9 * self.nx * self.ny, ("torch.float32", "torch.float64"), "populations")
        dt = 0 if str(t.dtype) == "torch.float32" else 1
        check(_lib.lib.lbm_set_populations(self._h, ptr, dt, 1))


class Ensemble:
    """Many independent lattices advanced together (one launch per step over
    the tiles of every active case).  `budgets[i]` (optional) stops case i
    after that many steps."""

    def __init__(self, params_list, budgets=None, stream=None, tune_cache: str | None = None):
        self.params = list(params_list)
        n = len(self.params)
        arr = (_lib.Params * n)(*self.params)
        bud = None
        if budgets is not None:
            bud = (ctypes.c_int64 * n)(*[int(b) for b in budgets])
        self._h = ctypes.c_void_p()
        check(_lib.lib.lbm_batch_create(arr, bud, n, _stream_handle(stream),
                                        tune_cache.encode() if tune_cache else None, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _lib.lib.lbm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def variant(self) -> int:
        return _lib.lib.lbm_batch_variant(self._h)

    def set_variant(self, v: int):
        check(_lib.lib.lbm_batch_set_variant(self._h, v))

    def step(self, n: int = 1):
        check(_lib.lib.lbm_batch_step(self._h, n))

    def sync(self):
        check(_lib.lib.lbm_batch_sync(self._h))

    def info(self, c: int):
        """(steps taken, first diverged step or 0) of case c."""
        s, d = ctypes.c_int64(), ctypes.c_int64()
        check(_lib.lib.lbm_batch_case_info(self._h, c, ctypes.byref(s), ctypes.byref(d)))
        return s.value, d.value

    def forces(self, c: int, first: int = 1, count: int | None = None):
        if count is None:
            count = self.info(c)[0] - first + 1
        p = self.params[c]
        fx, fy = np.zeros(count), np.zeros(count)
        coeff = p.diameter > 0 and p.u_in > 0
        cd = np.zeros(count) if coeff else None
        cl = np.zeros(count) if coeff else None
        check(_lib.lib.lbm_batch_forces(self._h, c, first, count, fx.ctypes.data, fy.ctypes.data,
                                        cd.ctypes.data if coeff else None, cl.ctypes.data if coeff else None))
        return fx, fy, cd, cl

    def fields(self, c: int):
        p = self.params[c]
        rho, ux, uy = (np.empty((p.ny, p.nx), np.float32) for _ in range(3))
        check(_lib.lib.lbm_batch_fields(self._h, c, rho.ctypes.data, ux.ctypes.data, uy.ctypes.data, 0))
        return rho, ux, uy

    def get_populations(self, c: int, dtype=np.float32):
        p = self.params[c]
        dt = 0 if np.dtype(dtype) == np.float32 else 1
        out = np.empty((9, p.ny, p.nx), dtype=np.float32 if dt == 0 else np.float64)
        check(_lib.lib.lbm_batch_get_populations(self._h, c, out.ctypes.data, dt, 0))
        return out

    def set_populations(self, c: int, f):
        """Load case c's state from a host array [9][ny][nx] (float32 or float64)."""
        p = self.params[c]
        f = np.asarray(f)
        dt = 0 if f.dtype == np.float32 else 1
        a = np.ascontiguousarray(f, dtype=np.float32 if dt == 0 else np.float64)
        if a.shape != (9, p.ny, p.nx):
            raise LbmError(f"populations of case {c} must have shape (9, {p.ny}, {p.nx}); got {a.shape}")
        check(_lib.lib.lbm_batch_set_populations(self._h, c, a.ctypes.data, dt, 0))


MLP_PARAMS = 6723


def column_moments(x, stream=None):
    """(mean, std) per column of a device tensor x [M][ncols] (FP64 sums)."""
    M, nc = x.shape
    mean, std = np.empty(nc), np.empty(nc)
    px = _device_ptr(x, M * nc, name="x")
    check(_lib.lib.lbm_column_moments(px, M, nc, mean.ctypes.data, std.ctypes.data, _stream_handle(stream)))
    return mean, std


def column_moments_noalloc(x, stream=None):
    """As column_moments, without a device allocation: the library's static
    device scratch holds the sums (ncols <= 4096; calls that overlap on one
    device race)."""
    M, nc = x.shape
    mean, std = np.empty(nc), np.empty(nc)
    px = _device_ptr(x, M * nc, name="x")
    check(_lib.lib.lbm_column_moments_noalloc(px, M, nc, mean.ctypes.data, std.ctypes.data, _stream_handle(stream)))
    return mean, std


class Mlp:
    """The closure network (36 -> 64 -> 64 -> 3) on the device.  Inputs and
    outputs are float32 device tensors (torch) of shape [M][36] / [M][3]."""

    def __init__(self, params=None, stream=None):
        self._h = ctypes.c_void_p()
        init = None
        if params is not None:
            self._init = np.ascontiguousarray(params, dtype=np.float32)
            if self._init.size != MLP_PARAMS:
                raise LbmError(f"the network has {MLP_PARAMS} parameters; got {self._init.size}")
            init = self._init.ctypes.data
        check(_lib.lib.lbm_mlp_create(init, _stream_handle(stream), ctypes.byref(self._h)))

    def close(self):
        if self._h:
            _lib.lib.lbm_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.empty(MLP_PARAMS, np.float32)
        check(_lib.lib.lbm_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, p):
        a = np.ascontiguousarray(p, dtype=np.float32)
        if a.size != MLP_PARAMS:
            raise LbmError(f"the network has {MLP_PARAMS} parameters; got {a.size}")
        check(_lib.lib.lbm_mlp_set_params(self._h, a.ctypes.data))

    def set_norm(self, norm):
        """z-score inside the kernels (75 floats) or None to switch it off."""
        if norm is None:
            check(_lib.lib.lbm_mlp_set_norm(self._h, None))
            return
        self._norm = np.ascontiguousarray(norm, dtype=np.float32)
        if self._norm.size != 75:
            raise LbmError(f"norm needs 75 values; got {self._norm.size}")
        check(_lib.lib.lbm_mlp_set_norm(self._h, self._norm.ctypes.data))

    def set_noise(self, amplitude: float, seed: int = 0):
        check(_lib.lib.lbm_mlp_set_noise(self._h, amplitude, seed))

    def forward(self, x, y):
        M = x.shape[0]
        px = _device_ptr(x, 36 * M, name="x")
        py = _device_ptr(y, 3 * M, name="y")
        check(_lib.lib.lbm_mlp_forward(self._h, px, M, py))

    def train_step(self, x, t, idx, batch: int, lr: float, want_loss=False):
        """One Adam step on rows idx[0..batch) of x / t (all rows 0..batch-1 if idx is None)."""
        M = x.shape[0]
        px = _device_ptr(x, 36 * M, name="x")
        pt = _device_ptr(t, 3 * M, name="t")
        if idx is not None:
            if idx.numel() < batch:
                raise LbmError(f"idx holds {idx.numel()} rows; batch is {batch}")
            ip = _device_ptr(idx, idx.numel(), ("torch.int32",), "idx")
        else:
            if batch > M:
                raise LbmError(f"batch {batch} exceeds the {M} rows of x")
            ip = None
        loss = ctypes.c_double()
        check(_lib.lib.lbm_mlp_train_step(self._h, px, pt, ip, batch, lr, ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def gradient(self, x, t):
        M = x.shape[0]
        px = _device_ptr(x, 36 * M, name="x")
        pt = _device_ptr(t, 3 * M, name="t")
        g = np.empty(MLP_PARAMS, np.float32)
        loss = ctypes.c_double()
        check(_lib.lib.lbm_mlp_gradient(self._h, px, pt, M, g.ctypes.data, ctypes.byref(loss)))
        return g, loss.value
