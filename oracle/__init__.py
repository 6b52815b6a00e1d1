"""FP64 CPU oracle for the D2Q9 BGK cylinder-flow method (arXiv 2605.02185).

TEST INFRASTRUCTURE ONLY.  The test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The GPU product package
never imports this module, and this module imports nothing from it.

``Oracle`` is a thin ctypes wrapper of ``lbm_oracle.c`` (the plain C solver);
``stats`` and ``mlp`` hold the oracle's own post-processing and its FP64 MLP.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")

WALL_FREE_SLIP, WALL_PERIODIC, WALL_NEBB, WALL_MOVING_BB = 0, 1, 2, 3
BGK, MRT = 0, 1
BB_HALFWAY, BB_INTERP, BB_FULLWAY = 0, 1, 2
# Relaxation rates of the paper's MRT (Sec. 2.1); the last two (shear) are 1/tau.
PAPER_S = (1.0, 1.1, 1.1, 1.0, 1.1, 1.0, 1.1, 0.0, 0.0)
OUTLET_COPY_ALL, OUTLET_COPY_UNKNOWN = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


NATIVE_FLAGS = ["-O3", "-march=native", "-fopenmp"]


def build_native(path: str) -> str:
    """A second build of the same source for timing on the machine it runs
    on (gcc -O3 -march=native, OpenMP), written to `path`.  The tests use
    the portable -O2 build; this one is compiled where it is timed, so that
    -march=native names that machine's CPU."""
    tmp = path + ".tmp"
    subprocess.check_call(["gcc", *NATIVE_FLAGS, "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, path)
    return path


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("diameter", ctypes.c_int),
        ("cx2", ctypes.c_int),
        ("cy2", ctypes.c_int),
        ("u_in", ctypes.c_double),
        ("re", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("wall", ctypes.c_int),
        ("u_wall_top", ctypes.c_double),
        ("u_wall_bottom", ctypes.c_double),
        ("outlet_mode", ctypes.c_int),
        ("x_periodic", ctypes.c_int),
        ("perturb_amp", ctypes.c_double),
        ("gx", ctypes.c_double),
        ("gy", ctypes.c_double),
        ("collision", ctypes.c_int),
        ("s_rates", ctypes.c_double * 9),
        ("bounce", ctypes.c_int),
        ("q_fixed", ctypes.c_double),
    ]


_libs = {}


def _load(path: str | None = None):
    path = path or _LIB_PATH
    if path in _libs:
        return _libs[path]
    if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER(_Params)
    dp = ctypes.POINTER(ctypes.c_double)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    lib.oracle_create.argtypes = [P, u8p]
    lib.oracle_create.restype = ctypes.c_void_p
    lib.oracle_destroy.argtypes = [ctypes.c_void_p]
    lib.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_long, dp, dp]
    lib.oracle_step.restype = ctypes.c_long
    lib.oracle_time.argtypes = [ctypes.c_void_p]
    lib.oracle_time.restype = ctypes.c_long
    lib.oracle_fields.argtypes = [ctypes.c_void_p, dp, dp, dp]
    for name in ("oracle_get_f", "oracle_set_f", "oracle_get_fstar", "oracle_set_fstar"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, dp]
    lib.oracle_digitise.argtypes = [P, u8p]
    lib.oracle_digitise.restype = ctypes.c_long
    lib.oracle_tau.argtypes = [P]
    lib.oracle_tau.restype = ctypes.c_double
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_mrt_matrix.argtypes = [dp]
    lib.oracle_links.restype = ctypes.c_long
    lib.oracle_links.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_mrt_meq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    _libs[path] = lib
    return lib


@dataclass
class OracleParams:
    """Problem statement in lattice units (Sec. 3.1; Eqs. 16-17 for tau)."""

    nx: int
    ny: int
    diameter: int = 0
    cx2: int | None = None  # doubled centre coordinates; default 21*D (10.5 D)
    cy2: int | None = None
    u_in: float = 0.1
    re: float = 100.0
    tau: float = 0.0
    wall: int = WALL_FREE_SLIP
    u_wall_top: float = math.nan
    u_wall_bottom: float = math.nan
    outlet_mode: int = OUTLET_COPY_ALL
    x_periodic: bool = False
    perturb_amp: float = 1e-3
    gx: float = 0.0
    gy: float = 0.0
    collision: int = BGK
    s_rates: tuple = PAPER_S
    bounce: int = BB_HALFWAY
    q_fixed: float = 0.0

    def _c(self) -> _Params:
        d = self.diameter
        return _Params(
            self.nx, self.ny, d,
            21 * d if self.cx2 is None else self.cx2,
            21 * d if self.cy2 is None else self.cy2,
            self.u_in, self.re, self.tau, self.wall,
            self.u_wall_top, self.u_wall_bottom, self.outlet_mode,
            1 if self.x_periodic else 0, self.perturb_amp, self.gx, self.gy,
            self.collision, (ctypes.c_double * 9)(*self.s_rates), self.bounce, self.q_fixed,
        )


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def digitise(p: OracleParams) -> np.ndarray:
    """Solid mask [ny][nx] (uint8) of the staircase disk."""
    lib = _load()
    out = np.zeros((p.ny, p.nx), dtype=np.uint8)
    cp = p._c()
    lib.oracle_digitise(ctypes.byref(cp), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    return out


def mrt_matrix() -> np.ndarray:
    out = np.empty((9, 9))
    _load().oracle_mrt_matrix(_dp(out))
    return out


def mrt_meq(rho, ux, uy) -> np.ndarray:
    out = np.empty(9)
    _load().oracle_mrt_meq(rho, ux, uy, _dp(out))
    return out


def threads(lib_path: str | None = None) -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return _load(lib_path).oracle_threads()


def set_threads(n: int, lib_path: str | None = None):
    """Threads of the oracle's parallel loops from now on (timing only)."""
    _load(lib_path).oracle_set_threads(n)


def tau_of(p: OracleParams) -> float:
    lib = _load()
    cp = p._c()
    return lib.oracle_tau(ctypes.byref(cp))


class Oracle:
    """Plain FP64 D2Q9 solver; state f[y][x][k] lives in C memory."""

    def __init__(self, p: OracleParams, solid: np.ndarray | None = None, lib_path: str | None = None):
        """`lib_path` selects another build of lbm_oracle.c (build_native)."""
        self.p = p
        self._lib = _load(lib_path)
        self._cp = p._c()
        sp = None
        if solid is not None:
            self._solid = np.ascontiguousarray(solid, dtype=np.uint8)
            assert self._solid.shape == (p.ny, p.nx)
            sp = self._solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self._h = self._lib.oracle_create(ctypes.byref(self._cp), sp)
        if not self._h:
            raise ValueError("oracle_create rejected the parameters")
        self.tau = tau_of(p)

    def links(self):
        """(node index y*nx + x, direction k, wall fraction q) of every
        fluid-to-solid link, in the oracle's order."""
        n = self._lib.oracle_links(self._h, None, None, None)
        node = np.empty(n, np.int64)
        k = np.empty(n, np.int32)
        q = np.empty(n, np.float64)
        self._lib.oracle_links(self._h, node.ctypes.data, k.ctypes.data, q.ctypes.data)
        return node, k, q

    def close(self):
        if self._h:
            self._lib.oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def t(self) -> int:
        return self._lib.oracle_time(self._h)

    def step(self, n: int):
        """Advance n steps; returns (fx, fy, diverged_at) with diverged_at 0 or the 1-based step."""
        fx = np.zeros(max(n, 1))
        fy = np.zeros(max(n, 1))
        bad = self._lib.oracle_step(self._h, n, _dp(fx), _dp(fy))
        return fx[:n], fy[:n], int(bad)

    def fields(self):
        shape = (self.p.ny, self.p.nx)
        rho, ux, uy = np.empty(shape), np.empty(shape), np.empty(shape)
        self._lib.oracle_fields(self._h, _dp(rho), _dp(ux), _dp(uy))
        return rho, ux, uy

    def _get(self, fn) -> np.ndarray:
        out = np.empty((9, self.p.ny, self.p.nx))
        fn(self._h, _dp(out))
        return out

    def get_f(self) -> np.ndarray:
        return self._get(self._lib.oracle_get_f)

    def get_fstar(self) -> np.ndarray:
        return self._get(self._lib.oracle_get_fstar)

    def set_f(self, f: np.ndarray):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.p.ny, self.p.nx)
        self._lib.oracle_set_f(self._h, _dp(a))

    def set_fstar(self, f: np.ndarray):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.p.ny, self.p.nx)
        self._lib.oracle_set_fstar(self._h, _dp(a))
