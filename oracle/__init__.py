"""Serial FP64 CPU oracle for the MUSCL step of Khrapov & Khoperskov (arXiv:1805.03442).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP library
shares no code with it, and the product path never calls it.

The arithmetic lives in ``muscl_oracle.c`` (the MUSCL step, eq. (15)) and
``csph_oracle.c`` (the CSPH-TVD step, eqs. (9)-(14), 1D), plain C in FP64
built with ``-ffp-contract=off`` into one library; this module only builds it
and marshals arrays through ctypes.  Each function cites the passage of the
paper it follows in the C files.

Arrays: a state is ``U[5, ny, nx]`` (rho, rho*u, rho*v, E, E_nu), FP64; a 1D
problem is ``ny == 1`` with ``rho*v == 0``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csph_oracle.c")      # includes muscl_oracle.c
_SRCS = [_SRC, os.path.join(_HERE, "muscl_oracle.c")]
_LIB = os.environ.get("NG_ORACLE_LIB") or os.path.join(_HERE, "_build", "liboracle.so")

BC_PERIODIC, BC_WALL, BC_OUTFLOW, BC_SOURCE = 0, 1, 2, 3
HLLC, HLL = 0, 1
OK, EINVAL, EPHYS = 0, -1, -3

GAS_FIELDS = ("gamma", "R", "Cv", "rho0", "T0", "tau0", "tau_rho", "tau_T",
              "Q0", "Q_rho", "Q_T", "I0", "I_rho", "I_T", "fx", "fy")


class OrGas(C.Structure):
    _fields_ = [(f, C.c_double) for f in GAS_FIELDS]


class OrGrid(C.Structure):
    _fields_ = [("nx", C.c_int64), ("ny", C.c_int64), ("h", C.c_double),
                ("bc", C.c_int32 * 4), ("src_amp", C.c_double), ("src_lambda", C.c_double),
                ("src_yc", C.c_double), ("src_hw", C.c_double), ("wedge_x0", C.c_double),
                ("wedge_y0", C.c_double), ("wedge_tan", C.c_double)]


class OrNum(C.Structure):
    _fields_ = [("cfl", C.c_double), ("riemann", C.c_int32), ("stiff_z", C.c_double)]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (serial, -O2, no FMA contraction)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if (force or not os.path.exists(_LIB)
            or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS)):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-I", _HERE, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.or_step.argtypes = [C.POINTER(OrGas), C.POINTER(OrGrid), C.POINTER(OrNum), dp, dp,
                              C.c_double, dp]
        L.or_step.restype = C.c_int
        L.or_step_at.argtypes = [C.POINTER(OrGas), C.POINTER(OrGrid), C.POINTER(OrNum), dp, dp,
                                 C.c_double, C.c_double, dp]
        L.or_step_at.restype = C.c_int
        L.or_run.argtypes = [C.POINTER(OrGas), C.POINTER(OrGrid), C.POINTER(OrNum), dp,
                             C.c_int64, C.c_double, dp, C.POINTER(C.c_int64), dp, dp]
        L.or_run.restype = C.c_int
        L.or_dt.argtypes = [C.POINTER(OrGas), C.POINTER(OrGrid), C.POINTER(OrNum), dp]
        L.or_dt.restype = C.c_double
        L.or_max_speed.argtypes = [C.POINTER(OrGas), C.POINTER(OrGrid), dp]
        L.or_max_speed.restype = C.c_double
        L.or_prim_to_cons.argtypes = [C.POINTER(OrGas), C.c_int64, dp, dp]
        L.or_cons_to_prim.argtypes = [C.POINTER(OrGas), C.c_int64, dp, dp]
        L.or_face_flux.argtypes = [C.POINTER(OrGas), C.c_int32, dp, dp, dp]
        L.or_source.argtypes = [C.POINTER(OrGas), dp, dp]
        # the CSPH-TVD entry points (absent from a build of the MUSCL file alone,
        # as the MUSCL mutation tests make)
        if hasattr(L, "cs_step"):
            L.cs_step.argtypes = [C.POINTER(OrGas), C.POINTER(OrGrid), C.POINTER(OrNum), dp,
                                  dp, C.c_double, C.c_double, dp, dp]
            L.cs_step.restype = C.c_int
            L.cs_run.argtypes = L.or_run.argtypes
            L.cs_run.restype = C.c_int
        _lib = L
    return _lib


def _gas(g: dict) -> OrGas:
    return OrGas(*[float(g.get(f, 0.0)) for f in GAS_FIELDS])


def _grid(nx: int, ny: int, h: float, bc=(0, 0, 0, 0), source=(0.0, 0.0),
          wedge=(0.0, 0.0, 0.0)) -> OrGrid:
    src = tuple(source) + (0.0, 0.0)[len(source) - 2:]
    return OrGrid(int(nx), int(ny), float(h), (C.c_int32 * 4)(*bc), *[float(v) for v in src[:4]],
                  *[float(v) for v in wedge])


def _num(cfl: float, riemann: int = HLLC, stiff_z: float = 0.5) -> OrNum:
    return OrNum(float(cfl), int(riemann), float(stiff_z))


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Problem:
    """Gas, grid and numerics of one solve (plain parameters, no state)."""

    def __init__(self, gas: dict, nx: int, ny: int = 1, h: float | None = None,
                 cfl: float = 0.4, riemann: int = HLLC, stiff_z: float = 0.5,
                 bc=(BC_PERIODIC,) * 4, source=(0.0, 0.0), wedge=(0.0, 0.0, 0.0)):
        """``source = (amplitude, wavelength[, y_centre, half_width])`` of the
        forced wave of a ``BC_SOURCE`` x-low end (half_width <= 0: the whole
        edge); ``wedge = (x0, y0, tan)``: pump and sink only inside the wedge
        x >= x0, |y - y0| <= (x - x0) tan (tan <= 0: everywhere)."""
        self.gas = dict(gas)
        self.nx, self.ny = int(nx), int(ny)
        self.h = float(h) if h is not None else 1.0 / self.nx
        self.cfl, self.riemann, self.stiff_z = float(cfl), int(riemann), float(stiff_z)
        self.bc = tuple(int(b) for b in bc)
        self.source = tuple(float(v) for v in source)
        self.wedge = tuple(float(v) for v in wedge)
        self._g = _gas(self.gas)
        self._gr = _grid(self.nx, self.ny, self.h, self.bc, self.source, self.wedge)
        self._nm = _num(self.cfl, self.riemann, self.stiff_z)

    @property
    def ncell(self) -> int:
        return self.nx * self.ny

    # --- conversions (eq. (5)) -------------------------------------------
    def prim_to_cons(self, W: np.ndarray) -> np.ndarray:
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(5, -1)
        U = np.empty_like(W)
        lib().or_prim_to_cons(C.byref(self._g), W.shape[1], _p(W), _p(U))
        return U.reshape(5, self.ny, self.nx)

    def cons_to_prim(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, -1)
        W = np.empty_like(U)
        lib().or_cons_to_prim(C.byref(self._g), U.shape[1], _p(U), _p(W))
        return W.reshape(5, self.ny, self.nx)

    # --- eq. (16) -----------------------------------------------------------
    def dt(self, U: np.ndarray) -> float:
        U = np.ascontiguousarray(U, dtype=np.float64)
        return lib().or_dt(C.byref(self._g), C.byref(self._gr), C.byref(self._nm), _p(U))

    def max_speed(self, U: np.ndarray) -> float:
        U = np.ascontiguousarray(U, dtype=np.float64)
        return lib().or_max_speed(C.byref(self._g), C.byref(self._gr), _p(U))

    # --- eq. (15) -----------------------------------------------------------
    def step(self, U: np.ndarray, dt: float, t: float = 0.0):
        """One step with a given dt from the state U at time t (t matters only
        to a source end).  Returns (status, U_new, src[2])."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, self.ny, self.nx)
        V = np.empty_like(U)
        src = np.zeros(2)
        st = lib().or_step_at(C.byref(self._g), C.byref(self._gr), C.byref(self._nm), _p(U),
                              _p(V), float(t), float(dt), _p(src))
        return st, V, src

    def run(self, U: np.ndarray, nsteps: int, t0: float = 0.0, t_end: float = 0.0):
        """Advance up to nsteps (dt from eq. (16) each step; stop at t_end if > 0).

        Returns dict(status, U, t, steps, budget[2], dt_last)."""
        U = np.array(U, dtype=np.float64, copy=True).reshape(5, self.ny, self.nx)
        t = C.c_double(t0)
        steps = C.c_int64(0)
        budget = np.zeros(2)
        dt_last = C.c_double(0.0)
        st = lib().or_run(C.byref(self._g), C.byref(self._gr), C.byref(self._nm), _p(U),
                          int(nsteps), float(t_end), C.byref(t), C.byref(steps), _p(budget),
                          C.byref(dt_last))
        return dict(status=st, U=U, t=t.value, steps=steps.value, budget=budget,
                    dt_last=dt_last.value)


class CsphProblem(Problem):
    """The CSPH-TVD scheme of section 2.3 (eqs. (9)-(14)) on a 1D grid with
    periodic, wall or outflow ends or a forced source at the x-low end: same
    gas, grid, time step (eq. (16)), source and state layout as ``Problem``;
    ``riemann`` and ``stiff_z`` are not used (HLL, explicit sources)."""

    def __init__(self, gas: dict, nx: int, h: float | None = None, cfl: float = 0.4,
                 bc=(BC_PERIODIC,) * 4, source=(0.0, 0.0)):
        super().__init__(gas, nx, 1, h=h, cfl=cfl, riemann=HLL, bc=bc, source=source)

    def step(self, U: np.ndarray, dt: float, t: float = 0.0, xi: bool = False):
        """One step with a given dt from the state U at time t.  Returns
        (status, U_new, src[2]), and with
        ``xi`` also the particles' displacements at the end of the Lagrangian
        stage (eq. (11)), one per cell."""
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(5, 1, self.nx)
        V = np.empty_like(U)
        src = np.zeros(2)
        X = np.zeros(self.nx)
        st = lib().cs_step(C.byref(self._g), C.byref(self._gr), C.byref(self._nm), _p(U),
                           _p(V), float(t), float(dt), _p(src), _p(X) if xi else None)
        return (st, V, src, X) if xi else (st, V, src)

    def run(self, U: np.ndarray, nsteps: int, t0: float = 0.0, t_end: float = 0.0):
        """As ``Problem.run`` with the CSPH-TVD step."""
        U = np.array(U, dtype=np.float64, copy=True).reshape(5, 1, self.nx)
        t = C.c_double(t0)
        steps = C.c_int64(0)
        budget = np.zeros(2)
        dt_last = C.c_double(0.0)
        st = lib().cs_run(C.byref(self._g), C.byref(self._gr), C.byref(self._nm), _p(U),
                          int(nsteps), float(t_end), C.byref(t), C.byref(steps), _p(budget),
                          C.byref(dt_last))
        return dict(status=st, U=U, t=t.value, steps=steps.value, budget=budget,
                    dt_last=dt_last.value)


def face_flux(gas: dict, WL, WR, riemann: int = HLLC) -> np.ndarray:
    """Interface flux for primitive states (rho, u_n, u_t, p, E_nu)."""
    g = _gas(gas)
    a = np.ascontiguousarray(WL, dtype=np.float64)
    b = np.ascontiguousarray(WR, dtype=np.float64)
    F = np.zeros(5)
    lib().or_face_flux(C.byref(g), int(riemann), _p(a), _p(b), _p(F))
    return F


def source(gas: dict, W) -> np.ndarray:
    """Source vector Y of eq. (15) at one primitive state."""
    g = _gas(gas)
    a = np.ascontiguousarray(W, dtype=np.float64)
    Y = np.zeros(5)
    lib().or_source(C.byref(g), _p(a), _p(Y))
    return Y
