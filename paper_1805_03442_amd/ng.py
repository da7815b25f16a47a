"""Python binding of the C ABI in ``include/ng.h`` (ctypes; argument
marshalling only).

Every step of the solver runs in the HIP library ``_lib/libng.so``; this module
never computes any part of the scheme.  PyTorch supplies device memory (a
``torch.uint8`` CUDA tensor) and the HIP stream.  Importing this module does not
load the library; the first call does, and raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libng.so")

NG_OK, NG_EINVAL, NG_ENOMEM, NG_EPHYS, NG_EDEVICE, NG_EFULL, NG_ESTALL = 0, -1, -2, -3, -4, -5, -6
NG_BC_PERIODIC, NG_BC_WALL, NG_BC_OUTFLOW, NG_BC_SOURCE = 0, 1, 2, 3
NG_HLLC, NG_HLL = 0, 1
NG_MINMOD = 0
NG_FP64, NG_FP32, NG_MIXED = 0, 1, 2
NG_MUSCL, NG_CSPH_TVD = 0, 1
NG_FLAG_NONFINITE, NG_FLAG_RHO, NG_FLAG_P, NG_FLAG_DONE = 1, 2, 4, 8

GAS_FIELDS = ("gamma", "R", "Cv", "rho0", "T0", "tau0", "tau_rho", "tau_T",
              "Q0", "Q_rho", "Q_T", "I0", "I_rho", "I_T", "fx", "fy")

EXPORTED = (
    "ng_strerror", "ng_state_bytes", "ng_init_state", "ng_init_conserved", "ng_step",
    "ng_run_to_time", "ng_diagnostics", "ng_get_state", "ng_get_conserved", "ng_set_launch",
    "ng_set_graph_steps", "ng_set_small_limit", "ng_set_coop", "ng_set_fused_accept", "ng_enable_timing", "ng_kernel_time", "ng_last_error", "ng_destroy",
    "ng_batch_create", "ng_batch_solve_bytes", "ng_batch_fits", "ng_batch_add", "ng_batch_run", "ng_batch_poll",
    "ng_batch_active", "ng_batch_diagnostics", "ng_batch_get_state", "ng_batch_get_conserved",
    "ng_batch_remove", "ng_batch_set_launch", "ng_batch_set_small_limit", "ng_batch_set_coop",
    "ng_batch_set_fused_accept", "ng_batch_last_error",
    "ng_batch_destroy", "ng_step_static", "ng_static_last_error",
)


class NgGas(C.Structure):
    _fields_ = [(f, C.c_double) for f in GAS_FIELDS]


class NgGrid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("reserved", C.c_int32), ("nx", C.c_int64),
                ("ny", C.c_int64), ("h", C.c_double), ("bc", C.c_int32 * 4),
                ("src_amp", C.c_double), ("src_lambda", C.c_double),
                ("src_yc", C.c_double), ("src_hw", C.c_double), ("wedge_x0", C.c_double),
                ("wedge_y0", C.c_double), ("wedge_tan", C.c_double)]


class NgNumerics(C.Structure):
    _fields_ = [("cfl", C.c_double), ("riemann", C.c_int32), ("limiter", C.c_int32),
                ("precision", C.c_int32), ("scheme", C.c_int32), ("stiff_z", C.c_double)]


class NgDiag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_last", C.c_double), ("dt_next", C.c_double),
                ("steps", C.c_int64), ("total", C.c_double * 5), ("src_budget", C.c_double * 2),
                ("rho_min", C.c_double), ("p_min", C.c_double), ("smax", C.c_double),
                ("flags", C.c_uint32), ("status", C.c_int32)]

    def as_dict(self):
        return dict(t=self.t, dt_last=self.dt_last, dt_next=self.dt_next, steps=self.steps,
                    total=list(self.total), src_budget=list(self.src_budget),
                    rho_min=self.rho_min, p_min=self.p_min, smax=self.smax,
                    flags=self.flags, status=self.status)


class NgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch's HIP runtime must be the one in the process before the library
        # is loaded, so that both resolve the same libamdhip64 (same SONAME)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, dp, i64, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.c_int32
        sig = {
            "ng_strerror": ([C.c_int], C.c_char_p),
            "ng_state_bytes": ([C.POINTER(NgGrid), C.POINTER(NgNumerics), C.POINTER(C.c_size_t)], C.c_int),
            "ng_init_state": ([C.POINTER(NgGas), C.POINTER(NgGrid), C.POINTER(NgNumerics), dp,
                               C.c_double, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
            "ng_init_conserved": ([C.POINTER(NgGas), C.POINTER(NgGrid), C.POINTER(NgNumerics), dp,
                                   C.c_double, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
            "ng_step": ([vp, i64], C.c_int),
            "ng_run_to_time": ([vp, C.c_double, i64, C.POINTER(i64)], C.c_int),
            "ng_diagnostics": ([vp, C.POINTER(NgDiag)], C.c_int),
            "ng_get_state": ([vp, dp], C.c_int),
            "ng_get_conserved": ([vp, dp], C.c_int),
            "ng_set_launch": ([vp, i32, i32], C.c_int),
            "ng_set_graph_steps": ([vp, i32], C.c_int),
            "ng_set_small_limit": ([vp, i64], C.c_int),
            "ng_set_coop": ([vp, i64, i32], C.c_int),
            "ng_set_fused_accept": ([vp, i32], C.c_int),
            "ng_enable_timing": ([vp, i32, i32], C.c_int),
            "ng_kernel_time": ([vp, dp, dp, C.POINTER(i64)], C.c_int),
            "ng_last_error": ([vp], C.c_char_p),
            "ng_destroy": ([vp], None),
            "ng_batch_create": ([i32, i32, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
            "ng_batch_solve_bytes": ([C.POINTER(NgGrid), i32, C.POINTER(C.c_size_t)], C.c_int),
            "ng_batch_fits": ([vp, C.POINTER(NgGrid), C.POINTER(i32)], C.c_int),
            "ng_batch_add": ([vp, C.POINTER(NgGas), C.POINTER(NgGrid), C.POINTER(NgNumerics), dp,
                              C.c_double, C.c_double, i64, C.POINTER(i32)], C.c_int),
            "ng_batch_run": ([vp, i64], C.c_int),
            "ng_batch_poll": ([vp, C.POINTER(i32), i32, C.POINTER(i32)], C.c_int),
            "ng_batch_active": ([vp, C.POINTER(i32)], C.c_int),
            "ng_batch_diagnostics": ([vp, i32, C.POINTER(NgDiag)], C.c_int),
            "ng_step_static": ([C.POINTER(NgGas), C.POINTER(NgGrid), C.POINTER(NgNumerics), vp,
                                vp, C.c_double, C.c_double, vp, C.POINTER(NgDiag)], C.c_int),
            "ng_static_last_error": ([], C.c_char_p),
            "ng_batch_get_state": ([vp, i32, dp], C.c_int),
            "ng_batch_get_conserved": ([vp, i32, dp], C.c_int),
            "ng_batch_remove": ([vp, i32], C.c_int),
            "ng_batch_set_launch": ([vp, i32, i32, i32], C.c_int),
            "ng_batch_set_small_limit": ([vp, i64], C.c_int),
            "ng_batch_set_coop": ([vp, i64, i32], C.c_int),
            "ng_batch_set_fused_accept": ([vp, i32], C.c_int),
            "ng_batch_last_error": ([vp], C.c_char_p),
            "ng_batch_destroy": ([vp], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def make_gas(g: dict) -> NgGas:
    return NgGas(*[float(g.get(f, 0.0)) for f in GAS_FIELDS])


def make_grid(nx: int, ny: int = 1, h: float | None = None, bc=(NG_BC_PERIODIC,) * 4,
              source=(0.0, 0.0), wedge=(0.0, 0.0, 0.0)) -> NgGrid:
    """bc = (x-low, x-high, y-low, y-high) boundary kinds; source = (amplitude,
    wavelength[, y_centre, half_width]) of the forced wave of an NG_BC_SOURCE
    x-low end; wedge = (x0, y0, tan) of an active wedge (tan <= 0: none)."""
    ndim = 1 if ny == 1 else 2
    h = float(h) if h is not None else 1.0 / nx
    src = tuple(float(v) for v in source) + (0.0, 0.0)[len(source) - 2:]
    return NgGrid(ndim, 0, int(nx), int(ny), h, (C.c_int32 * 4)(*[int(b) for b in bc]),
                  *src[:4], *[float(v) for v in wedge])


def make_numerics(cfl=0.4, riemann=NG_HLLC, precision=NG_FP64, stiff_z=0.5,
                  scheme=NG_MUSCL) -> NgNumerics:
    return NgNumerics(float(cfl), int(riemann), NG_MINMOD, int(precision), int(scheme),
                      float(stiff_z))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _planes(W: np.ndarray, ny: int) -> np.ndarray:
    """(5, ny, nx) primitive/conserved arrays -> the ABI's plane layout (4 planes
    in 1D: the v / rho v plane is dropped)."""
    W = np.asarray(W, dtype=np.float64)
    if ny == 1:
        W = W.reshape(W.shape[0], -1)
        if W.shape[0] == 5:
            W = W[[0, 1, 3, 4]]
    return np.ascontiguousarray(W)


def _unplanes(A: np.ndarray, nx: int, ny: int) -> np.ndarray:
    """ABI plane layout -> (5, ny, nx) with a zero v plane in 1D."""
    if ny == 1:
        out = np.zeros((5, 1, nx))
        out[[0, 1, 3, 4], 0] = A.reshape(4, nx)
        return out
    return A.reshape(5, ny, nx)


def stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def device_buffer(nbytes: int, device="cuda"):
    """Caller-owned device memory (256-byte aligned) as a torch tensor."""
    import torch
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t, t.data_ptr() + off


def check(code: int, what: str, err: str | None = None):
    if code != NG_OK:
        msg = lib().ng_strerror(code).decode()
        raise NgError(code, f"{what}: {msg}" + (f" [{err}]" if err else ""))


class Solver:
    """One solve: ``ng_init_state`` on a torch-owned device buffer."""

    def __init__(self, gas: dict, nx: int, ny: int = 1, W=None, U=None, h=None, cfl=0.4,
                 riemann=NG_HLLC, precision=NG_FP64, stiff_z=0.5, t0=0.0, stream=None,
                 bc=(NG_BC_PERIODIC,) * 4, source=(0.0, 0.0), wedge=(0.0, 0.0, 0.0),
                 scheme=NG_MUSCL):
        L = lib()
        self.nx, self.ny = int(nx), int(ny)
        self.gas = make_gas(gas)
        self.grid = make_grid(nx, ny, h, bc, source, wedge)
        self.num = make_numerics(cfl, riemann, precision, stiff_z, scheme)
        nbytes = C.c_size_t(0)
        check(L.ng_state_bytes(C.byref(self.grid), C.byref(self.num), C.byref(nbytes)),
              "ng_state_bytes")
        self.nbytes = nbytes.value
        self._buf, ptr = device_buffer(self.nbytes)
        self._stream = stream
        h_ = C.c_void_p(0)
        if U is not None:
            arr = _planes(U, self.ny)
            rc = L.ng_init_conserved(C.byref(self.gas), C.byref(self.grid), C.byref(self.num),
                                     _dp(arr), float(t0), C.c_void_p(ptr), self.nbytes,
                                     C.c_void_p(stream_handle(stream)), C.byref(h_))
        else:
            arr = _planes(W, self.ny)
            rc = L.ng_init_state(C.byref(self.gas), C.byref(self.grid), C.byref(self.num),
                                 _dp(arr), float(t0), C.c_void_p(ptr), self.nbytes,
                                 C.c_void_p(stream_handle(stream)), C.byref(h_))
        check(rc, "ng_init_state")
        self.h = h_

    def _err(self):
        return lib().ng_last_error(self.h).decode()

    def step(self, n: int):
        check(lib().ng_step(self.h, int(n)), "ng_step", self._err())

    def run_to_time(self, t_end: float, max_steps: int = 2**62) -> int:
        taken = C.c_int64(0)
        check(lib().ng_run_to_time(self.h, float(t_end), int(max_steps), C.byref(taken)),
              "ng_run_to_time", self._err())
        return taken.value

    def diagnostics(self) -> dict:
        d = NgDiag()
        check(lib().ng_diagnostics(self.h, C.byref(d)), "ng_diagnostics", self._err())
        return d.as_dict()

    def conserved(self) -> np.ndarray:
        nc = 4 if self.ny == 1 else 5
        out = np.empty(nc * self.nx * self.ny)
        check(lib().ng_get_conserved(self.h, _dp(out)), "ng_get_conserved", self._err())
        return _unplanes(out, self.nx, self.ny)

    def primitive(self) -> np.ndarray:
        nc = 4 if self.ny == 1 else 5
        out = np.empty(nc * self.nx * self.ny)
        check(lib().ng_get_state(self.h, _dp(out)), "ng_get_state", self._err())
        return _unplanes(out, self.nx, self.ny)

    def set_launch(self, rows: int = 0, waves: int = 0):
        check(lib().ng_set_launch(self.h, int(rows), int(waves)), "ng_set_launch", self._err())

    def set_small_limit(self, max_cells: int):
        check(lib().ng_set_small_limit(self.h, int(max_cells)), "ng_set_small_limit", self._err())

    def set_coop(self, max_cells: int = -1, spin_limit: int = -1):
        check(lib().ng_set_coop(self.h, int(max_cells), int(spin_limit)), "ng_set_coop",
              self._err())

    def set_fused_accept(self, on: bool):
        check(lib().ng_set_fused_accept(self.h, 1 if on else 0), "ng_set_fused_accept")

    def set_graph_steps(self, k: int):
        check(lib().ng_set_graph_steps(self.h, int(k)), "ng_set_graph_steps", self._err())

    def enable_timing(self, nsteps: int, every: int = 1):
        check(lib().ng_enable_timing(self.h, int(nsteps), int(every)), "ng_enable_timing")

    def kernel_time(self):
        a, b, n = C.c_double(0), C.c_double(0), C.c_int64(0)
        check(lib().ng_kernel_time(self.h, C.byref(a), C.byref(b), C.byref(n)), "ng_kernel_time")
        return a.value, b.value, n.value

    def close(self):
        if self.h:
            lib().ng_destroy(self.h)
            self.h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_static(gas: dict, nx: int, ny: int, U_in, U_out, t: float = 0.0, t_end: float = 0.0,
                h=None, cfl=0.4, riemann=NG_HLLC, stiff_z=0.5, bc=(NG_BC_PERIODIC,) * 4,
                source=(0.0, 0.0), wedge=(0.0, 0.0, 0.0), stream=None, diag: bool = True,
                scheme=NG_MUSCL):
    """One FP64 step (``ng_step_static``) from the device buffer U_in to U_out
    (torch CUDA tensors or device addresses: FP64 conserved planes in the ABI
    layout), with the library's static scratch; returns the diagnostics dict
    (diag=True, synchronising) or None (asynchronous)."""
    def addr(x):
        return int(x.data_ptr()) if hasattr(x, "data_ptr") else int(x)
    d = NgDiag()
    rc = lib().ng_step_static(C.byref(make_gas(gas)), C.byref(make_grid(nx, ny, h, bc, source, wedge)),
                              C.byref(make_numerics(cfl, riemann, NG_FP64, stiff_z, scheme)),
                              C.c_void_p(addr(U_in)), C.c_void_p(addr(U_out)), float(t),
                              float(t_end), C.c_void_p(stream_handle(stream)),
                              C.byref(d) if diag else None)
    check(rc, "ng_step_static", lib().ng_static_last_error().decode())
    return d.as_dict() if diag else None


class Batch:
    """Many solves of one precision advanced together (``ng_batch_*``)."""

    def __init__(self, capacity: int, arena_bytes: int, precision=NG_FP32, stream=None):
        L = lib()
        self._buf, ptr = device_buffer(arena_bytes)
        self.precision = precision
        h_ = C.c_void_p(0)
        check(L.ng_batch_create(int(capacity), int(precision), C.c_void_p(ptr), int(arena_bytes),
                                C.c_void_p(stream_handle(stream)), C.byref(h_)), "ng_batch_create")
        self.h = h_
        self.shapes = {}

    def _err(self):
        return lib().ng_batch_last_error(self.h).decode()

    @staticmethod
    def solve_bytes(nx, ny, precision=NG_FP32) -> int:
        g = make_grid(nx, ny)
        n = C.c_size_t(0)
        check(lib().ng_batch_solve_bytes(C.byref(g), int(precision), C.byref(n)),
              "ng_batch_solve_bytes")
        return n.value

    def fits(self, nx: int, ny: int) -> bool:
        """A solve of this grid would be admitted now (free slot and arena block)."""
        g = make_grid(nx, ny)
        f = C.c_int32(0)
        check(lib().ng_batch_fits(self.h, C.byref(g), C.byref(f)), "ng_batch_fits", self._err())
        return bool(f.value)

    def add(self, gas: dict, nx: int, ny: int, W, t_end: float, max_steps: int = 2**62,
            h=None, cfl=0.4, riemann=NG_HLLC, stiff_z=0.5, t0=0.0, bc=(NG_BC_PERIODIC,) * 4,
            source=(0.0, 0.0), wedge=(0.0, 0.0, 0.0), scheme=NG_MUSCL):
        """Returns the slot, or None when the batch is full (NG_EFULL)."""
        g, gr = make_gas(gas), make_grid(nx, ny, h, bc, source, wedge)
        nm = make_numerics(cfl, riemann, self.precision, stiff_z, scheme)
        arr = _planes(W, ny)
        slot = C.c_int32(-1)
        rc = lib().ng_batch_add(self.h, C.byref(g), C.byref(gr), C.byref(nm), _dp(arr),
                                float(t0), float(t_end), int(max_steps), C.byref(slot))
        if rc == NG_EFULL:
            return None
        check(rc, "ng_batch_add", self._err())
        self.shapes[slot.value] = (int(nx), int(ny))
        return slot.value

    def run(self, nsteps: int):
        check(lib().ng_batch_run(self.h, int(nsteps)), "ng_batch_run", self._err())

    def poll(self, cap: int = 4096):
        arr = (C.c_int32 * cap)()
        n = C.c_int32(0)
        check(lib().ng_batch_poll(self.h, arr, int(cap), C.byref(n)), "ng_batch_poll", self._err())
        return [arr[i] for i in range(n.value)]

    def active(self) -> int:
        n = C.c_int32(0)
        check(lib().ng_batch_active(self.h, C.byref(n)), "ng_batch_active", self._err())
        return n.value

    def diagnostics(self, slot: int) -> dict:
        d = NgDiag()
        check(lib().ng_batch_diagnostics(self.h, int(slot), C.byref(d)), "ng_batch_diagnostics",
              self._err())
        return d.as_dict()

    def conserved(self, slot: int) -> np.ndarray:
        nx, ny = self.shapes[slot]
        nc = 4 if ny == 1 else 5
        out = np.empty(nc * nx * ny)
        check(lib().ng_batch_get_conserved(self.h, int(slot), _dp(out)), "ng_batch_get_conserved",
              self._err())
        return _unplanes(out, nx, ny)

    def primitive(self, slot: int) -> np.ndarray:
        nx, ny = self.shapes[slot]
        nc = 4 if ny == 1 else 5
        out = np.empty(nc * nx * ny)
        check(lib().ng_batch_get_state(self.h, int(slot), _dp(out)), "ng_batch_get_state",
              self._err())
        return _unplanes(out, nx, ny)

    def remove(self, slot: int):
        check(lib().ng_batch_remove(self.h, int(slot)), "ng_batch_remove", self._err())
        self.shapes.pop(slot, None)

    def set_launch(self, dim: int, rows: int = 0, waves: int = 0):
        check(lib().ng_batch_set_launch(self.h, int(dim), int(rows), int(waves)),
              "ng_batch_set_launch", self._err())

    def set_small_limit(self, max_cells: int):
        check(lib().ng_batch_set_small_limit(self.h, int(max_cells)), "ng_batch_set_small_limit",
              self._err())

    def set_coop(self, max_cells: int = -1, spin_limit: int = -1):
        check(lib().ng_batch_set_coop(self.h, int(max_cells), int(spin_limit)), "ng_batch_set_coop",
              self._err())

    def set_fused_accept(self, on: bool):
        check(lib().ng_batch_set_fused_accept(self.h, 1 if on else 0), "ng_batch_set_fused_accept")

    def close(self):
        if self.h:
            lib().ng_batch_destroy(self.h)
            self.h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
