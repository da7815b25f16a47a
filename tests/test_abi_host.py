"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
function that include/ng.h declares, sizes device buffers and rejects invalid
arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ng.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ng_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def ng():
    from paper_1805_03442_amd import ng as _ng
    if not os.path.exists(_ng.LIB_PATH):
        from paper_1805_03442_amd import build
        build.build()
    _ng.lib()
    return _ng


def test_every_declared_symbol_is_exported(ng):
    names = declared_functions()
    assert len(names) >= 25
    L = ng.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(ng.EXPORTED)


def test_struct_sizes_match_header(ng):
    # the ctypes mirrors must have the C layout (checked through the sizes the
    # library itself reports for a known grid)
    assert C.sizeof(ng.NgGas) == 16 * 8
    assert C.sizeof(ng.NgGrid) == 4 + 4 + 8 + 8 + 8 + 16 + 16 + 16 + 24
    assert C.sizeof(ng.NgNumerics) == 8 + 4 * 4 + 8


def test_state_bytes(ng):
    L = ng.lib()
    out = C.c_size_t(0)
    for nx, ny, prec, nc, rs in ((1024, 1, ng.NG_FP64, 4, 8), (4096, 4096, ng.NG_FP32, 5, 4)):
        g = ng.make_grid(nx, ny)
        nm = ng.make_numerics(precision=prec)
        assert L.ng_state_bytes(C.byref(g), C.byref(nm), C.byref(out)) == 0
        state = 2 * nc * nx * ny * rs
        assert state <= out.value <= state * 1.02 + 65536
    bad = ng.make_grid(2, 1)
    assert L.ng_state_bytes(C.byref(bad), C.byref(ng.make_numerics()), C.byref(out)) == ng.NG_EINVAL


@pytest.mark.parametrize("field,value", [("gamma", 1.0), ("tau0", 0.0), ("R", -1.0),
                                         ("cfl", 1.5), ("nx", 3), ("riemann", 7),
                                         ("fy_1d", 0.1), ("precision", 5), ("bc", (4, 2)),
                                         ("bc", (0, 1)), ("bc", (2, 3)), ("bc", (3, 0)),
                                         ("source", (0.0, 0.1)), ("source", (0.6, 0.1)),
                                         ("segment_1d", 0.1), ("wedge_1d", 0.3),
                                         ("wedge_x0", -0.1), ("huge", 1 << 30),
                                         ("scheme", 2), ("scheme", -1),
                                         ("csph", "hllc"), ("csph", "fp32"), ("csph", "mixed"),
                                         ("csph", "2d"), ("csph", "segment")])
def test_invalid_arguments_rejected_before_device_use(ng, field, value):
    import numpy as np
    from paper_1805_03442_amd import workloads as wl
    L = ng.lib()
    gas = dict(wl.BASE_GAS)
    nx, ny = 64, 1
    cfl, riemann, prec = 0.4, ng.NG_HLLC, ng.NG_FP64
    scheme = ng.NG_MUSCL
    if field in ("gamma", "tau0", "R"):
        gas[field] = value
    elif field == "cfl":
        cfl = value
    elif field == "nx":
        nx = value
    elif field == "riemann":
        riemann = value
    elif field == "fy_1d":
        gas["fy"] = value
    elif field == "precision":
        prec = value
    elif field == "scheme":
        scheme = value
    elif field == "csph":
        # the CSPH-TVD step: 1D, FP64 and HLL only
        scheme, riemann = ng.NG_CSPH_TVD, ng.NG_HLL
        if value == "hllc":
            riemann = ng.NG_HLLC
        elif value == "fp32":
            prec = ng.NG_FP32
        elif value == "mixed":
            prec = ng.NG_MIXED
        elif value == "2d":
            ny = 64
    bc = (0, 0, 0, 0)
    source = (0.0, 0.0)
    if field == "bc":
        bc = tuple(value) + (0, 0)
    if field == "source":
        # a source end with a zero wavelength, or an amplitude of rho0 / 2 or more
        bc = (3, 2, 0, 0)
        source = (value[1], value[0]) if value[0] == 0.0 else value
    if field == "csph" and value == "segment":
        # a source segment needs a 2D grid, for either scheme
        bc, source = (3, 2, 0, 0), (1e-3, 0.1, 0.5, 0.1)
    wedge = (0.0, 0.0, 0.0)
    if field == "segment_1d":
        # a source segment needs a 2D grid
        bc, source = (3, 2, 0, 0), (1e-3, 0.1, 0.5, value)
    elif field == "wedge_1d":
        wedge = (0.0, 0.5, value)
    elif field == "wedge_x0":
        # the wedge's apex must not lie before x = 0
        ny = 64
        wedge = (value, 0.5, 0.3)
    grid = ng.make_grid(nx, ny, bc=bc, source=source, wedge=wedge)
    if field == "huge":
        # 2^30 cells of FP64: byte offsets beyond 32 bits (the state is never read)
        grid = ng.make_grid(value, 1)
        nx = 64
    W = wl.uniform_state(dict(wl.BASE_GAS), max(nx, 4), ny)[:, :, :nx]
    arr = np.ascontiguousarray(W[[0, 1, 3, 4]].reshape(4, -1) if ny == 1 else W.reshape(5, -1))
    h = C.c_void_p(0)
    rc = L.ng_init_state(C.byref(ng.make_gas(gas)), C.byref(grid),
                         C.byref(ng.make_numerics(cfl, riemann, prec, scheme=scheme)),
                         arr.ctypes.data_as(C.POINTER(C.c_double)), 0.0, C.c_void_p(256),
                         1 << 30, None, C.byref(h))
    assert rc == ng.NG_EINVAL
    assert not h.value


def test_too_small_buffer_is_enomem(ng):
    import numpy as np
    from paper_1805_03442_amd import workloads as wl
    L = ng.lib()
    W = wl.uniform_state(dict(wl.BASE_GAS), 64)
    arr = np.ascontiguousarray(W[[0, 1, 3, 4]].reshape(4, -1))
    h = C.c_void_p(0)
    rc = L.ng_init_state(C.byref(ng.make_gas(wl.BASE_GAS)), C.byref(ng.make_grid(64, 1)),
                         C.byref(ng.make_numerics()), arr.ctypes.data_as(C.POINTER(C.c_double)),
                         0.0, C.c_void_p(256), 1024, None, C.byref(h))
    assert rc == ng.NG_ENOMEM


def test_strerror(ng):
    L = ng.lib()
    for code in (0, -1, -2, -3, -4, -5):
        assert len(L.ng_strerror(code)) > 0


def test_autotune_uses_exact_buckets_only(tmp_path):
    """A tuned launch shape applies only to its own size bucket; other sizes
    keep the library's automatic shape (lookup gives None)."""
    import json
    from paper_1805_03442_amd import autotune
    from paper_1805_03442_amd import ng as _ng
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps({"2d_fp32_4096x4096": {"rows": 32, "waves": 4, "step_ms": 0.2}}))
    assert autotune.lookup(4096, 4096, _ng.NG_FP32, str(p)) == (32, 4)
    assert autotune.lookup(4000, 4200, _ng.NG_FP32, str(p)) == (32, 4)   # same bucket
    assert autotune.lookup(2048, 2048, _ng.NG_FP32, str(p)) is None
    assert autotune.lookup(4096, 4096, _ng.NG_FP64, str(p)) is None
    assert autotune.lookup(4096, 1, _ng.NG_FP32, str(p)) is None


def test_static_step_refuses_before_device_use(ng):
    """The entry point that allocates nothing refuses another precision, equal
    input and output buffers, and a grid beyond its static scratch, before any
    device call (the placeholder addresses are never touched)."""
    L = ng.lib()
    gas = ng.make_gas(dict(gamma=1.4, R=1.0, Cv=1.0, rho0=1.0, T0=1.0, tau0=0.05,
                           tau_rho=-1.0, tau_T=-1.0, Q0=0.1, Q_rho=0.5, Q_T=1.0,
                           I0=0.1, I_rho=1.0, I_T=2.0))
    a, b = C.c_void_p(0x1000), C.c_void_p(0x2000)
    cases = [
        (ng.make_grid(64, 64), ng.make_numerics(precision=ng.NG_FP32), a, b, ng.NG_EINVAL,
         b"FP64"),
        (ng.make_grid(64, 64), ng.make_numerics(precision=ng.NG_FP64), a, a, ng.NG_EINVAL,
         b"distinct"),
        (ng.make_grid(16384, 16384), ng.make_numerics(precision=ng.NG_FP64), a, b,
         ng.NG_ENOMEM, b"static scratch"),
        (ng.make_grid(2, 1), ng.make_numerics(precision=ng.NG_FP64), a, b, ng.NG_EINVAL, b""),
    ]
    for grid, num, u_in, u_out, code, text in cases:
        rc = L.ng_step_static(C.byref(gas), C.byref(grid), C.byref(num), u_in, u_out, 0.0, 0.0,
                              None, None)
        assert rc == code, (rc, code)
        assert text in L.ng_static_last_error()
