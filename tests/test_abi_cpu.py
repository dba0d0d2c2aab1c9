"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes as C
import math
import re

import numpy as np
import pytest

from paper_2104_06784_amd import _abi as A
from paper_2104_06784_amd import inputs as I
from paper_2104_06784_amd.sim import make_params


def _declared_symbols():
    text = open(A.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(m2p_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    syms = _declared_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L, s), s
        assert s in A.SIGNATURES, f"binding lacks {s}"


def test_version_and_strerror():
    L = A.lib()
    assert b"gfx950" in L.m2p_version()
    for code in range(0, -10, -1):
        assert L.m2p_strerror(code)
    assert L.m2p_strerror(-99) == b"unknown status"


def test_buffer_bytes():
    L = A.lib()
    n = C.c_size_t()
    A.check(L.m2p_buffer_bytes(C.byref(A.Grid(100, 30, 5.0, 5.0)), A.M2P_FP32, C.byref(n)))
    assert n.value == 6 * 30 * 128 * 4
    A.check(L.m2p_buffer_bytes(C.byref(A.Grid(128, 30, 5.0, 5.0)), A.M2P_FP64, C.byref(n)))
    assert n.value == 6 * 30 * 128 * 8
    assert L.m2p_buffer_bytes(C.byref(A.Grid(3, 30, 5.0, 5.0)), A.M2P_FP32, C.byref(n)) == A.M2P_EINVAL
    assert L.m2p_buffer_bytes(C.byref(A.Grid(8, 8, 5.0, 5.0)), 7, C.byref(n)) == A.M2P_EINVAL


def _create(grid, params, prec=A.M2P_FP64, dem=None):
    L = A.lib()
    dem = np.zeros((grid.ny, grid.nx)) if dem is None else dem
    h = C.c_void_p()
    rc = L.m2p_create(C.byref(h), C.byref(grid), C.byref(params), prec, A.dptr(np.ascontiguousarray(dem)),
                      None, None)
    return rc, h


@pytest.mark.parametrize("field,value", [
    ("delta_b_deg", 90.0), ("delta_b_deg", -1.0), ("cfl", 0.0), ("cfl", 1.5), ("rho_f", 3000.0),
    ("H", 0.0), ("m_dry", 0.0), ("a_min", -1.0), ("c_d", -2.0), ("chi", math.inf)])
def test_create_rejects_bad_parameters(field, value):
    p = I.Params()
    setattr(p, field, value)
    rc, h = _create(A.Grid(8, 8, 10.0, 10.0), make_params(p))
    assert rc == A.M2P_EINVAL and not h.value
    assert A.lib().m2p_last_error()


def test_create_rejects_bad_grid_and_dem():
    p = make_params(I.Params())
    assert _create(A.Grid(3, 8, 10.0, 10.0), p)[0] == A.M2P_EINVAL
    assert _create(A.Grid(8, 8, 0.0, 10.0), p)[0] == A.M2P_EINVAL
    assert _create(A.Grid(8, 8, 10.0, 10.0), p, prec=5)[0] == A.M2P_EINVAL
    dem = np.zeros((8, 8))
    dem[2, 3] = np.nan
    assert _create(A.Grid(8, 8, 10.0, 10.0), p, dem=dem)[0] == A.M2P_EINVAL
    bc = I.Params(bc=(0, 0, 2, 0))
    assert _create(A.Grid(8, 8, 10.0, 10.0), make_params(bc))[0] == A.M2P_EINVAL


@pytest.mark.parametrize("kw", [
    dict(flags=64),                                                      # unknown flag
    dict(flags=I.F_WELL_BALANCED | I.F_EARTH_PRESSURE, delta_int_deg=35.0),  # well-balanced with earth pressure
    dict(flags=I.F_SMOOTH_FRICTION, v_eps=0.0),                          # smooth friction without a speed
    dict(flags=I.F_SMOOTH_FRICTION, v_eps=math.nan),
    dict(flags=I.F_EARTH_PRESSURE, delta_b_deg=20.0, delta_int_deg=15.0),  # basal above internal friction
    dict(flags=I.F_EARTH_PRESSURE, delta_int_deg=90.0),
    dict(flags=I.F_EARTH_PRESSURE, delta_int_deg=-1.0)])
def test_create_rejects_bad_options(kw):
    """Option flags are validated before any device call: unknown bits, the
    well-balanced option with earth pressure, a smooth friction without a
    positive regularisation speed, and earth-pressure angles outside
    delta_b <= delta_int < 90 deg."""
    rc, h = _create(A.Grid(8, 8, 10.0, 10.0), make_params(I.Params(**kw)))
    assert rc == A.M2P_EINVAL and not h.value
    assert A.lib().m2p_last_error()


def test_null_arguments_rejected():
    L = A.lib()
    assert L.m2p_create(None, None, None, 0, None, None, None) == A.M2P_EINVAL
    assert L.m2p_step(None, None) == A.M2P_EINVAL
    assert L.m2p_run(None, 1) == A.M2P_EINVAL
    assert L.m2p_get_diag(None, None) == A.M2P_EINVAL
    assert L.m2p_device_count(None) == A.M2P_EINVAL
    L.m2p_destroy(None)


def test_no_device_means_no_context():
    """Without a GPU the create call reports a HIP error instead of silently
    falling back to any CPU path."""
    L = A.lib()
    n = C.c_int()
    A.check(L.m2p_device_count(C.byref(n)))
    if n.value > 0:
        pytest.skip("a GPU is visible")
    rc, h = _create(A.Grid(8, 8, 10.0, 10.0), make_params(I.Params()))
    assert rc == A.M2P_EHIP and not h.value


def _flops(stage, visc):
    out = (C.c_double * 5)()
    assert A.lib().m2p_stage_flops(stage, visc, out) == 0
    return np.array(list(out))


def test_stage_flop_count():
    """The per-cell operation tally of the stage arithmetic (used for the ALU
    roofline; the formulas in the folded forms of the FP32 kernels) against
    counts derived by hand from the formulas.

    Viscous term on minus off: two face fluxes (13 add, 16 mul, 2 div each),
    two y central differences (1 add, 1 mul, 1 div each), the two divergences
    (3 add, 2 div each) and two prefactors (3 mul each): 34 add, 40 mul,
    10 div.  Stage 2 minus stage 1: the Heun average (6 add, 6 mul) and the
    cell's speeds in both directions (thicknesses 2 mul 1 add; two pairs of
    desingularised velocities, 2 add 4 mul 1 div 1 cmp per pair;
    (1 - alpha)/2 (h + h^s) 1 add 1 mul; eps A_nn c twice, 4 mul; the four
    squared speeds 4 mul; |v| + sqrt(max(., 0)) four times: 4 add 4 sqrt
    4 cmp; the maxima over the phases and the running maxima, 4 cmp):
    16 add, 25 mul, 2 div, 4 sqrt, 10 cmp; plus the flux form of stage 1, which
    carries face fluxes as 2 H: its two central fluxes save 2 mul per
    component (24 mul), while both updates multiply each flux difference by
    dt over the cell width (dt / 2 dxi in stage 1, dt / dxi in stage 2): 16
    add, 49 mul, 2 div, 4 sqrt, 10 cmp."""
    f10, f11, f20, f21 = _flops(1, 0), _flops(1, 1), _flops(2, 0), _flops(2, 1)
    assert np.array_equal(f11 - f10, [34, 40, 10, 0, 0])
    assert np.array_equal(f21 - f20, [34, 40, 10, 0, 0])
    assert np.array_equal(f20 - f10, [16, 49, 2, 4, 10])
    # square roots: 4 face sides x 2 phase speeds, the new row's geometry, the
    # norm of the solid momentum in the Coulomb clamp
    assert f10[3] == 10
    assert 500 <= f10[:4].sum() <= 1200
    out = (C.c_double * 5)()
    assert A.lib().m2p_stage_flops(3, 0, out) == A.M2P_EINVAL
    assert A.lib().m2p_stage_flops(1, 0, None) == A.M2P_EINVAL
