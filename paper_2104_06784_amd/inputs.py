"""Seeded synthetic inputs for the two-phase shallow-flow step.

This module only *generates data*: digital elevation models (DEMs), release
piles, inflow hydrographs and parameter sets in SI units.  It holds none of
the method's arithmetic (no geometry, fluxes, sources or time stepping), so
both the FP64 CPU oracle and the HIP path can be driven from it.

The paper's own workloads (the Hsiaolin landslide and the DF004 debris flow,
Sect. 4) use government DEMs that are not distributed; the recipes below are
stand-ins that keep the paper's cell sizes (10 m and 5 m), release scale
(about 2.5e7 m^3 over about 57 ha, Sect. 4.1), an edge-segment inflow
(Sect. 4.2) and the Table 1 material parameters.

Conventions: arrays are row-major ``[ny, nx]`` (y outer), cell-centred, so
cell (i, j) sits at X = (i + 0.5) dx, Y = (j + 0.5) dy.  Thicknesses given to
a release are *vertical* thicknesses in metres.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Boundary modes per side (W, E, S, N).
BC_TRANSMISSIVE = 0
BC_WALL = 1
SIDE_W, SIDE_E, SIDE_S, SIDE_N = 0, 1, 2, 3

# Flags.
F_FLUID_PRESSURE_AS_PRINTED = 1
F_RK3 = 2                       # three-stage SSP Runge-Kutta instead of Heun
F_CENTRAL_UPWIND = 4            # central-upwind face flux (one-sided local speeds)
F_EARTH_PRESSURE = 8            # Savage-Hutter earth-pressure coefficients from delta_int
F_SMOOTH_FRICTION = 16          # smooth Coulomb friction (finite-difference checks of gradients)
F_WELL_BALANCED = 32            # well-balanced hydrostatic reconstruction of the face states (Mode-I)


@dataclasses.dataclass
class Params:
    """Material and numerical parameters, SI units (Sect. 3.1.2, Table 1)."""

    delta_b_deg: float = 16.0     # basal friction angle
    c_d: float = 6.0              # interphase drag coefficient
    inv_n_r: float = 1.0 / 268.0  # 1 / N_R (0 switches fluid friction and viscosity off)
    theta_b: float = 5.0          # fluid basal friction coefficient
    rho_s: float = 2700.0
    rho_f: float = 1000.0
    delta_int_deg: float = 35.0   # used only with F_EARTH_PRESSURE (the paper's model has no such coefficient)
    cfl: float = 0.1              # Sect. 2.2
    L: float = 1000.0             # length scale (m)
    H: float = 10.0               # thickness scale (m)
    chi: float = 0.0              # exponent of the aspect ratio in the basal pressure
    g: float = 9.81
    m_dry: float = 1e-6           # desingularisation thickness (m)
    a_min: float = 1.0            # floor on the CFL wave speed (m/s)
    bc: tuple = (BC_TRANSMISSIVE,) * 4
    flags: int = 0
    v_eps: float = 0.01           # regularisation speed (m/s) of F_SMOOTH_FRICTION


@dataclasses.dataclass
class Inflow:
    """One Mode-II inflow segment: ``ncells`` boundary cells from ``i0`` on
    ``side``, with a piecewise-linear hydrograph of discharge Q (m^3/s) and
    solid fraction over time (s)."""

    side: int
    i0: int
    ncells: int
    t: np.ndarray
    Q: np.ndarray
    phi_s: np.ndarray


@dataclasses.dataclass
class InflowState:
    """One Mode-II inflow segment given as the state of the inflowing flow:
    ``ncells`` boundary cells from ``i0`` on ``side``, with piecewise-linear
    hydrographs over time (s) of the vertical flow thickness h (m), the solid
    fraction and the speed v (m/s) of both phases along the inward normal."""

    side: int
    i0: int
    ncells: int
    t: np.ndarray
    h: np.ndarray
    phi_s: np.ndarray
    v: np.ndarray


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    dx: float
    dy: float
    params: Params
    dem: np.ndarray                       # [ny, nx] metres
    h_vert: np.ndarray                    # [ny, nx] initial vertical thickness (m)
    phi_s: np.ndarray                     # [ny, nx] initial solid fraction
    inflows: List[Inflow] = dataclasses.field(default_factory=list)
    inflow_states: List[InflowState] = dataclasses.field(default_factory=list)
    steps: int = 0
    precision: str = "f64"
    tan_mu: Optional[np.ndarray] = None   # optional per-cell tan(delta_b)
    vel: Optional[tuple] = None           # optional (vxs, vys, vxf, vyf) m/s

    @property
    def cells(self) -> int:
        return self.nx * self.ny


# ---------------------------------------------------------------------------
# grids and DEM recipes
# ---------------------------------------------------------------------------

def cell_centres(nx: int, ny: int, dx: float, dy: float):
    x = (np.arange(nx, dtype=np.float64) + 0.5) * dx
    y = (np.arange(ny, dtype=np.float64) + 0.5) * dy
    return np.meshgrid(x, y)  # X, Y with shape [ny, nx]


def fractal_noise(n: int, seed: int, exponent: float = 2.0, ny: Optional[int] = None) -> np.ndarray:
    """Spectral synthesis: white noise N(0,1), FFT, amplitude times |k|^-exponent
    (k = 0 removed), inverse FFT, real part, zero mean, peak-to-peak 1."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, n))
    kx = np.fft.fftfreq(n)
    ky = np.fft.fftfreq(ny)
    KX, KY = np.meshgrid(kx, ky)
    k = np.sqrt(KX * KX + KY * KY)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (-exponent)
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * amp))
    f -= f.mean()
    ptp = f.max() - f.min()
    return f / ptp if ptp > 0 else f


def fractal_dem(n: int, dx: float, seed: int, relief: float, tilt_deg: float = 0.0,
                ny: Optional[int] = None) -> np.ndarray:
    ny = n if ny is None else ny
    X, _ = cell_centres(n, ny, dx, dx)
    return relief * fractal_noise(n, seed, ny=ny) - X * math.tan(math.radians(tilt_deg))


def plane_dem(nx: int, ny: int, dx: float, dy: float, tilt_deg: float, axis: int = 0) -> np.ndarray:
    X, Y = cell_centres(nx, ny, dx, dy)
    return -(X if axis == 0 else Y) * math.tan(math.radians(tilt_deg))


def cylinder(nx, ny, dx, dy, xc, yc, radius, height) -> np.ndarray:
    X, Y = cell_centres(nx, ny, dx, dy)
    inside = (X - xc) ** 2 + (Y - yc) ** 2 <= radius * radius
    return np.where(inside, height, 0.0)


def half_ellipsoid(nx, ny, dx, dy, xc, yc, ax, ay, h0) -> np.ndarray:
    X, Y = cell_centres(nx, ny, dx, dy)
    r2 = ((X - xc) / ax) ** 2 + ((Y - yc) / ay) ** 2
    return np.where(r2 < 1.0, h0 * np.sqrt(np.clip(1.0 - r2, 0.0, None)), 0.0)


def paraboloid(nx, ny, dx, dy, xc, yc, radius, h0) -> np.ndarray:
    X, Y = cell_centres(nx, ny, dx, dy)
    r2 = ((X - xc) ** 2 + (Y - yc) ** 2) / (radius * radius)
    return np.where(r2 < 1.0, h0 * (1.0 - r2), 0.0)


def triangular_hydrograph(q_peak: float, t_peak: float, t_end: float, phi: float):
    t = np.array([0.0, t_peak, t_end], dtype=np.float64)
    Q = np.array([0.0, q_peak, 0.0], dtype=np.float64)
    return t, Q, np.full(3, phi, dtype=np.float64)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def plane_bump_pile(n: int = 128) -> Problem:
    """FP64 parity case: 128^2, dx = 10 m, 30 deg plane plus a 20 m Gaussian bump
    (sigma 150 m), 10 m cylinder of radius 200 m with solid fraction 0.6,
    delta_b = 20 deg, closed walls, CFL 0.5, 200 steps.  The bump and the pile
    are centred on the face Y = 640 m, so the problem is mirror-symmetric."""
    dx = 10.0
    X, Y = cell_centres(n, n, dx, dx)
    dem = -X * math.tan(math.radians(30.0)) + 20.0 * np.exp(
        -((X - 800.0) ** 2 + (Y - 640.0) ** 2) / (2.0 * 150.0 ** 2))
    h = cylinder(n, n, dx, dx, 320.0, 640.0, 200.0, 10.0)
    p = Params(delta_b_deg=20.0, delta_int_deg=35.0, cfl=0.5, bc=(BC_WALL,) * 4)
    return Problem("plane-bump-pile", n, n, dx, dx, p, dem, h, np.where(h > 0, 0.6, 0.0), steps=200, precision="f64")


def fractal_hydrograph(n: int = 1024, steps: int = 5000) -> Problem:
    """FP32-vs-FP64 case: 1024^2, dx = 5 m, fractal DEM (200 m relief) on a 20 deg
    tilt, Mode-II triangular hydrograph (peak 500 m^3/s at 180 s, end 360 s,
    solid fraction 0.5) on a 10-cell segment centred on the west side."""
    dx = 5.0
    dem = fractal_dem(n, dx, 2104, 200.0, tilt_deg=20.0)
    t, Q, ph = triangular_hydrograph(500.0, 180.0, 360.0, 0.5)
    seg = Inflow(SIDE_W, n // 2 - 5, 10, t, Q, ph)
    z = np.zeros((n, n))
    p = Params(delta_b_deg=16.0, bc=(BC_TRANSMISSIVE,) * 4)
    return Problem("fractal-hydrograph", n, n, dx, dx, p, dem, z, z.copy(), [seg], steps=steps, precision="f32")


def valley_event(n: int = 4096, steps: int = 20000) -> Problem:
    """Large event: 4096^2, dx = 5 m, exponential longitudinal relief (1.5 km),
    parabolic valley (100 m wall height at 500 m from the axis) plus 50 m of
    fractal roughness; half-ellipsoid release of 2.5e7 m^3 (600 m x 300 m),
    solid fraction 0.55, delta_b = 16 deg, transmissive."""
    dx = 5.0
    X, Y = cell_centres(n, n, dx, dx)
    yc = 0.5 * n * dx
    dem = (1500.0 * np.exp(-X / 3000.0) + 100.0 * ((Y - yc) / 500.0) ** 2
           + 50.0 * fractal_noise(n, 2105))
    V = 2.5e7
    h0 = 3.0 * V / (2.0 * math.pi * 600.0 * 300.0)
    h = half_ellipsoid(n, n, dx, dx, 1000.0, yc, 600.0, 300.0, h0)
    p = Params(delta_b_deg=16.0)
    return Problem("valley-event", n, n, dx, dx, p, dem, h, np.where(h > 0, 0.55, 0.0), steps=steps, precision="f32")


def ensemble_member(i: int) -> Problem:
    """Scenario i of the 256-member ensemble: side U{128..512}, dx = 10 m,
    fractal DEM minus a 20 deg tilt, delta_b ~ U(15, 30) deg, release volume
    lognormal (median 1e6 m^3, sigma 0.5), solid fraction U(0.4, 0.7)."""
    rng = np.random.default_rng(3000 + i)
    n = int(rng.integers(128, 513))
    delta = float(rng.uniform(15.0, 30.0))
    V = float(rng.lognormal(math.log(1e6), 0.5))
    phi = float(rng.uniform(0.4, 0.7))
    dx = 10.0
    dem = fractal_dem(n, dx, 3000 + i, 200.0, tilt_deg=20.0)
    hgt = 10.0
    r = math.sqrt(V / (hgt * math.pi))
    rmax = 0.2 * n * dx
    if r > rmax:
        r = rmax
        hgt = V / (math.pi * r * r)
    h = cylinder(n, n, dx, dx, 0.25 * n * dx, 0.5 * n * dx, r, hgt)
    p = Params(delta_b_deg=delta)
    return Problem(f"member-{i}", n, n, dx, dx, p, dem, h, np.where(h > 0, phi, 0.0), steps=2000, precision="f32")


def calibration_case(n: int = 512, truth: bool = False) -> Problem:
    """Adjoint case: 512^2, dx = 10 m, fractal DEM on a 20 deg tilt, 10 m cylinder
    (r = 200 m) at (1280, 2560) m, solid fraction 0.6, 2000 FP32 steps.  With
    ``truth`` the hidden per-cell friction tan(20 deg + 3 deg g) and the volume
    scale 1.2 are applied; otherwise the initial guess tan 20 deg, scale 1."""
    dx = 10.0
    dem = fractal_dem(n, dx, 5000, 200.0, tilt_deg=20.0)
    h = cylinder(n, n, dx, dx, 1280.0, 0.5 * n * dx, 200.0, 10.0)
    p = Params(delta_b_deg=20.0)
    if truth:
        gfield = smooth_field(n, 5001, 5.0)
        tan_mu = np.tan(np.radians(20.0 + 3.0 * gfield))
        h = 1.2 * h
    else:
        tan_mu = np.full((n, n), math.tan(math.radians(20.0)))
    return Problem("calibration", n, n, dx, dx, p, dem, h, np.where(h > 0, 0.6, 0.0), steps=2000,
                   precision="f32", tan_mu=tan_mu)


def smooth_field(n: int, seed: int, sigma_cells: float) -> np.ndarray:
    """Gaussian-filtered white noise normalised to [-1, 1] (periodic filter via FFT)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n)
    KX, KY = np.meshgrid(k, k)
    filt = np.exp(-2.0 * (math.pi * sigma_cells) ** 2 * (KX * KX + KY * KY))
    f = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    f -= f.min()
    return 2.0 * f / f.max() - 1.0


def paper_shaped(nx: int, ny: int, seed: int = 4000, precision: str = "f32") -> Problem:
    """Grid shapes of the paper's events (377 x 228 and 180 x 154 including the
    paper's ghost cells) on the ensemble DEM recipe with a central release."""
    dx = 10.0
    dem = fractal_dem(nx, dx, seed, 200.0, tilt_deg=20.0, ny=ny)
    h = cylinder(nx, ny, dx, dx, 0.3 * nx * dx, 0.5 * ny * dx, 0.15 * min(nx, ny) * dx, 10.0)
    return Problem(f"paper_{nx}x{ny}", nx, ny, dx, dx, Params(), dem, h,
                   np.where(h > 0, 0.5, 0.0), steps=10000, precision=precision)


def df004_shaped(precision: str = "f32") -> Problem:
    """Mode-II stand-in with the shape of the paper's second event (180 x 154
    cells of 5 m, inflow given as a state hydrograph on 30 boundary cells,
    12 minutes): a tilted fractal valley side, dry at the start, fed through
    30 cells of the west edge by a synthetic hydrograph (thickness rising to
    3 m at 2 min and falling to zero at 12 min, solid fraction 0.5, inward
    speed 2 -> 5 -> 1 m/s).  The event's DEM and measured hydrograph are not
    available; only the shapes are taken from the paper."""
    nx, ny, dx = 180, 154, 5.0
    dem = fractal_dem(nx, dx, 4004, 30.0, tilt_deg=15.0, ny=ny)
    z = np.zeros((ny, nx))
    seg = InflowState(SIDE_W, 62, 30, np.array([0.0, 120.0, 720.0]), np.array([0.0, 3.0, 0.0]),
                      np.array([0.5, 0.5, 0.5]), np.array([2.0, 5.0, 1.0]))
    return Problem("df004_shaped", nx, ny, dx, dx, Params(), dem, z, z.copy(), inflow_states=[seg],
                   steps=0, precision=precision)
