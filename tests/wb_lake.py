"""Lake-at-rest inputs of the well-balanced option's tests (oracle pins and
GPU parity)."""
import numpy as np

from paper_2104_06784_amd import inputs as I


def lake(along_y=False, wb=True, n=64, m=24, seed=5, flat_edges=True, level_above=5.0):
    """A lake at rest on a bed that varies in one direction only (a smoothed
    random profile of 30 m relief, flat within four cells of its two ends so the
    ghost cells' copies continue the lake), closed walls, fully wet: eta = eps c^2 m
    = (level - b) / L per cell, no momentum."""
    rng = np.random.default_rng(seed)
    prof = np.cumsum(rng.standard_normal(n))
    prof = np.convolve(prof, np.ones(5) / 5, mode="same")
    prof = (prof - prof.min()) / np.ptp(prof) * 30.0
    if flat_edges:
        prof[:4] = prof[4]
        prof[-4:] = prof[-5]
    nx, ny = (m, n) if along_y else (n, m)
    dx = 10.0
    dem = np.tile(prof[:, None], (1, m)) if along_y else np.tile(prof, (m, 1))
    p = I.Params(delta_b_deg=20.0, cfl=0.25, bc=(1, 1, 1, 1), flags=I.F_WELL_BALANCED if wb else 0)
    z = np.zeros((ny, nx))
    prob = I.Problem("lake", nx, ny, dx, dx, p, dem, z, z.copy(), [])
    eps = p.H / p.L
    b = dem / p.L
    bp = np.pad(b, 1, mode="reflect", reflect_type="odd")  # the DEM's linear extension
    bX = (bp[1:-1, 2:] - bp[1:-1, :-2]) / (2 * dx / p.L)
    bY = (bp[2:, 1:-1] - bp[:-2, 1:-1]) / (2 * dx / p.L)
    c2 = 1.0 / (1.0 + bX ** 2 + bY ** 2)
    U = np.zeros((6, ny, nx))
    U[3] = np.maximum((dem.max() + level_above) / p.L - b, 0.0) / (eps * c2)
    return prob, U
