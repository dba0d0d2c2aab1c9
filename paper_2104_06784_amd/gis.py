"""ESRI ASCII grid input and output through the library (``m2p_esri_*``).

DEMs and initial fields come from GIS systems as ASCII grids and results go
back in that form (the paper's Sect. 1 and Sect. 3.1.2, Stages 1 and 3).
Arrays are [ny, nx] float64 with row 0 at the southern edge, as everywhere
in this package.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from . import _abi as A


def read_esri_ascii(path: str):
    """Return (values [ny, nx], info) with info = {dx, x0, y0, nodata}; x0, y0
    is the lower-left cell corner, nodata is NaN when the file has none.  Cells
    holding the NODATA value come back as NaN."""
    L = A.lib()
    g = A.Grid()
    x0, y0, nd = C.c_double(), C.c_double(), C.c_double()
    p = os.fsencode(path)
    A.check(L.m2p_esri_read(p, C.byref(g), C.byref(x0), C.byref(y0), C.byref(nd), None, 0), "m2p_esri_read")
    out = np.empty((g.ny, g.nx), dtype=np.float64)
    A.check(L.m2p_esri_read(p, C.byref(g), None, None, None, A.dptr(out), out.size), "m2p_esri_read")
    return out, {"dx": g.dx, "x0": x0.value, "y0": y0.value, "nodata": nd.value}


def write_esri_ascii(path: str, values, dx: float, x0: float = 0.0, y0: float = 0.0, nodata: float = -9999.0):
    """Write [ny, nx] values (row 0 south); non-finite values become nodata."""
    v = np.ascontiguousarray(values, dtype=np.float64)
    if v.ndim != 2 or not math.isfinite(nodata):
        raise ValueError("values must be [ny, nx] and nodata finite")
    g = A.Grid(v.shape[1], v.shape[0], float(dx), float(dx))
    A.check(A.lib().m2p_esri_write(os.fsencode(path), C.byref(g), float(x0), float(y0), float(nodata), A.dptr(v)),
            "m2p_esri_write")


def read_dem(path: str, fill=None):
    """Read a DEM grid for ``m2p_create``.  Cells without data are an error
    unless ``fill`` says how to fill them: a number (metres), or "nearest"
    (the value of the nearest cell with data, by grid distance).  Returns
    (dem [ny, nx], info) as :func:`read_esri_ascii`."""
    dem, info = read_esri_ascii(path)
    miss = ~np.isfinite(dem)
    if not miss.any():
        return dem, info
    if fill is None:
        raise ValueError(f"{path}: {int(miss.sum())} cells without data; pass fill= a value or 'nearest'")
    if miss.all():
        raise ValueError(f"{path}: no cell has data")
    if fill == "nearest":
        from scipy import ndimage
        _, (jj, ii) = ndimage.distance_transform_edt(miss, return_indices=True)
        return dem[jj, ii], info
    v = float(fill)
    if not math.isfinite(v):
        raise ValueError("fill value must be finite")
    out = dem.copy()
    out[miss] = v
    return out, info
