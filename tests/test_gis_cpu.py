"""ESRI ASCII grid reader and writer of the library (host only)."""
import numpy as np
import pytest

from paper_2104_06784_amd import _abi as A
from paper_2104_06784_amd.gis import read_esri_ascii, write_esri_ascii

SMALL = """NCOLS 3
nrows 2
xllcenter 105.0
yllcenter 205.0
cellsize 10
NODATA_value -9999
1 2 3
4 -9999 6
"""


def test_reads_a_hand_written_grid(tmp_path):
    p = tmp_path / "small.asc"
    p.write_text(SMALL)
    v, info = read_esri_ascii(str(p))
    # the first file row is the northern edge: it becomes the last array row
    assert np.array_equal(v, [[4, np.nan, 6], [1, 2, 3]], equal_nan=True)
    assert info == {"dx": 10.0, "x0": 100.0, "y0": 200.0, "nodata": -9999.0}


def test_round_trip_is_exact_and_maps_non_finite_to_nodata(tmp_path):
    rng = np.random.default_rng(3)
    dem = rng.standard_normal((37, 53)) * 123.456
    dem[5, 7] = np.nan
    p = tmp_path / "dem.asc"
    write_esri_ascii(str(p), dem, 5.0, x0=250000.5, y0=2.6e6, nodata=-9999.0)
    v, info = read_esri_ascii(str(p))
    assert np.array_equal(v, dem, equal_nan=True) and np.isnan(v[5, 7])
    assert info["dx"] == 5.0 and info["x0"] == 250000.5 and info["y0"] == 2.6e6


@pytest.mark.parametrize("text", [
    SMALL.replace("4 -9999 6\n", "4 -9999\n"),        # too few values
    SMALL + "7\n",                                    # too many values
    SMALL.replace("cellsize 10", "cellsize -1"),      # bad cell size
    SMALL.replace("NCOLS 3", "colour 3"),             # unknown key
    "ncols 3\nnrows 2\n",                             # truncated header
])
def test_malformed_grids_are_rejected(tmp_path, text):
    p = tmp_path / "bad.asc"
    p.write_text(text)
    with pytest.raises(A.M2PError) as e:
        read_esri_ascii(str(p))
    assert e.value.code == A.M2P_EINVAL


def test_missing_file_is_an_io_error(tmp_path):
    with pytest.raises(A.M2PError) as e:
        read_esri_ascii(str(tmp_path / "none.asc"))
    assert e.value.code == A.M2P_EIO


def test_dem_without_data_is_rejected_or_filled(tmp_path):
    from paper_2104_06784_amd.gis import read_dem
    p = tmp_path / "small.asc"
    p.write_text(SMALL)
    with pytest.raises(ValueError):
        read_dem(str(p))
    v, _ = read_dem(str(p), fill="nearest")
    assert np.isfinite(v).all() and v[0, 1] in (2.0, 4.0, 6.0)
    v, _ = read_dem(str(p), fill=7.5)
    assert v[0, 1] == 7.5 and v[0, 0] == 4.0 and v[1, 1] == 2.0


def test_nodata_dem_is_rejected_by_create(tmp_path):
    """A grid with a NODATA cell cannot reach m2p_create as a number: the NaN
    the reader returns is refused (needs no GPU: validation runs first)."""
    import ctypes as C
    from paper_2104_06784_amd.sim import make_params
    from paper_2104_06784_amd import inputs as I
    p = tmp_path / "small.asc"
    p.write_text("ncols 4\nnrows 4\nxllcorner 0\nyllcorner 0\ncellsize 10\nNODATA_value -9999\n"
                 "1 2 3 4\n4 -9999 6 7\n1 2 3 4\n4 5 6 7\n")
    v, info = read_esri_ascii(str(p))
    assert v.shape == (4, 4) and np.isnan(v).sum() == 1
    g = A.Grid(4, 4, info["dx"], info["dx"])
    prm = make_params(I.Params())
    h = C.c_void_p()
    rc = A.lib().m2p_create(C.byref(h), C.byref(g), C.byref(prm), A.M2P_FP64,
                            A.dptr(np.ascontiguousarray(v)), None, None)
    assert rc == A.M2P_EINVAL and not h.value
