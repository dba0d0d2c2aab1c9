"""GPU runs whose memory or inputs come from outside the library: state
buffers owned by torch tensors (m2p_bind_buffers, PyTorch supplying device
memory) and DEM, release and results passed through ESRI ASCII grids (the
paper's GIS input and output, Sect. 1 and Sect. 3.1.2 Stages 1 and 3)."""
import sys

import numpy as np
import pytest

from paper_2104_06784_amd import inputs as I

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision,own_stream", [("f64", False), ("f32", False), ("f32", True)])
def test_torch_owned_state_buffers_bitwise(precision, own_stream):
    """The same run with the state in two torch tensors and in context-owned
    memory is bitwise equal (direct launches, and graph replay on a stream
    of its own); after each step the first tensor holds U^n."""
    import torch

    from paper_2104_06784_amd.sim import Sim

    n = 56
    prob = I.plane_bump_pile(n=n)
    _say(f"[io] torch buffers {precision} stream={own_stream}")
    need = Sim.buffer_bytes(n, n, precision)
    a = torch.empty(need, dtype=torch.uint8, device="cuda")
    b = torch.empty(need, dtype=torch.uint8, device="cuda")
    assert a.data_ptr() % 256 == 0 and b.data_ptr() % 256 == 0
    torch.cuda.synchronize()
    st = torch.cuda.Stream() if own_stream else None
    s1 = Sim(prob, precision=precision, buffers=(a, b), stream=st)
    s2 = Sim(prob, precision=precision, stream=torch.cuda.Stream() if own_stream else None)
    for _ in range(2):
        s1.run(40)
        s2.run(40)
        s1.synchronize()
        s2.synchronize()
        U1, U2 = s1.state(), s2.state()
        assert np.array_equal(U1, U2)
        dt = torch.float64 if precision == "f64" else torch.float32
        pitch = (n + 63) // 64 * 64
        esz = 8 if precision == "f64" else 4
        Ut = a[: 6 * n * pitch * esz].view(dt).view(6, n, pitch)[:, :, :n].cpu().numpy().astype(np.float64)
        assert np.array_equal(Ut, U1)
    assert np.max(np.abs(U1[1])) > 0


def test_torch_buffers_rejected_when_too_small():
    import torch

    from paper_2104_06784_amd.sim import Sim

    prob = I.plane_bump_pile(n=24)
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        Sim(prob, precision="f64", buffers=(small, small))


def test_gis_grids_drive_a_gpu_run(tmp_path):
    """DEM, release thickness and solid fraction written as ESRI ASCII grids
    and read back drive an FP64 GPU run that matches the oracle on the read
    grids; the output fields written as grids read back bitwise."""
    import oracle

    from paper_2104_06784_amd.gis import read_dem, read_esri_ascii, write_esri_ascii
    from paper_2104_06784_amd.sim import Sim

    src = I.plane_bump_pile(n=48)
    paths = {k: str(tmp_path / f"{k}.asc") for k in ("dem", "h", "phi")}
    write_esri_ascii(paths["dem"], src.dem, src.dx, x0=250000.0, y0=2.6e6)
    write_esri_ascii(paths["h"], src.h_vert, src.dx, x0=250000.0, y0=2.6e6)
    write_esri_ascii(paths["phi"], src.phi_s, src.dx, x0=250000.0, y0=2.6e6)
    dem, info = read_dem(paths["dem"])
    h, _ = read_esri_ascii(paths["h"])
    phi, _ = read_esri_ascii(paths["phi"])
    assert np.array_equal(dem, src.dem) and np.array_equal(h, src.h_vert) and np.array_equal(phi, src.phi_s)
    prob = I.Problem("gis", dem.shape[1], dem.shape[0], info["dx"], info["dx"], src.params, dem, h, phi)
    _say(f"[io] GIS-driven run {prob.nx}x{prob.ny}")
    g = Sim(prob, precision="f64")
    o = oracle.OracleSim(prob)
    dtg = np.array([g.step() for _ in range(40)])
    dto = o.run(40)
    np.testing.assert_allclose(dtg, dto, rtol=1e-12, atol=0)
    fg, fo = g.fields(), o.fields()
    for k in fg:
        scale = max(np.max(np.abs(fo[k])), 1e-300)
        assert np.max(np.abs(fg[k] - fo[k])) <= 1e-12 * scale, k
        p = str(tmp_path / f"out_{k}.asc")
        write_esri_ascii(p, fg[k], info["dx"], x0=info["x0"], y0=info["y0"])
        back, binfo = read_esri_ascii(p)
        assert np.array_equal(back, fg[k]) and binfo["x0"] == info["x0"], k
    assert np.max(fg["h"]) > 0 and np.max(np.abs(fg["vxs"])) > 0


def test_gis_dem_with_missing_cells_needs_a_fill(tmp_path):
    """A DEM grid with NODATA cells is refused by m2p_create; filled with the
    nearest data it runs."""
    from paper_2104_06784_amd import _abi as A
    from paper_2104_06784_amd.gis import read_dem, read_esri_ascii, write_esri_ascii
    from paper_2104_06784_amd.sim import Sim

    src = I.plane_bump_pile(n=32)
    dem = src.dem.copy()
    dem[10:12, 20] = np.nan
    p = str(tmp_path / "dem.asc")
    write_esri_ascii(p, dem, src.dx)
    raw, _ = read_esri_ascii(p)
    bad = I.Problem("nodata", 32, 32, src.dx, src.dy, src.params, raw, src.h_vert, src.phi_s)
    with pytest.raises(A.M2PError) as e:
        Sim(bad, precision="f64")
    assert e.value.code == A.M2P_EINVAL
    filled, _ = read_dem(p, fill="nearest")
    ok = I.Problem("filled", 32, 32, src.dx, src.dy, src.params, filled, src.h_vert, src.phi_s)
    s = Sim(ok, precision="f64")
    s.run(10)
    assert np.isfinite(s.state()).all()
