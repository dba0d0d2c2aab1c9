"""Batched ensembles (persistent work-list kernel + HIP graphs): every member
must equal a single-scenario run of the same tile height bitwise, and the
oracle to the FP64 parity bar."""
import sys

import numpy as np
import pytest

from paper_2104_06784_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small(i, nx, ny):
    dx = 10.0
    rng = np.random.default_rng(100 + i)
    dem = I.fractal_dem(nx, dx, 100 + i, 60.0, tilt_deg=float(rng.uniform(15, 25)), ny=ny)
    h = I.cylinder(nx, ny, dx, dx, 0.3 * nx * dx, 0.5 * ny * dx, 0.25 * min(nx, ny) * dx, 6.0 + i)
    bc = tuple(int(x) for x in rng.integers(0, 2, 4))
    p = I.Params(delta_b_deg=float(rng.uniform(15, 30)), cfl=0.2, bc=bc)
    tan_mu = None
    if i % 2 == 1:
        tan_mu = np.tan(np.radians(18.0 + 4.0 * rng.random((ny, nx))))
    return I.Problem(f"b{i}", nx, ny, dx, dx, p, dem, h, np.where(h > 0, 0.4 + 0.05 * i, 0.0), tan_mu=tan_mu)


SHAPES = [(40, 30), (61, 57), (64, 64), (130, 17), (97, 121)]


@pytest.mark.parametrize("blocks", [0, 3])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_members_equal_single_runs(precision, blocks):
    """blocks 0: a wavefront per work item (the flat kernel); 3 workgroups:
    twelve wavefronts walk the work list (the persistent kernel)."""
    from paper_2104_06784_amd.sim import Batch, Sim
    probs = [_small(i, nx, ny) for i, (nx, ny) in enumerate(SHAPES)]
    _say(f"[batch] {len(probs)} scenarios {precision} blocks={blocks}")
    b = Batch(probs, precision=precision)
    b.set_tile(8, blocks)
    b.set_graph(10)
    b.run(25)
    b.synchronize()
    for i, p in enumerate(probs):
        s = Sim(p, precision=precision, variant=2, tile_rows=8)
        s.run(25)
        Us, Ub = s.state(), b.state(i)
        assert np.array_equal(Us, Ub), (i, float(np.max(np.abs(Us - Ub))))
        ds, db = s.diag(), b.diag(i)
        assert ds["t"] == db["t"] and ds["steps"] == db["steps"] == 25


def test_batch_fp64_matches_oracle():
    import oracle
    from paper_2104_06784_amd.sim import Batch
    probs = [_small(i, nx, ny) for i, (nx, ny) in enumerate(SHAPES[:3])]
    b = Batch(probs, precision="f64")
    b.run(40)
    for i, p in enumerate(probs):
        o = oracle.OracleSim(p)
        o.run(40)
        Uo, Ub = o.state(), b.state(i)
        for k in range(6):
            sc = max(np.max(np.abs(Uo[k])), 1e-300)
            assert np.max(np.abs(Ub[k] - Uo[k])) <= 1e-12 * sc
        assert abs(b.diag(i)["t"] - o.diag()["t"]) <= 1e-12 * o.diag()["t"]


def test_graph_replay_equals_direct_launches():
    from paper_2104_06784_amd.sim import Batch
    probs = [_small(i, nx, ny) for i, (nx, ny) in enumerate(SHAPES)]
    a = Batch(probs, precision="f32")
    b = Batch(probs, precision="f32")
    a.set_graph(0)
    b.set_graph(7)
    for _ in range(3):  # replays with eager work and synchronisation between them
        a.run(15)
        b.run(15)
        a.synchronize()
        b.synchronize()
        for i in range(len(probs)):
            assert np.array_equal(a.state(i), b.state(i))


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_autotune_restores_state_and_keeps_results(precision):
    """The tuner's trial steps leave no trace: the state and scalars are restored
    bitwise, and later steps equal a fresh batch run with the chosen shape
    bitwise, in FP64 and in FP32 (results do not depend on the tile height)."""
    from paper_2104_06784_amd.sim import Batch
    probs = [_small(i, nx, ny) for i, (nx, ny) in enumerate(SHAPES)]
    a = Batch(probs, precision=precision)
    a.run(5)
    before = [a.state(i) for i in range(len(probs))]
    rows, blocks, ms = a.autotune(2)
    _say(f"[batch] autotune {precision} rows={rows} blocks={blocks} {ms:.3f} ms/step")
    assert rows in (8, 16, 32, 64) and blocks > 0 and ms > 0
    for i in range(len(probs)):
        assert np.array_equal(before[i], a.state(i))
        assert a.diag(i)["steps"] == 5
    a.run(10)
    c = Batch(probs, precision=precision)
    c.set_tile(rows, blocks)
    c.run(15)
    for i in range(len(probs)):
        assert np.array_equal(a.state(i), c.state(i))


def test_batch_rejects_bad_input():
    from paper_2104_06784_amd import _abi as A
    from paper_2104_06784_amd.sim import Batch
    p = _small(0, 20, 20)
    p.params.cfl = 2.0
    with pytest.raises(A.M2PError) as e:
        Batch([_small(1, 20, 20), p])
    assert e.value.code == A.M2P_EINVAL
