"""The allocation-free loss (m2p_loss_noalloc) against m2p_loss, through the C ABI.

Two calls in a row on one GPU, the second on a smaller grid, each compared
bitwise with the allocating entry point (both sum the same per-block partials
in the same order)."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def test_loss_noalloc_equals_loss_twice_second_smaller():
    import torch

    from paper_2104_06784_amd import _abi as A
    from paper_2104_06784_amd import inputs as I
    from paper_2104_06784_amd.sim import Sim

    rng = np.random.default_rng(2104)
    got = []
    for n, prec in ((72, "f64"), (40, "f32")):
        _say(f"[noalloc] grid {n}x{n} {prec}")
        s = Sim(I.plane_bump_pile(n=n), precision=prec)
        s.run(12)
        s.synchronize()
        target = rng.uniform(0.0, 4.0, (n, n))
        ref = s.loss(target)
        tdev = torch.from_numpy(target).to("cuda")
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        A.check(A.lib().m2p_loss_noalloc(s._h, C.c_void_p(tdev.data_ptr()), C.c_void_p(out.data_ptr())),
                "m2p_loss_noalloc")
        s.synchronize()
        v = out.item()
        _say(f"[noalloc] loss {v!r} vs {ref!r}")
        assert v == ref and v > 0.0
        got.append(v)
        s.close()
    assert got[0] != got[1]


def test_loss_noalloc_rejects_null_and_missing_state():
    from paper_2104_06784_amd import _abi as A
    from paper_2104_06784_amd import inputs as I
    from paper_2104_06784_amd.sim import Sim

    s = Sim(I.plane_bump_pile(n=16), precision="f64")
    assert A.lib().m2p_loss_noalloc(s._h, None, None) == A.M2P_EINVAL
    t = Sim(I.plane_bump_pile(n=16), precision="f64", set_state=False)
    dummy = C.c_void_p(1)
    assert A.lib().m2p_loss_noalloc(t._h, dummy, dummy) == A.M2P_ESTATE
