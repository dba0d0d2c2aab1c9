"""Tangent and adjoint of the step on the GPU.

- the stage JVP (dual arithmetic of the executed scheme) against central
  finite differences of the stage itself (FP64);
- the stage VJP is the exact transpose of the JVP: <J du, lam> = <du, J^T lam>
  to 1e-12 (FP64), for several boundary modes, viscosity and a friction field;
- the checkpointed adjoint gradient of the deposit loss with respect to the
  per-cell friction field and the release volume against central finite
  differences of the FP64 CPU oracle with the same frozen time steps;
- FP32 adjoint against the FP64 adjoint; bitwise reproducibility.
"""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2104_06784_amd import inputs as I

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("oracle_lib")]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _prob(nx=40, ny=36, bc=(0, 0, 0, 0), visc=True, mu=True, seed=7, smooth=False):
    dx = 10.0
    dem = I.fractal_dem(nx, dx, seed, 40.0, tilt_deg=22.0, ny=ny)
    h = I.cylinder(nx, ny, dx, dx, 0.35 * nx * dx, 0.5 * ny * dx, 0.25 * min(nx, ny) * dx, 8.0)
    p = I.Params(delta_b_deg=20.0, cfl=0.2, bc=bc, inv_n_r=(1.0 / 268.0 if visc else 0.0),
                 flags=I.F_SMOOTH_FRICTION if smooth else 0, v_eps=0.05)
    tan_mu = None
    if mu:
        tan_mu = np.tan(np.radians(20.0 + 2.0 * I.smooth_field(max(nx, ny), seed + 1, 3.0)[:ny, :nx]))
    return I.Problem("adj", nx, ny, dx, dx, p, dem, h, np.where(h > 0, 0.6, 0.0), tan_mu=tan_mu)


def _moving_state(prob, steps=12):
    from paper_2104_06784_amd.sim import Sim
    s = Sim(prob, precision="f64")
    s.run(steps)
    return s.state()


def _dot(a, b):
    return float(np.sum(a * b))


def test_stage_jvp_matches_finite_difference():
    from paper_2104_06784_amd.sim import Sim
    prob = _prob()
    U = _moving_state(prob)
    rng = np.random.default_rng(1)
    # a generic point: resting or dry neighbours hold exactly equal values, so
    # minmod(0, 0) and max(a, a) sit on their kinks, where the derivative takes
    # the branch the values select and a finite difference sees one-sided
    # slopes.  Small noise on the wet cells removes the ties; perturbations
    # stay on wet cells.
    wet = (U[0] + U[3]) > 1e-3
    U = U + wet * 1e-3 * np.abs(U).max(axis=(1, 2))[:, None, None] * rng.random(U.shape)
    dU = rng.standard_normal(U.shape) * (np.abs(U) + 1e-3) * 1e-2 * wet
    lam = rng.standard_normal(U.shape)
    # freeze the step: the CFL step of the unperturbed state
    s2 = Sim(prob, precision="f64", set_state=False)
    s2.set_state_raw(U)
    dt = s2.step()
    s = Sim(prob, precision="f64", set_state=False)
    s.set_state_raw(U)
    s.set_dt_schedule([dt])
    _, dE = s.stage_jvp(dU)
    eps = 1e-6
    vals = []
    for sgn in (1, -1):
        q = Sim(prob, precision="f64", set_state=False)
        q.set_state_raw(U + sgn * eps * dU)
        q.set_dt_schedule([dt])
        E, _ = q.stage_jvp(np.zeros_like(U))
        vals.append(E)
    fd = (vals[0] - vals[1]) / (2 * eps)
    a, b = _dot(dE, lam), _dot(fd, lam)
    _say(f"[jvp] <dE,lam> {a:.12e} fd {b:.12e}")
    assert abs(a - b) <= 1e-6 * max(abs(a), abs(b))


CASES = [
    dict(bc=(0, 0, 0, 0), visc=True, mu=True),
    dict(bc=(1, 1, 1, 1), visc=True, mu=False),
    dict(bc=(1, 0, 0, 1), visc=False, mu=True, nx=61, ny=23),
    # fewer than five rows: every cell is an edge-ring cell of the gather
    dict(bc=(0, 1, 1, 0), visc=True, mu=True, nx=13, ny=4),
    # smooth friction option
    dict(bc=(0, 0, 1, 1), visc=True, mu=True, smooth=True),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("stage", [0, 1])
def test_stage_vjp_is_transpose_of_jvp(case, stage):
    from paper_2104_06784_amd.sim import Sim
    kw = dict(CASES[case])
    prob = _prob(**kw)
    U = _moving_state(prob)
    rng = np.random.default_rng(10 + case)
    s = Sim(prob, precision="f64", set_state=False)
    s.set_state_raw(U)
    dU = rng.standard_normal(U.shape)
    dmu = rng.standard_normal((prob.ny, prob.nx))
    lam = rng.standard_normal(U.shape)
    _, dE = s.stage_jvp(dU, dmu, stage=stage)
    li, gmu = s.stage_vjp(lam, stage=stage)
    lhs = _dot(dE, lam)
    rhs = _dot(dU, li) + _dot(dmu, gmu)
    _say(f"[vjp] case {case} stage {stage}: {lhs:.15e} {rhs:.15e}")
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs), 1e-300)


def _loss_oracle(prob, tan_mu, scale, dts, target):
    import dataclasses

    import oracle
    q = dataclasses.replace(prob, tan_mu=tan_mu, h_vert=prob.h_vert * scale)
    o = oracle.OracleSim(q)
    o.set_dt_schedule(dts)
    o.run(len(dts))
    h = o.fields()["h"]
    return 0.5 * float(np.sum((h - target) ** 2)) * prob.dx * prob.dy


def _calibration_case():
    prob = _prob(48, 44, bc=(0, 0, 0, 0), visc=True, mu=True, seed=21)
    mu_true = np.tan(np.radians(20.0 + 3.0 * I.smooth_field(48, 31, 4.0)[:44, :48]))
    return prob, mu_true


def test_adjoint_gradient_against_oracle_finite_differences():
    import dataclasses

    import oracle
    from paper_2104_06784_amd.sim import Sim
    prob, mu_true = _calibration_case()
    nsteps = 60
    # hidden truth on the oracle: friction field mu_true, volume x 1.2
    ot = oracle.OracleSim(dataclasses.replace(prob, tan_mu=mu_true, h_vert=prob.h_vert * 1.2))
    ot.run(nsteps)
    target = ot.fields()["h"]
    # base run's time steps, frozen for every finite difference
    ob = oracle.OracleSim(prob)
    dts = ob.run(nsteps)
    g = Sim(prob, precision="f64")
    loss, gmu, gvol = g.adjoint_run(nsteps, 16, target, 1.0)
    lo = _loss_oracle(prob, prob.tan_mu, 1.0, dts, target)
    _say(f"[adj] loss gpu {loss:.12e} oracle {lo:.12e}")
    assert abs(loss - lo) <= 1e-10 * lo
    rng = np.random.default_rng(5)
    eps = 1e-6
    for k in range(3):
        d = I.smooth_field(48, 40 + k, 3.0)[:44, :48] * (0.5 + rng.random())
        lp = _loss_oracle(prob, prob.tan_mu + eps * d, 1.0, dts, target)
        lm = _loss_oracle(prob, prob.tan_mu - eps * d, 1.0, dts, target)
        fd = (lp - lm) / (2 * eps)
        ad = float(np.sum(gmu * d))
        _say(f"[adj] mu direction {k}: adjoint {ad:.10e} oracle FD {fd:.10e}")
        assert abs(ad - fd) <= 1e-5 * max(abs(fd), 1e-30)
    lp = _loss_oracle(prob, prob.tan_mu, 1.0 + eps, dts, target)
    lm = _loss_oracle(prob, prob.tan_mu, 1.0 - eps, dts, target)
    fd = (lp - lm) / (2 * eps)
    _say(f"[adj] volume: adjoint {gvol:.10e} oracle FD {fd:.10e}")
    assert abs(gvol - fd) <= 1e-5 * abs(fd)
    assert np.all(np.isfinite(gmu)) and np.max(np.abs(gmu)) > 0


def test_adjoint_fp32_close_to_fp64_and_reproducible():
    import oracle
    from paper_2104_06784_amd.sim import Sim
    prob, _ = _calibration_case()
    nsteps = 60
    ot = oracle.OracleSim(prob)
    ot.run(nsteps)
    target = ot.fields()["h"] * 1.1
    res = {}
    for prec in ("f64", "f32", "f32"):
        g = Sim(prob, precision=prec)
        res.setdefault(prec, []).append(g.adjoint_run(nsteps, 25, target, 1.0))
    g64 = res["f64"][0][1]
    a, b = res["f32"]
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and a[2] == b[2]
    g32 = a[1]
    cos = float(np.sum(g32 * g64) / (np.linalg.norm(g32) * np.linalg.norm(g64)))
    rel = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    _say(f"[adj] fp32 vs fp64: cosine {cos:.6f}, rel L2 {rel:.3e}, vol {a[2]:.6e} vs {res['f64'][0][2]:.6e}")
    assert cos >= 0.999 and rel <= 1e-2
    assert abs(a[2] - res["f64"][0][2]) <= 1e-2 * abs(res["f64"][0][2])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_taped_adjoint_equals_checkpointed(prec):
    """With one segment (ckpt_every >= nsteps) the forward run writes the tape
    and nothing is recomputed; the loss, both gradients, the final state and
    the diagnostics are the same bits as with checkpoints every 7 and every 25
    steps (segments recomputed, the last one shorter)."""
    import oracle
    from paper_2104_06784_amd.sim import Sim
    prob, _ = _calibration_case()
    nsteps = 60
    ot = oracle.OracleSim(prob)
    ot.run(nsteps)
    target = ot.fields()["h"] * 1.1
    out = []
    for ck in (nsteps, 1000, 7, 25):
        g = Sim(prob, precision=prec)
        r = g.adjoint_run(nsteps, ck, target, 1.0)
        out.append((r, g.state(), g.diag()))
    for r, U, d in out[1:]:
        assert r[0] == out[0][0][0] and np.array_equal(r[1], out[0][0][1]) and r[2] == out[0][0][2]
        assert np.array_equal(U, out[0][1]) and d == out[0][2]


def test_autograd_function_matches_adjoint_and_descends():
    """DepositLoss (torch.autograd.Function over the adjoint) returns the
    library's gradient, and a few projected gradient steps on (mu, s) lower
    the deposit misfit towards the hidden parameters."""
    import dataclasses

    import torch

    import oracle
    from paper_2104_06784_amd.calibrate import DepositLoss
    from paper_2104_06784_amd.sim import Sim
    prob, mu_true = _calibration_case()
    nsteps = 60
    ot = oracle.OracleSim(dataclasses.replace(prob, tan_mu=mu_true, h_vert=prob.h_vert * 1.2))
    ot.run(nsteps)
    target = ot.fields()["h"]
    f = DepositLoss(prob, target, nsteps, ckpt_every=16, precision="f64")
    mu = torch.tensor(prob.tan_mu, dtype=torch.float64, requires_grad=True)
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    loss = f(mu, s)
    loss.backward()
    g = Sim(prob, precision="f64")
    l2, gmu2, gv2 = g.adjoint_run(nsteps, 16, target, 1.0)
    assert loss.item() == l2 and np.array_equal(mu.grad.numpy(), gmu2) and s.grad.item() == gv2
    with torch.no_grad():
        assert float(f(mu, s)) == l2  # forward-only path, same loss
    hist = [loss.item()]
    for it in range(4):
        with torch.no_grad():
            mu -= 0.02 * mu.grad / mu.grad.abs().max()
            s -= 0.05 * torch.sign(s.grad)
        mu.grad = None
        s.grad = None
        loss = f(mu, s)
        loss.backward()
        hist.append(loss.item())
    _say(f"[adj] calibration losses {['%.4e' % x for x in hist]}, s {float(s):.3f}")
    assert all(b < a for a, b in zip(hist, hist[1:]))


# ------------------------------------------------- gradients at full strength
#
# With the smooth-friction option the Coulomb term has no kink at rest, so
# central finite differences of the loss converge to the derivative the
# adjoint computes (minmod, the speed maxima and positivity keep kinks of
# their own; a difference that straddles one shows up as a larger error).


def _smooth(prob):
    p = dataclasses.replace(prob.params, flags=prob.params.flags | I.F_SMOOTH_FRICTION, v_eps=0.05)
    return dataclasses.replace(prob, params=p)


def test_adjoint_against_oracle_fd_64x64_200_steps_smooth_friction():
    """64 x 64 cells, 200 FP64 steps with smooth friction: the adjoint's loss
    equals the oracle's to 1e-10, and its gradient along the release-volume
    scale and along 8 random smooth friction directions matches central
    finite differences of the oracle's loss with the same frozen time steps
    to 1e-6 relative (step 1e-7; the step 1e-6 is reported beside it: the
    longer secant is more likely to straddle a kink of minmod, the speed
    maxima or positivity somewhere in the 200 steps)."""
    import oracle
    from paper_2104_06784_amd.sim import Sim
    n, nsteps = 64, 200
    prob = _smooth(_prob(n, n, bc=(0, 0, 0, 0), visc=True, mu=True, seed=23))
    mu_true = np.tan(np.radians(20.0 + 3.0 * I.smooth_field(n, 33, 4.0)))
    ot = oracle.OracleSim(dataclasses.replace(prob, tan_mu=mu_true, h_vert=prob.h_vert * 1.2))
    ot.run(nsteps)
    target = ot.fields()["h"]
    dts = oracle.OracleSim(prob).run(nsteps)
    g = Sim(prob, precision="f64")
    loss, gmu, gvol = g.adjoint_run(nsteps, 25, target, 1.0)
    lo = _loss_oracle(prob, prob.tan_mu, 1.0, dts, target)
    _say(f"[p12] 64^2 x {nsteps}: loss gpu {loss:.12e} oracle {lo:.12e}")
    assert abs(loss - lo) <= 1e-10 * lo
    rng = np.random.default_rng(12)
    worst = {1e-6: 0.0, 1e-7: 0.0}
    for k in range(8):
        d = I.smooth_field(n, 60 + k, 3.0) * (0.5 + rng.random())
        ad = float(np.sum(gmu * d))
        for eps in worst:
            fd = (_loss_oracle(prob, prob.tan_mu + eps * d, 1.0, dts, target)
                  - _loss_oracle(prob, prob.tan_mu - eps * d, 1.0, dts, target)) / (2 * eps)
            e = abs(ad - fd) / abs(fd)
            worst[eps] = max(worst[eps], e)
            _say(f"   friction direction {k} step {eps:g}: adjoint {ad:.12e} FD {fd:.12e} rel {e:.2e}")
    for eps in worst:
        fd = (_loss_oracle(prob, prob.tan_mu, 1.0 + eps, dts, target)
              - _loss_oracle(prob, prob.tan_mu, 1.0 - eps, dts, target)) / (2 * eps)
        ev = abs(gvol - fd) / abs(fd)
        _say(f"   volume step {eps:g}: adjoint {gvol:.12e} FD {fd:.12e} rel {ev:.2e}")
        worst[eps] = max(worst[eps], ev)
    assert worst[1e-7] <= 1e-6


def _calibration_target(prec, smooth, nsteps):
    from paper_2104_06784_amd.sim import Sim
    truth = I.calibration_case(truth=True)
    truth = _smooth(truth) if smooth else truth
    t = Sim(truth, precision=prec)
    t.run(nsteps)
    return t.fields()["h"]


def test_adjoint_calibration_full_length_directional_fd_fp64():
    """The calibration workload at full size and length (512^2, 2000 steps,
    checkpoint every 100, smooth friction), FP64: the adjoint's directional
    derivative along a smooth friction field and along the volume scale
    against central differences of the same loss computed by the forward
    path with the same frozen time steps, to 1e-6 relative."""
    from paper_2104_06784_amd.sim import Sim
    nsteps = 2000
    prob = _smooth(I.calibration_case())
    target = _calibration_target("f64", True, nsteps)
    _say("[p12] 512^2 x 2000 FP64: base steps")
    base = Sim(prob, precision="f64")
    dts = np.array([base.step() for _ in range(nsteps)])
    a = Sim(prob, precision="f64")
    loss, gmu, gvol = a.adjoint_run(nsteps, 100, target, 1.0)
    assert abs(loss - base.loss(target)) <= 1e-12 * loss

    def L(mu_shift=None, scale=1.0):
        q = dataclasses.replace(prob, tan_mu=prob.tan_mu + (0.0 if mu_shift is None else mu_shift),
                                h_vert=prob.h_vert * scale)
        s = Sim(q, precision="f64")
        s.set_dt_schedule(dts)
        s.run(nsteps)
        return s.loss(target)

    eps = 1e-6
    d = I.smooth_field(512, 77, 5.0) * 0.5
    fd = (L(eps * d) - L(-eps * d)) / (2 * eps)
    ad = float(np.sum(gmu * d))
    fv = (L(scale=1.0 + eps) - L(scale=1.0 - eps)) / (2 * eps)
    _say(f"   friction: adjoint {ad:.12e} FD {fd:.12e} rel {abs(ad - fd) / abs(fd):.2e}; "
         f"volume: adjoint {gvol:.12e} FD {fv:.12e} rel {abs(gvol - fv) / abs(fv):.2e}")
    assert abs(ad - fd) <= 1e-6 * abs(fd)
    assert abs(gvol - fv) <= 1e-6 * abs(fv)


@pytest.mark.parametrize("smooth", [False, True])
def test_adjoint_fp32_against_fp64_calibration_full_length(smooth):
    """The calibration workload at full size and length (512^2, 2000 steps,
    checkpoint every 100, 20 recomputed segments): the FP32 adjoint's
    friction gradient against the FP64 adjoint's, cosine >= 0.999 and
    relative L2 <= 1e-2, and the volume derivative to 1e-2 -- with the
    paper's stop-clamp and with smooth friction."""
    from paper_2104_06784_amd.sim import Sim
    nsteps = 2000
    prob = _smooth(I.calibration_case()) if smooth else I.calibration_case()
    target = _calibration_target("f64", smooth, nsteps)
    res = {}
    for prec in ("f64", "f32"):
        g = Sim(prob, precision=prec)
        res[prec] = g.adjoint_run(nsteps, 100, target, 1.0)
    g64, g32 = res["f64"][1], res["f32"][1]
    cos = float(np.sum(g32 * g64) / (np.linalg.norm(g32) * np.linalg.norm(g64)))
    rel = float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64))
    v64, v32 = res["f64"][2], res["f32"][2]
    _say(f"[p12] calibration 512^2 x 2000 smooth={smooth}: cosine {cos:.6f} rel L2 {rel:.3e} volume {v32:.6e} vs {v64:.6e}")
    assert cos >= 0.999 and rel <= 1e-2
    assert abs(v32 - v64) <= 1e-2 * abs(v64)
