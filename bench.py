"""Throughput of the two-phase shallow-flow step on one MI355X.

``python bench.py [--steps K] [--warmup W]`` times K steps of the 4096^2
large-event workload (fractal valley DEM, 2.5e7 m^3 release, FP32 state with
FP64 dt / time / volume sums) with the inputs resident in HBM, and prints one
JSON line: Mcell-steps/s; the roofline of the dominant kernel (stage 2, timed
live with HIP events on the stream it runs on), which is bound by vector-ALU
issue: algorithmic FLOPs per launch over the launch time against the non-packed
vector peak, with its HBM rate and fraction beside it; the batched-ensemble and
forward+adjoint throughputs; and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-steps/s (fwd, batched, fwd+adjoint) + % HBM roofline at fixed accuracy"
HBM_PEAK_GBS = 8000.0
# vector ALU peak without packed FP32 (the kernels are built without packed
# instructions): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz; the
# FP64 vector peak is the same 78.6 TFLOP/s
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# algorithmic bytes per cell and launch (S = bytes per scalar): stage 1 reads
# U^n (6 fields) and the DEM and writes U* (6); stage 2 reads U* (6), the
# cell's own U^n (6) and the DEM and writes U^{n+1} (6)
FIELDS_STAGE1 = 13
FIELDS_STAGE2 = 19


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the HIP sources (comments and blank lines removed) and of the
    build flags: the counters recorded in profiles/ apply only while this hash
    is unchanged, i.e. while the code they were taken on is unchanged."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2104_06784_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".h", ".hip")):
            text = open(os.path.join(csrc, f), encoding="utf-8").read()
            code = "\n".join(ln.rstrip() for ln in re.sub(r"//[^\n]*", "", text).splitlines() if ln.strip())
            h.update(f.encode())
            h.update(code.encode())
    h.update(open(os.path.join(ROOT, "paper_2104_06784_amd", "build_lib.py"), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(n: int, precision: str):
    """HBM bytes per stage-2 launch from the rocprofv3 counter summary in
    profiles/, if it was taken on the current kernel sources and workload."""
    path = os.path.join(ROOT, "profiles", f"stage2_valley_event_{n}_{precision}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic_json:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_source_hash") == kernel_source_hash():
                return rec["stage2_hbm_bytes_per_launch"]
    return None


def stage_flops(stage: int, visc: bool) -> float:
    """Algorithmic FLOPs of one cell in one stage (add, mul, div, sqrt)."""
    import ctypes as C

    from paper_2104_06784_amd import _abi
    out = (C.c_double * 5)()
    _abi.check(_abi.lib().m2p_stage_flops(stage, 1 if visc else 0, out), "m2p_stage_flops")
    return float(out[0] + out[1] + out[2] + out[3])


def recorded_valu(n: int, precision: str):
    """VALU busy fraction of the stage-2 kernel from the rocprofv3 counter
    summary in profiles/, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"stage_kernels_valley_event_{n}_{precision}_valu_counters.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("valu_json:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_source_hash") == kernel_source_hash():
                return rec
    return None


def cpu_baseline(prob, nsteps: int) -> dict:
    """The FP64 oracle (unchanged) on the host cores: one warm-up step, then
    three timed runs of nsteps steps of the full grid (the paper's protocol
    averages three runs), their mean as the value and the best beside it; one
    step on one thread (the paper's single-core comparison); and the small
    plane-bump-pile workload (128^2, 200 steps) on all threads."""
    import oracle

    from paper_2104_06784_amd import inputs
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    threads = min(threads, 16)
    used = oracle.set_threads(threads)
    o = oracle.OracleSim(prob)
    o.run(1)
    els = []
    for _ in range(3):
        t0 = time.perf_counter()
        o.run(nsteps)
        els.append(time.perf_counter() - t0)
    el = sum(els) / len(els)
    oracle.set_threads(1)
    o1 = oracle.OracleSim(prob)
    t0 = time.perf_counter()
    o1.run(1)
    el1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    small = inputs.plane_bump_pile()
    os_ = oracle.OracleSim(small)
    t0 = time.perf_counter()
    os_.run(small.steps)
    els_ = time.perf_counter() - t0
    return {"value": prob.cells * nsteps / el / 1e6, "unit": "Mcell-steps/s", "cores": used, "kind": "oracle",
            "sample": f"mean of 3 runs of {nsteps} steps of the full {prob.nx}x{prob.ny} grid after one warm-up "
                      f"step (FP64, OpenMP over rows on {used} threads), {el:.2f} s each; single thread: 1 step, "
                      f"{el1:.1f} s; plane-bump-pile 128^2: {small.steps} steps, {els_:.2f} s",
            "best_value": round(prob.cells * nsteps / min(els) / 1e6, 3),
            "single_thread_value": round(prob.cells / el1 / 1e6, 3),
            "plane_bump_pile_value": round(small.cells * small.steps / els_ / 1e6, 3)}


def bench_batched(stream, steps: int, warmup: int, nscen: int = 256) -> dict:
    """Ensemble: nscen scenarios of sides U{128..512} advanced together by the
    persistent work-list kernels (autotuned tile shape, graph replay), against
    the same scenarios run one after another with single-scenario contexts."""
    import torch

    from paper_2104_06784_amd import inputs
    from paper_2104_06784_amd.sim import Batch, Sim

    log(f"[bench] batched: generating {nscen} scenarios")
    probs = [inputs.ensemble_member(i) for i in range(nscen)]
    cells = sum(p.cells for p in probs)
    b = Batch(probs, precision="f32", stream=stream)
    rows, blocks, tune_ms = b.autotune(3)
    b.run(warmup)
    b.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    b.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    b.synchronize()
    ms_b = e0.elapsed_time(e1)
    del b
    log("[bench] batched: one-by-one reference")
    sims = [Sim(p, precision="f32", stream=stream) for p in probs]
    for s_ in sims:
        s_.run(warmup)
    torch.cuda.synchronize()
    e0.record(stream)
    for s_ in sims:
        s_.run(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_1 = e0.elapsed_time(e1)
    for s_ in sims:
        if s_.diag()["status"] != 0:
            raise SystemExit("device status set in the one-by-one reference")
    del sims
    vb = cells * steps / (ms_b / 1e3) / 1e6
    v1 = cells * steps / (ms_1 / 1e3) / 1e6
    return {"value": round(vb, 2), "unit": "Mcell-steps/s", "scenarios": nscen, "cells": cells, "steps": steps,
            "ms_per_step": round(ms_b / steps, 4), "tile_rows": rows, "blocks": blocks,
            "one_by_one_value": round(v1, 2), "one_by_one_ms_per_step": round(ms_1 / steps, 4),
            "speedup_vs_one_by_one": round(vb / v1, 3)}


def bench_sweep(stream, steps: int) -> dict:
    """Single-scenario forward over the paper's mesh sizes (Sect. 3.2: 10k to
    1M cells, plus its two events' grids 377 x 228 and 180 x 154), FP32,
    steps replayed from HIP graphs and launched kernel by kernel."""
    import math

    from paper_2104_06784_amd import inputs
    from paper_2104_06784_amd.sim import Sim
    import torch
    rows = []
    shapes = [(int(round(math.sqrt(c))),) * 2 for c in (10_000, 50_000, 100_000, 250_000, 500_000, 1_000_000)]
    for nx, ny in shapes + [(377, 228), (180, 154)]:
        prob = inputs.paper_shaped(nx, ny)
        rec = {"nx": nx, "ny": ny, "cells": nx * ny}
        for chunk, key in ((32, "graph"), (0, "direct")):
            sim = Sim(prob, precision="f32", stream=stream)
            sim.set_graph(chunk)
            sim.run(64)
            sim.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            sim.run(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            if sim.diag()["status"] != 0:
                raise SystemExit(f"device status in the mesh sweep at {nx}x{ny}")
            rec[key] = round(nx * ny * steps / (ms / 1e3) / 1e6, 1)
            rec[key + "_us_per_step"] = round(ms * 1e3 / steps, 2)
            del sim
        rows.append(rec)
        log(f"[bench] sweep {nx}x{ny}: {rec['graph']} Mcell-steps/s (graph), {rec['direct']} (direct)")
    return {"unit": "Mcell-steps/s", "steps": steps, "precision": "f32", "rows": rows}


def bench_variants(stream, steps: int, prob3) -> dict:
    """The scheme variants on their workloads: the three-stage Runge-Kutta,
    central-upwind flux, earth-pressure and well-balanced options on the
    large event (prob3, FP32, tiled kernel),
    and Mode-II inflow as a state hydrograph on the paper's second event's
    grid shape (180 x 154, graph replay) next to the same grid without the
    segment."""
    import torch

    from paper_2104_06784_amd import inputs
    from paper_2104_06784_amd.sim import Sim

    def timed(sim, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.run(k)
        e1.record(stream)
        torch.cuda.synchronize()
        if sim.diag()["status"] != 0:
            raise SystemExit("device status in the variants leg")
        return e0.elapsed_time(e1)

    out = {}
    for key, flag in (("rk3", inputs.F_RK3), ("central_upwind", inputs.F_CENTRAL_UPWIND),
                      ("earth_pressure", inputs.F_EARTH_PRESSURE), ("well_balanced", inputs.F_WELL_BALANCED)):
        p3 = dataclasses.replace(prob3, params=dataclasses.replace(prob3.params, flags=flag))
        sim = Sim(p3, precision="f32", stream=stream)
        sim.run(5)
        ms = timed(sim, steps)
        out[key] = {"value": round(p3.cells * steps / (ms / 1e3) / 1e6, 2), "unit": "Mcell-steps/s",
                    "ms_per_step": round(ms / steps, 4), "steps": steps, "cells": p3.cells}
        del sim
    pd = inputs.df004_shaped()
    k = 50 * steps
    rec = {"nx": pd.nx, "ny": pd.ny, "steps": k}
    for key, prob in (("state_inflow", pd), ("no_inflow", dataclasses.replace(pd, inflow_states=[]))):
        sim = Sim(prob, precision="f32", stream=stream)
        sim.run(64)
        ms = timed(sim, k)
        rec[key + "_us_per_step"] = round(ms * 1e3 / k, 2)
        if key == "state_inflow":
            d = sim.diag()
            rec["simulated_s"] = round(d["t"], 2)
            rec["inflow_m3"] = round(-(d["out_s"] + d["out_f"]), 1)  # state segments: negative outflow
        del sim
    out["mode2_state"] = rec
    log(f"[bench] variants: rk3 {out['rk3']['value']}, central-upwind {out['central_upwind']['value']}, "
        f"earth pressure {out['earth_pressure']['value']}, well-balanced {out['well_balanced']['value']} "
        f"Mcell-steps/s; state inflow "
        f"{rec['state_inflow_us_per_step']} us/step ({rec['no_inflow_us_per_step']} without)")
    return out


def bench_adjoint(stream, nsteps: int, ckpt: int) -> dict:
    """Calibration case (512^2): gradient of the deposit misfit with respect to the per-cell
    friction field and the release volume through nsteps FP32 steps
    (checkpoint every ckpt steps, segments recomputed; ckpt >= nsteps tapes
    the whole forward run), against the plain forward run of the same
    workload."""
    import torch

    from paper_2104_06784_amd import inputs
    from paper_2104_06784_amd.sim import Sim

    log("[bench] adjoint: target from the hidden-parameter run")
    truth = inputs.calibration_case(truth=True)
    t = Sim(truth, precision="f32", stream=stream)
    t.run(nsteps)
    target = t.fields()["h"]
    del t
    prob = inputs.calibration_case()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f = Sim(prob, precision="f32", stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    f.run(nsteps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1)
    del f
    g = Sim(prob, precision="f32", stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, gmu, gvol = g.adjoint_run(nsteps, ckpt, target, 1.0)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    cells = prob.cells
    return {"value": round(cells * nsteps / sec / 1e6, 2), "unit": "Mcell-steps/s", "cells": cells,
            "steps": nsteps, "checkpoint_every": ckpt, "seconds": round(sec, 3),
            "forward_only_value": round(cells * nsteps / (ms_fwd / 1e3) / 1e6, 2),
            "cost_vs_forward": round(sec / (ms_fwd / 1e3), 2), "loss": loss,
            "grad_mu_l2": float(np.linalg.norm(gmu)), "grad_vol": gvol}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=4096, help="grid side of the large-event workload")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=50, help="0 skips the batched-ensemble measurement")
    ap.add_argument("--adjoint-steps", type=int, default=2000, help="0 skips the forward+adjoint measurement")
    ap.add_argument("--sweep-steps", type=int, default=1000, help="0 skips the mesh-size sweep")
    ap.add_argument("--variant-steps", type=int, default=30,
                    help="steps of each scheme option on the large event (x50 on the Mode-II grid); 0 skips the variants")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, run 3 device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch

    from paper_2104_06784_amd import inputs
    from paper_2104_06784_amd.sim import Sim

    log(f"[bench] generating the valley event at {args.n}^2")
    prob = inputs.valley_event(n=args.n)
    stream = torch.cuda.Stream()
    sim = Sim(prob, precision=args.precision, stream=stream, variant=args.variant)
    log("[bench] warmup")
    sim.run(args.warmup)
    sim.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    sim.set_profiling(True)
    sim.kernel_times()  # clear
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    ev0.record(stream)
    sim.run(args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    kt, nk = sim.kernel_times()
    sim.set_profiling(False)
    d = sim.diag()
    if d["status"] != 0 or not np.isfinite(d["t"]):
        raise SystemExit(f"device status {d['status']} after the timed steps")
    cells = prob.cells
    S = 4 if args.precision == "f32" else 8
    value = cells * args.steps / (ms / 1e3) / 1e6
    t2 = kt[1] / nk / 1e3
    t1 = kt[0] / nk / 1e3
    bytes2 = FIELDS_STAGE2 * S * cells
    gbs = bytes2 / t2 / 1e9
    visc = prob.params.inv_n_r > 0
    fl2 = stage_flops(2, visc)
    ach = fl2 * cells / t2 / 1e12
    valu = recorded_valu(args.n, args.precision)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"large event {prob.nx}x{prob.ny}, dx 5 m, fractal valley DEM, 2.5e7 m^3 "
                               f"half-ellipsoid release, phi_s 0.55, {args.precision} state + FP64 dt/volume",
                   "cells": cells, "parallelism": "single GPU"},
        # the stage kernels are bound by vector-ALU instruction issue, not by
        # HBM: achieved = algorithmic FLOPs of a stage-2 launch / its time
        "roofline": {"bound": "alu", "achieved": round(ach, 2), "peak": round(ALU_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(ach / ALU_PEAK_TFLOPS, 4),
                     "traffic": recorded_traffic(args.n, args.precision),
                     "kernel": "stage 2 (U* stencil + own U^n + DEM -> U^{n+1})",
                     "flops_per_cell": fl2, "flops_per_launch": fl2 * cells,
                     "kernel_ms": round(t2 * 1e3, 4), "stage1_ms": round(t1 * 1e3, 4),
                     "finalize_ms": round(kt[2] / nk, 4),
                     "valu_busy": None if valu is None else valu.get("stage2_valu_busy"),
                     "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes_per_launch": bytes2,
                             "step_algorithmic_frac": round((FIELDS_STAGE1 + FIELDS_STAGE2) * S * cells
                                                            / (ms / args.steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}},
    }
    log(f"[bench] {value:.1f} Mcell-steps/s, stage2 {t2 * 1e3:.3f} ms ({ach:.1f} TFLOP/s, {gbs:.0f} GB/s)")
    del sim
    if args.batched_steps > 0:
        out["batched"] = bench_batched(stream, args.batched_steps, 5)
        log(f"[bench] batched {out['batched']['value']:.1f} Mcell-steps/s "
            f"({out['batched']['speedup_vs_one_by_one']:.2f}x one-by-one)")
    if args.adjoint_steps > 0:
        # the whole run taped (2 x 2000 states of 6.3 MB fit in HBM easily):
        # the forward writes the tape and the reverse sweep recomputes nothing
        out["fwd_adjoint"] = bench_adjoint(stream, args.adjoint_steps, args.adjoint_steps)
        log(f"[bench] forward+adjoint {out['fwd_adjoint']['value']:.1f} Mcell-steps/s "
            f"({out['fwd_adjoint']['cost_vs_forward']:.1f}x the forward)")
    if args.sweep_steps > 0:
        out["mesh_sweep"] = bench_sweep(stream, args.sweep_steps)
    if args.variant_steps > 0:
        out["variants"] = bench_variants(stream, args.variant_steps, prob)
    if args.copy_probe_mib > 0:
        # plain device-to-device copies of known size, so that hardware byte
        # counters of the step kernels can be calibrated against them
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 4 * n
        del a, b
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: {args.cpu_steps} oracle steps")
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
