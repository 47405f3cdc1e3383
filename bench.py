#!/usr/bin/env python3
"""Throughput of the IB-GM step on one MI355X.

Workload: 3-D periodic unit cube, 256^3 MAC grid, rho = 1, mu = 0.01,
dt = 5e-4; an ellipsoidal shell (semi-axes 0.3/0.25/0.2) triangulated into
65,536 points joined by zero-rest-length links of stiffness 1; fluid at rest.
One step = Steps 1a-3f of the method (interpolate, evolve, link force, spread,
explicit momentum, three momentum sweeps, three pressure-increment sweeps and
the pressure update), all in the library's HIP kernels, inputs resident in HBM.

Prints ONE JSON line: IB steps/s under the mixed policy (FP32 grid, FP64
positions and pressure) as `value`, the FP64 run beside it, per-kernel times
from HIP events recorded on the library's stream over the timed region, the
roofline of the dominant kernel, the error of each precision against the
FP64 oracle after the oracle's sample steps, and the oracle's own rate on the
host cores as `cpu_baseline`.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# HBM bytes per launch of the dominant kernel from hardware counters (FETCH_SIZE
# x 2.0 + WRITE_SIZE x 1.0, calibrated on a device copy), taken on the kernel
# as it is built now; see profiles/hbm_counters_shell3d_256.md.  None when not
# measured for the current build.
TRAFFIC_BYTES = {"explicit": 1.0553e9}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--points", type=int, default=65536)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="let ib_tune pick the sweep tiles (the library defaults are faster "
                         "on the 256^3 step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate CPU budget of the oracle sample")
    ap.add_argument("--config2-steps", type=int, default=1000,
                    help="steps of the 512^2 ellipse run compared with the FP64 oracle in "
                         "every precision (part of the CPU leg; 0 = skip)")
    ap.add_argument("--ensemble-steps", type=int, default=500,
                    help="steps of the batched 2-D ensemble (0 = skip it)")
    ap.add_argument("--closure", choices=("full", "small", "off"), default="full",
                    help="learned closure: 128^3 coarse vs 256^3 fine (full), 32^3 vs 64^3 "
                         "(small) or skip")
    ap.add_argument("--closure-oracle-interval", type=int, default=4, metavar="K",
                    help="compare the closure rollout after interval K with the FP64 oracle's "
                         "own fine run (0: skip)")
    ap.add_argument("--cylinder", type=int, nargs="*", default=[256, 128], metavar="N",
                    help="grid sizes of the 3-D cylinder row (100 steps each, mixed and "
                         "FP64); none to skip")
    ap.add_argument("--no-channel", action="store_true",
                    help="skip the channel row (the 256^3 shell between no-slip walls)")
    ap.add_argument("--no-poisson", action="store_true",
                    help="skip the directional-split Poisson row (three line-solve sweeps)")
    ap.add_argument("--poisson-only", action="store_true",
                    help="run only the directional-split Poisson row and print it")
    ap.add_argument("--cylinder-only", action="store_true",
                    help="run only the cylinder row (for profiling it alone) and print it")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (3 times), the reference "
                         "for scaling hardware byte counters")
    return ap.parse_args()


def kernel_bytes(name: str, b: int, ncell: int, dim: int) -> float:
    """Algorithmic HBM bytes of one launch: every grid array the kernel must
    read or write, once (b = bytes per grid value; p is always FP64)."""
    per_cell = {
        # u, nl, psi, p read; delta, nl written (f is read only in the few
        # tiles the spreading flagged, and not counted)
        "explicit": (4 * dim + 1) * b + 8,
        # momentum sweeps carry all dim components
        "mom_x_plain": 2 * b * dim, "mom_s_plain": 2 * b * dim,
        "mom_x_final": 3 * b * dim, "mom_s_final": 3 * b * dim,
        # D.u^{n+1}: reads u, writes div; psi: the first sweep reads div and
        # writes psi; the last reads psi, the div pair, p and writes psi, p, div
        "divergence": (dim + 1) * b,
        "psi_x_first": 2 * b, "psi_s_first": 2 * b,
        "psi_x_plain": 2 * b, "psi_s_plain": 2 * b,
        "psi_x_pfinal": 5 * b + 16, "psi_s_pfinal": 5 * b + 16,
        # mean of psi before the last sweep (FP32 work arrays): the sweep
        # before it leaves one partial sum per workgroup, so the gauge kernel
        # reads a few thousand doubles, not psi
        "psi_gauge": 0,
        # FP64-state policy: u += d in FP64
        "add_increment": (8 + b + 8) * dim,
    }.get(name)
    return None if per_cell is None else per_cell * ncell


def model_step_bytes(b: int, ncell: int, dim: int) -> float:
    """Algorithmic bytes of one step from the byte model of each of its kernels."""
    mom = (dim - 1) * 2 * b * dim + 3 * b * dim
    psi = (dim + 1) * b + 2 * b + (dim - 2) * 2 * b + 5 * b + 16
    return ((4 * dim + 1) * b + 8 + mom + psi) * ncell


def step_bytes(kern: dict, b: int, ncell: int, dim: int, steps: int) -> float:
    """Algorithmic bytes of one step as the timed steps ran it: the byte
    model of every grid kernel times its launches, over the steps."""
    tot = 0.0
    for name, (_, cnt) in kern.items():
        by = kernel_bytes(name, b, ncell, dim)
        if by is not None:
            tot += by * cnt
    return tot / steps


def run_gpu(w, precision, steps, warmup, tune=False, walls=False):
    import torch
    from paper_1305_3976_amd import ibgm
    cfg = ibgm.Config(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi,
                      precision=precision, walls_y=walls,
                      body_force=(1.0, 0.0, 0.0) if walls else (0.0, 0.0, 0.0))
    sim = ibgm.Simulation(cfg, w.u0, w.structure)
    stream = sim.stream
    picks = sim.tune(3) if tune else None
    sim.step(warmup)
    sim.sync()
    # timed region: K steps with per-kernel HIP events on the library's stream
    sim.profile(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    kern = sim.profile_read()
    sim.profile(False)
    # same K steps with no per-kernel events (the library launches only)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    sim.sync()
    ms_plain = e0.elapsed_time(e1)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return ms, ms_plain, wall, kern, picks


# The paper's directional-split solve alone (Table StrongScaling:PoissonProblem3d):
# wall time in seconds on one core and on its fastest partition.
PAPER_POISSON_3D = {128: {"P=1": 0.205, "P=128": 1.88e-3}, 256: {"P=1": 1.71, "P=256": 7.46e-3}}


def run_poisson(sizes=(256, 128), reps=20):
    """(1 - D_xx)(1 - D_yy)(1 - D_zz) psi = sin 2 pi x cos 2 pi y cos 2 pi z
    (Sec. "Comparison with Poisson Solvers") through ib_line_solve, one sweep
    per axis, FP64 and FP32 storage (FP64 recurrences), timed with HIP events;
    checked against the closed-form solution f / (1 + (4/h^2) sin^2(pi h))^3."""
    import torch
    from paper_1305_3976_amd import ibgm
    out = []
    for N in sizes:
        h = 1.0 / N
        c = (torch.arange(N, dtype=torch.float64, device="cuda") + 0.5) * h
        f = (torch.sin(2 * math.pi * c)[None, None, :] * torch.cos(2 * math.pi * c)[None, :, None]
             * torch.cos(2 * math.pi * c)[:, None, None])
        lam = 1 + (4 / h ** 2) * math.sin(math.pi * h) ** 2
        for dt_ in (torch.float64, torch.float32):
            t = f.to(dt_).contiguous()
            work = t.clone()
            for axis in (0, 1, 2):
                ibgm.line_solve(work, axis, 1 + 2 / h ** 2, -1 / h ** 2)
            err = ((work.double() - f / lam ** 3).abs().max() / (f / lam ** 3).abs().max()).item()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                for axis in (0, 1, 2):
                    ibgm.line_solve(work, axis, 1 + 2 / h ** 2, -1 / h ** 2)
            e1.record()
            torch.cuda.synchronize()
            sec = e0.elapsed_time(e1) * 1e-3 / reps
            paper = PAPER_POISSON_3D.get(N, {})
            row = {"n": N, "dtype": "f64" if dt_ == torch.float64 else "f32",
                   "s_per_solve": round(sec, 7), "gcell_per_s": round(N ** 3 / sec / 1e9, 2),
                   "max_rel_err_vs_closed_form": float("%.3g" % err),
                   "paper_s_per_solve": paper}
            for key, v in paper.items():
                row["ratio_vs_paper_" + key] = round(v / sec, 1)
            out.append(row)
            del t, work
        del f, c
        torch.cuda.empty_cache()
    return {"workload": "directional-split Poisson solve, 3 sweeps on N^3 cell centres",
            "note": "paper times are a CPU cluster (FP64 assumed): context, not a target",
            "runs": out}


# Wall time in seconds of the paper's first 100 steps of the cylinder on its
# CPU cluster (Table CylinderScaling): one core and its fastest partition.
PAPER_CYLINDER_100 = {128: {"P=1": 401.0, "P=128 (32,2,2)": 7.76},
                      256: {"P=1": 2600.0, "P=128 (32,2,2)": 30.2}}


def run_cylinder(sizes, steps=100, warmup=5, fp64=True):
    """The 3-D cylindrical shell of Sec. "Cylindrical Shell in 3D" (N_s = 19N/4
    by N_r = 3N points, axial rest length L = 1, dt = 0.04/N), timed over the
    paper's 100 steps; the paper's wall times are context (CPU cluster)."""
    from paper_1305_3976_amd import inputs
    out = []
    for n in sizes:
        w = inputs.config_cylinder(n, steps=steps)
        for prec, tag in ((1, "mixed"), (0, "fp64")):
            if prec == 0 and not fp64:
                continue
            ms, ms_plain, _, kern, _ = run_gpu(w, prec, steps, warmup)
            top = sorted(kern.items(), key=lambda kv: -kv[1][0])[:6]
            paper = PAPER_CYLINDER_100.get(n, {})
            row = {"n": n, "points": w.structure.np, "links": w.structure.nlinks,
                   "precision": tag, "steps": steps,
                   "ms_per_step": round(ms_plain / steps, 4),
                   "wall_s_100_steps": round(ms_plain * 1e-3 * 100 / steps, 4),
                   "gcell_updates_per_s": round(n ** 3 * steps / (ms_plain * 1e-3) / 1e9, 3),
                   "top_kernels_avg_us": {k: round(t / c * 1e3, 2) for k, (t, c) in top},
                   "paper_wall_s_100_steps": paper}
            for key, t in paper.items():
                row["ratio_vs_paper_" + key.split()[0]] = round(t / (ms_plain * 1e-3 * 100 / steps), 1)
            out.append(row)
            print("# cylinder N=%d %s: %.3f ms/step" % (n, tag, ms_plain / steps),
                  file=sys.stderr, flush=True)
    return {"workload": "cylinder3d: N^3, mu=0.01, dt=0.04/N, sigma_s=sigma_r=1, L=1, "
                        "r1=5/28, r2=7/20",
            "note": "paper times are FP64 (assumed) on a CPU cluster: context, not a target",
            "runs": out}


def run_channel(w, steps, warmup, fp64=True, plain_ms=None):
    """The same shell workload between no-slip walls at y = 0 and y = 1 (a
    channel driven by a body force along x): the y sweeps then solve the
    mirrored lines of twice the length."""
    out = {"workload": w.name + " between walls at y = 0, 1 (body force 1 along x)", "runs": []}
    for prec, tag in ((1, "mixed"), (0, "fp64")):
        if prec == 0 and not fp64:
            continue
        ms, ms_plain, _, kern, _ = run_gpu(w, prec, steps, warmup, walls=True)
        row = {"precision": tag, "ms_per_step": round(ms_plain / steps, 4),
               "kernels_avg_us": {k: round(t / c * 1e3, 2) for k, (t, c) in kern.items()}}
        if plain_ms and tag in plain_ms:
            row["vs_periodic"] = round(plain_ms[tag] / (ms_plain / steps), 3)
        out["runs"].append(row)
        print("# channel %s: %.3f ms/step" % (tag, ms_plain / steps), file=sys.stderr, flush=True)
    return out


def run_ensemble(steps, spl_choices=(2, 10), seed=4):
    """Batched ensemble: 64 independent 2-D problems (N drawn from
    {128,...,512}, 4N-point ellipses, stiffness log-uniform in [0.1, 100], time
    step per member), FP32 grid.  Step 0 runs eagerly (start-up rules); then
    every variant (steps per graph launch x one chain / one branch per size
    class, and one branch per context with the largest class split in two) is
    timed over the same number of steps after tuning, and the fastest is
    reported, beside eager launches of the same steps."""
    import torch
    from paper_1305_3976_amd import ensemble, ibgm, inputs
    members, shared = inputs.config_ensemble(nsims=64, seed=seed, steps=steps)
    per_size = {}
    for m in members:
        per_size[m.n] = per_size.get(m.n, 0) + 1
    split = (max(n * n * c for n, c in per_size.items()) + 1) // 2
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    timed = steps - 1 - (steps - 1) % (2 * max(spl_choices))
    variants = {}
    for split_cells in (0, split):
        ens = ensemble.Ensemble(members, rho=shared["rho"], mu=shared["mu"],
                                precision=ibgm.IB_PREC_MIXED, split_cells=split_cells)
        st = ens.stream
        t0 = time.perf_counter()
        pk = ens.tune(reps=10)
        if split_cells == 0:
            picks, tune_s = pk, time.perf_counter() - t0
        ens.step(1)
        ens.sync()
        if split_cells == 0:
            # eager launches of the same steps
            e0.record(st)
            ens.step(timed)
            e1.record(st)
            ens.sync()
            eager_ms = e0.elapsed_time(e1)
        for spl in spl_choices:
            for br in ((False, True) if split_cells == 0 else (True,)):
                ens.capture(spl, branches=br)
                ens.launch(1)                      # warm the instantiated graph
                ens.sync()
                e0.record(st)
                ens.launch(timed // spl)
                e1.record(st)
                ens.sync()
                key = "spl%d_%s%s" % (spl, "branches" if br else "chain",
                                      "_split" if split_cells else "")
                variants[key] = e0.elapsed_time(e1)
        ens.close()
        del ens
        torch.cuda.empty_cache()
    best = min(variants, key=variants.get)
    ms = variants[best]
    cells = sum(m.n ** 2 for m in members)
    sizes = {}
    for m in members:
        sizes[m.n] = sizes.get(m.n, 0) + 1
    return {
        "workload": "ensemble2d_64: 64 independent 2-D periodic problems, N from {128,192,256,384,512} "
                    "(seed %d), 4N-point 0.3x0.2 ellipses, stiffness log-uniform [0.1,100], "
                    "mu=0.01, per-member dt from the stiffness table, FP32 grid" % seed,
        "members": len(members), "members_per_size": sizes, "cells": cells,
        "split_cells": split,
        "timed_steps": timed,
        "member_steps_per_s": round(len(members) * timed / (ms * 1e-3), 1),
        "ensemble_steps_per_s": round(timed / (ms * 1e-3), 2),
        "gcell_updates_per_s": round(cells * timed / (ms * 1e-3) / 1e9, 3),
        "ms_per_ensemble_step": round(ms / timed, 4),
        "step_GB_s": round(model_step_bytes(4, cells, 2) / (ms / timed * 1e-3) / 1e9, 1),
        "best_variant": best,
        "variants_ms_per_step": {k: round(v / timed, 4) for k, v in variants.items()},
        "eager_ms_per_step": round(eager_ms / timed, 4),
        "tune_s": round(tune_s, 3),
        "tuned_tiles": [{"n": n, "picks": {"%d/%s" % (a, "f64" if r else "f32"): list(v)
                                           for (a, r), v in pk.items()}}
                        for (n, _), pk in zip(ens_classes_sizes(members), picks)],
    }


def ens_classes_sizes(members):
    return [(n, None) for n in sorted({m.n for m in members})]


def lagrangian_traffic(rows, npts, dim, b):
    """Per-point stencil traffic of the Lagrangian kernels, reported apart
    from the grid roofline (it is mostly served from L2, not HBM):
    interp + evolve reads the 4^dim stencil of every velocity component
    (dim 4^dim b) and X^n, U^{n-1} (2 dim 8), and writes U^n, X^{n+1},
    X^{n+1/2} (3 dim 8); spreading adds every point's 4^dim stencil values
    into f, counted as a read-modify-write (2 dim 4^dim b)."""
    st = 4 ** dim
    per = {"interp_evolve": dim * st * b + 5 * dim * 8, "spread": 2 * dim * st * b}
    out = {"points": npts, "note": "per-point stencil bytes, mostly L2-resident (not an HBM bound)"}
    for k, bpp in per.items():
        if k in rows:
            mb = npts * bpp / 1e6
            out[k] = {"bytes_per_point": bpp, "alg_MB_per_launch": round(mb, 2),
                      "avg_us": rows[k]["avg_us"],
                      "GB_s": round(mb * 1e6 / (rows[k]["avg_us"] * 1e-6) / 1e9, 1)}
    return out


def achievable_rates() -> dict:
    """The HBM rates a plain hand-written streaming kernel reaches on this GPU
    (the library's ib_probe_stream_rate, 256 MiB per stream, far beyond the
    256 MB last-level cache): 3 read + 3 write streams, and the explicit
    step's own mix (7 FP32 reads, p as two more FP32 reads, 6 FP32 writes =
    60 B per cell).  GB/s."""
    import torch
    from paper_1305_3976_amd import ibgm
    out = {"read3_write3": ibgm.stream_rate(3, 3, 256) / 1e9,
           "explicit_mix_read9_write6": ibgm.stream_rate(9, 6, 256) / 1e9}
    torch.cuda.empty_cache()
    return {k: round(v, 1) for k, v in out.items()}


def closure_vs_oracle(keep):
    """The closure row's error against the FP64 oracle: the oracle's own run of
    the held-out case on the fine grid (the rollout's restart step plus two
    fine steps per interval), restricted to the coarse grid, against the
    corrected and the plain coarse velocities after interval k of the
    rollout, and against the restricted GPU fine run that the rollout uses as
    its reference (mixed policy)."""
    import oracle
    from oracle import closure as oc
    case, nf, warm, snap = keep["case"], keep["n_fine"], keep["warmup"], keep["snap"]
    k = snap["interval"]
    P = oracle.make_params(3, (nf, nf, nf), 1.0 / nf, rho=1.0, mu=0.01, dt=case.dt_fine)
    S = case.structure
    t0 = time.time()
    sim = oracle.Sim(P, [np.asarray(c, dtype=np.float64) for c in case.u0], S.X, S.links, S.w)
    sim.advance(warm + 2 * k)
    el = time.time() - t0
    ref = [oc.restrict_face(sim.u[c], c) for c in range(3)]
    nr = math.sqrt(sum(float(np.sum(r ** 2)) for r in ref))
    rel = lambda us: math.sqrt(sum(float(np.sum((u - r) ** 2)) for u, r in zip(us, ref))) / nr
    return {"interval": k, "oracle_fine_steps": warm + 2 * k, "oracle_s": round(el, 1),
            "oracle_threads": oracle.num_threads(),
            "rel_l2_vs_restricted_oracle": {
                "coarse_plus_closure": round(rel(snap["corrected"]), 6),
                "plain_coarse": round(rel(snap["plain"]), 6),
                "gpu_fine_restricted": float("%.3g" % rel(snap["fine"]))},
            "note": "velocity after interval k against the FP64 oracle's fine run restricted "
                    "to the coarse grid (relative discrete l2 over the three components)"}


def oracle_sample(w, budget_s):
    import oracle
    P = oracle.make_params(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi)
    S = w.structure
    sim = oracle.Sim(P, [np.asarray(c, dtype=np.float64) for c in w.u0], S.X, S.links, S.w)
    t0 = time.perf_counter()
    n = 0
    while True:
        sim.advance(1)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 5 or el / n * (n + 1) > 2.5 * budget_s:
            break
    return sim, n, el, oracle.num_threads()


def config2_errors(steps: int):
    """The 512^2 ellipse workload (2048 points, sigma = 10, a seeded smooth
    flow, dt = 0.01/512) after `steps` steps: every GPU policy against the
    FP64 oracle, per field (relative discrete l2 and max |gpu - oracle| /
    max |oracle|).  The oracle run is started in a thread (it is C with
    OpenMP and releases the interpreter) so it overlaps the GPU rows."""
    import threading
    import oracle
    from paper_1305_3976_amd import inputs
    w = inputs.config_ellipse_512(steps=steps)
    P = oracle.make_params(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi)
    S = w.structure
    sim = oracle.Sim(P, [np.asarray(c, dtype=np.float64) for c in w.u0], S.X, S.links, S.w)
    box = {}

    def run():
        t0 = time.perf_counter()
        sim.advance(steps)
        box["s"] = time.perf_counter() - t0

    th = threading.Thread(target=run, daemon=True)
    th.start()
    return w, sim, th, box


def config2_finish(w, sim, th, box, steps):
    from paper_1305_3976_amd import ibgm
    th.join()
    out = {"workload": "ellipse2d_512: 512^2, mu=0.01, dt=0.01/512, 2048-point ellipse "
                       "sigma=10, seeded smooth flow", "steps": steps,
           "oracle_s": round(box.get("s", float("nan")), 1), "errors": {}}
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
    mx = lambda a, b: float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))
    for prec, tag in ((0, "fp64"), (1, "mixed"), (2, "mixed_state64")):
        cfg = ibgm.Config(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi,
                          precision=prec)
        g = ibgm.Simulation(cfg, w.u0, w.structure)
        g.step(steps)
        g.sync()
        st = g.state()
        g.close()
        e = {}
        for c in range(w.dim):
            e["u%d" % c] = [rel(st["u"][c], sim.u[c]), mx(st["u"][c], sim.u[c])]
        e["p"] = [rel(st["p"], sim.p), mx(st["p"], sim.p)]
        e["X"] = [rel(st["X"], sim.X), mx(st["X"], sim.X)]
        out["errors"][tag] = e
    out["errors_note"] = "[relative l2, max abs / max |oracle|] per field"
    return out


def gpu_errors(w, precision, nsteps, ref):
    from paper_1305_3976_amd import ibgm
    cfg = ibgm.Config(w.dim, w.n, w.h, rho=w.rho, mu=w.mu, dt=w.dt, chi=w.chi,
                      precision=precision)
    sim = ibgm.Simulation(cfg, w.u0, w.structure)
    sim.step(nsteps)
    sim.sync()
    st = sim.state()
    sim.close()
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
    out = {"u%d" % c: rel(st["u"][c], ref.u[c]) for c in range(w.dim)}
    out["p"] = rel(st["p"], ref.p)
    out["X"] = rel(st["X"], ref.X)
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs an MI355X (no GPU visible)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        src = torch.empty(args.copy_calibration * 2 ** 20 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.poisson_only:
        print(json.dumps({"poisson": run_poisson()}), flush=True)
        return
    if args.cylinder_only:
        print(json.dumps({"cylinder": run_cylinder(args.cylinder or [256],
                                                   steps=args.steps, warmup=args.warmup,
                                                   fp64=not args.no_fp64)}), flush=True)
        return
    achievable = achievable_rates()
    ach_gbs = achievable["read3_write3"]
    # the long 512^2 comparison: its oracle run starts now, beside the GPU rows
    c2 = None
    if not args.no_cpu_baseline and args.config2_steps > 0:
        c2 = config2_errors(args.config2_steps)
    from paper_1305_3976_amd import inputs
    w = inputs.config_shell_256(steps=args.steps, n=args.n, npts=args.points)
    ncell = w.n[0] * w.n[1] * w.n[2]
    print("# workload %s: %d cells, %d points, %d links" % (
        w.name, ncell, w.structure.np, w.structure.nlinks), file=sys.stderr, flush=True)

    res = {}
    for prec, tag in ((1, "mixed"), (0, "fp64")):
        if prec == 0 and args.no_fp64:
            continue
        ms, ms_plain, wall, kern, picks = run_gpu(w, prec, args.steps, args.warmup,
                                                  args.tune)
        res[tag] = (ms, ms_plain, wall, kern, picks)
        print("# %s: %.3f ms/step (profiled), %.3f ms/step (plain)" % (
            tag, ms / args.steps, ms_plain / args.steps), file=sys.stderr, flush=True)

    ms, ms_plain, wall, kern, picks = res["mixed"]
    b = 4
    rows = {}
    for name, (tot, cnt) in kern.items():
        by = kernel_bytes(name, b, ncell, w.dim)
        avg_ms = tot / cnt
        rows[name] = {"avg_us": round(avg_ms * 1e3, 2), "launches": cnt,
                      "share": round(tot / sum(t for t, _ in kern.values()), 4)}
        if by is not None:
            rows[name]["alg_GB_per_launch"] = round(by / 1e9, 4)
            rows[name]["GB_s"] = round(by / (avg_ms * 1e-3) / 1e9, 1)
    # dominant kernel = largest total time among the grid kernels with a byte model
    dom = max((n for n in rows if "GB_s" in rows[n]), key=lambda n: kern[n][0])
    ach = rows[dom]["GB_s"]
    steps_s = args.steps / (ms_plain * 1e-3)
    line = {
        "metric": "IB steps/s and Gcell-updates/s at 256^3, FP32 vs FP64, % of HBM roofline",
        "value": round(steps_s, 3),
        "unit": "IB steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_plain / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 grid / f64 positions+pressure",
        "data": "synthetic",
        "config": {"workload": "shell3d_256: 256^3 periodic MAC grid, mu=0.01, dt=5e-4, "
                               "ellipsoidal shell 0.3/0.25/0.2 with %d points, membrane modulus 1 (cotangent links)"
                               % w.structure.np,
                   "cells": ncell, "points": w.structure.np, "links": w.structure.nlinks},
        "gcell_updates_per_s": round(ncell * steps_s / 1e9, 3),
        "ms_per_step_profiled": round(ms / args.steps, 4),
        "wall_s_timed_region": round(wall, 3),
        "step_alg_bytes_GB": round(step_bytes(kern, b, ncell, w.dim, args.steps) / 1e9, 4),
        "step_GB_s": round(step_bytes(kern, b, ncell, w.dim, args.steps)
                           / (ms_plain / args.steps * 1e-3) / 1e9, 1),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": (round(TRAFFIC_BYTES[dom] / 1e9, 4)
                                 if dom in TRAFFIC_BYTES and args.n == 256 else None),
                     "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE)",
                     "achievable_GB_s": achievable,
                     "achievable_note": "a plain hand-written streaming kernel on this GPU "
                                        "(ib_probe_stream_rate), 256 MiB per stream",
                     "frac_of_achievable": round(ach / ach_gbs, 4),
                     "frac_of_same_mix": round(ach / achievable["explicit_mix_read9_write6"], 4)
                     if dom == "explicit" else None,
                     "sweeps": {n: {"GB_s": rows[n]["GB_s"],
                                    "frac": round(rows[n]["GB_s"] / HBM_PEAK_GBS, 4),
                                    "frac_of_achievable": round(rows[n]["GB_s"] / ach_gbs, 4)}
                                for n in rows if (n.startswith("mom_") or n.startswith("psi_"))
                                and "GB_s" in rows[n]},
                     "sweeps_note": "HIP-event time of each line-sweep kernel inside the step "
                                    "(the psi sweeps share the GPU with the overlapped "
                                    "Lagrangian work), algorithmic bytes"},
        "kernels": rows,
        "lagrangian": lagrangian_traffic(rows, w.structure.np, w.dim, b),
        "tuned_tiles": None if picks is None else {
            "%d/%s" % (a, "f64" if r else "f32"): list(v) for (a, r), v in picks.items()},
    }
    if "fp64" in res:
        ms64, ms64_plain, _, kern64, _ = res["fp64"]
        s64 = args.steps / (ms64_plain * 1e-3)
        line["fp64"] = {"value": round(s64, 3), "unit": "IB steps/s",
                        "ms_per_step": round(ms64_plain / args.steps, 4),
                        "gcell_updates_per_s": round(ncell * s64 / 1e9, 3),
                        "step_GB_s": round(step_bytes(kern64, 8, ncell, w.dim, args.steps)
                                           / (ms64_plain / args.steps * 1e-3) / 1e9, 1),
                        "kernels_avg_us": {k: round(t / c * 1e3, 2) for k, (t, c) in kern64.items()}}
        line["mixed_vs_fp64_speedup"] = round(steps_s / s64, 3)
    if not args.no_poisson:
        line["poisson"] = run_poisson()
    if not args.no_channel:
        plain = {"mixed": ms_plain / args.steps}
        if "fp64" in res:
            plain["fp64"] = res["fp64"][1] / args.steps
        line["channel"] = run_channel(w, args.steps, args.warmup, fp64=not args.no_fp64,
                                      plain_ms=plain)
    if args.cylinder:
        line["cylinder"] = run_cylinder(args.cylinder, fp64=not args.no_fp64)
    if args.ensemble_steps:
        line["ensemble"] = run_ensemble(args.ensemble_steps)
        print("# ensemble: %.1f member-steps/s, %.3f Gcell/s (%s)" % (
            line["ensemble"]["member_steps_per_s"], line["ensemble"]["gcell_updates_per_s"],
            line["ensemble"]["best_variant"]), file=sys.stderr, flush=True)
    if c2 is not None:  # (joined before the closure, whose host work it would slow)
        line["config2_%d_steps" % args.config2_steps] = config2_finish(*c2, args.config2_steps)
        print("# config 2: %d steps compared with the oracle (oracle %.1f s)" % (
            args.config2_steps, line["config2_%d_steps" % args.config2_steps]["oracle_s"]),
            file=sys.stderr, flush=True)
    if args.closure != "off":
        from paper_1305_3976_amd import closure_run
        cargs = [] if args.closure == "full" else [
            "--n-fine", "64", "--traj", "20", "--held", "4", "--snapshots", "12",
            "--iters", "1200", "--crop", "26", "--rollout", "10"]
        keep = {"interval": args.closure_oracle_interval} if args.closure_oracle_interval else None
        line["closure"] = closure_run.main(cargs, keep=keep)
        torch.cuda.empty_cache()
        if keep is not None and keep.get("snap", {}).get("fine") is not None:
            line["closure"]["error_vs_fp64_oracle"] = chk = closure_vs_oracle(keep)
            print("# closure vs FP64 oracle after interval %d (oracle %.1f s): corrected %.3e, "
                  "plain %.3e, GPU fine %.2e" % (
                      chk["interval"], chk["oracle_s"],
                      chk["rel_l2_vs_restricted_oracle"]["coarse_plus_closure"],
                      chk["rel_l2_vs_restricted_oracle"]["plain_coarse"],
                      chk["rel_l2_vs_restricted_oracle"]["gpu_fine_restricted"]),
                  file=sys.stderr, flush=True)
            del keep
    if not args.no_cpu_baseline:
        ref, n, el, thr = oracle_sample(w, args.cpu_seconds)
        line["cpu_baseline"] = {"value": round(n / el, 5), "unit": "IB steps/s", "cores": thr,
                                "kind": "oracle",
                                "sample": "%d step(s) of the same 256^3 workload from rest, FP64 "
                                          "oracle, OpenMP over independent lines/cells" % n}
        errs = {"mixed": gpu_errors(w, 1, n, ref)}
        if not args.no_fp64:
            errs["fp64"] = gpu_errors(w, 0, n, ref)
        line["error_vs_fp64_oracle"] = {"steps": n, "rel_l2": errs}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
