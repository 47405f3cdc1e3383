"""Train and evaluate the learned closure on method-generated pairs.

    python -m paper_1305_3976_amd.closure_run [--n-fine 256] [--traj 11] ...

Fine runs (n_fine^3, time step dt) of a seeded family of ellipsoidal shells
with random smooth flow; each snapshot restarts a coarse run (n_fine/2, 2 dt)
from the restricted fine state, takes one coarse step and pairs its fields
with the restricted fine velocity two fine steps later.  The network trains on
crops (valid convolutions with a 3-voxel margin) from the training
trajectories; the held-out trajectories (about 10% of the seeds) evaluate it,
once per interval and in a rollout where the correction is applied after
every coarse step.  Prints one JSON line with the errors against the
restricted fine solve and the per-step times of the fine solve, the plain
coarse solve and the corrected coarse solve, plus the matrix-core rate of
the network's forward pass on the whole coarse grid.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import closure as cl
from . import inputs

MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix-core peak, published


def conv_rates(net: cl.ConvNet, nc: int, reps: int = 10):
    """Forward pass of the network on a periodic nc^3 grid: time per layer
    (HIP events on the current stream) and the achieved matrix-core rate of
    each, counting the FLOPs of the real channel counts."""
    x = torch.zeros(nc ** 3 * 16, dtype=torch.bfloat16, device=net.device)
    net.forward(x, 1, (nc, nc, nc), cl.PERIODIC)
    B = net._buffers(1, (nc, nc, nc), cl.PERIODIC)
    st = cl._stream()
    d = (nc, nc, nc)
    calls = [
        (lambda: cl.lib.ib_conv3d_fwd(cl._p(x), 1, cl._i3(d), 16, cl._p(net.P[0]), cl._p(net.b[0]),
                                      cl.PERIODIC, cl.RELU, cl._p(B["a1"]), 32, 32, st), cl.CIN, cl.HID),
        (lambda: cl.lib.ib_conv3d_fwd(cl._p(B["a1"]), 1, cl._i3(d), 32, cl._p(net.P[1]),
                                      cl._p(net.b[1]), cl.PERIODIC, cl.RELU, cl._p(B["a2"]), 32, 32,
                                      st), cl.HID, cl.HID),
        (lambda: cl.lib.ib_conv3d_fwd(cl._p(B["a2"]), 1, cl._i3(d), 32, cl._p(net.P[2]),
                                      cl._p(net.b[2]), cl.PERIODIC, cl.OUT_F32 | cl.NARROW,
                                      cl._p(B["y"]), 3, 3, st), cl.HID, cl.COUT),
    ]
    out = []
    for fn, ci, co in calls:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        e0.record()
        for _ in range(reps):
            cl.check(fn())
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        flops = 2.0 * 27 * ci * co * nc ** 3
        out.append({"ci": ci, "co": co, "us": round(ms * 1e3, 2),
                    "tflops": round(flops / (ms * 1e-3) / 1e12, 2)})
    return out


def main(argv=None, keep: dict = None):
    """The closure experiment; returns the bench line's closure row.  With
    `keep` = {"interval": k}, also leaves in it what a check of the row against
    an independent fine solve needs: the held-out case ("case"), the fine grid
    ("n_fine"), the restart step ("warmup") and the velocities after interval
    k of the main rollout ("snap": see closure.rollout)."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-fine", type=int, default=256)
    ap.add_argument("--traj", type=int, default=11, help="trajectories (the last ~10%% held out)")
    ap.add_argument("--held", type=int, default=1)
    ap.add_argument("--snapshots", type=int, default=200, help="pairs per trajectory")
    ap.add_argument("--every", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=6)
    ap.add_argument("--crop", type=int, default=32)
    ap.add_argument("--crops", type=int, default=1, help="crops per pair")
    ap.add_argument("--iters", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--rollout", type=int, default=20, help="coarse steps of the rollout")
    ap.add_argument("--dagger-syncs", type=int, default=10,
                    help="restarts per training trajectory for pairs along corrected runs")
    ap.add_argument("--dagger-horizon", type=int, default=10,
                    help="corrected coarse intervals after each restart")
    ap.add_argument("--dagger-iters", type=int, default=2000)
    ap.add_argument("--check-every", type=int, default=4,
                    help="coarse intervals between the fine solve's audits (guarded rollout)")
    ap.add_argument("--late-start", type=int, default=400,
                    help="fine steps before the second rollout (mid-trajectory start)")
    ap.add_argument("--seed", type=int, default=5)
    a = ap.parse_args(argv)
    t0 = time.time()
    log = lambda *s: print("#", *s, file=sys.stderr, flush=True)
    cases = inputs.closure_family(a.traj, seed=a.seed, n_fine=a.n_fine)
    ntr = a.traj - a.held
    nc = a.n_fine // 2
    log("family of %d shells built in %.1f s" % (a.traj, time.time() - t0))
    tr = cl.PairSet(ntr * a.snapshots * a.crops, nc, mode=cl.VALID, crop=a.crop)
    ho = cl.PairSet(a.held * a.snapshots * a.crops, nc, mode=cl.VALID, crop=a.crop)
    t1 = time.time()
    scales = cl.collect(cases[:ntr], a.n_fine, a.snapshots, a.every, a.warmup, tr, crops=a.crops)
    cl.collect(cases[ntr:], a.n_fine, a.snapshots, a.every, a.warmup, ho, scales=scales,
               crops=a.crops, seed=1)
    torch.cuda.synchronize()
    gen_s = time.time() - t1
    log("%d training and %d held-out pairs in %.1f s" % (tr.count, ho.count, gen_s))
    net = cl.ConvNet(seed=7)
    t2 = time.time()
    losses = cl.train(net, tr, a.iters, a.batch, a.lr)
    train_s = time.time() - t2
    e0, e1 = cl.evaluate(net, ho, 0, ho.count, batch=a.batch)
    r0, r1 = cl.evaluate(net, tr, 0, min(tr.count, 256), batch=a.batch)
    log("held-out one-interval error ratio %.3f (train %.3f), %.1f s training" % (e1 / e0, r1 / r0, train_s))
    errs1, _, _ = cl.rollout(cases[-1], a.n_fine, a.rollout, net, scales, a.warmup)
    log("rollout (one-interval training): plain %.3e -> %.3e, corrected %.3e -> %.3e" % (
        errs1[0][0], errs1[-1][0], errs1[0][1], errs1[-1][1]))
    # second phase: pairs along the network's own corrected runs (the states
    # it meets in service), trained together with the first-phase pairs
    dag = None
    if a.dagger_syncs and a.dagger_horizon:
        t3 = time.time()
        tr2 = cl.PairSet(ntr * a.dagger_syncs * a.dagger_horizon * a.crops, nc, mode=cl.VALID,
                         crop=a.crop)
        span = a.snapshots * a.every
        gap = max(0, (span - a.dagger_syncs * 2 * a.dagger_horizon) // a.dagger_syncs)
        cl.collect_rollouts(cases[:ntr], a.n_fine, net, scales, tr2, a.dagger_syncs,
                            a.dagger_horizon, gap, a.warmup, crops=a.crops)
        torch.cuda.synchronize()
        gen2 = time.time() - t3
        t4 = time.time()
        losses2 = cl.train(net, [tr, tr2], a.dagger_iters, a.batch, 0.5 * a.lr)
        train2 = time.time() - t4
        e0, e1 = cl.evaluate(net, ho, 0, ho.count, batch=a.batch)
        log("corrected-run pairs: %d in %.1f s, %.1f s training; held-out ratio now %.3f" % (
            tr2.count, gen2, train2, e1 / e0))
        dag = {"pairs": tr2.count, "generation_s": round(gen2, 1), "train_s": round(train2, 1),
               "iters": a.dagger_iters,
               "loss_first_last": [float(losses2[:50].mean()), float(losses2[-50:].mean())]}
        del tr2
    snap = {"interval": keep.get("interval", 4)} if keep is not None else None
    errs, t_plain, t_corr = cl.rollout(cases[-1], a.n_fine, a.rollout, net, scales, a.warmup,
                                       snap=snap)
    if keep is not None:
        keep.update(case=cases[-1], n_fine=a.n_fine, warmup=a.warmup, snap=snap)
    log("rollout: plain %.3e -> %.3e, corrected %.3e -> %.3e" % (errs[0][0], errs[-1][0], errs[0][1], errs[-1][1]))
    errs_late, _, _ = cl.rollout(cases[-1], a.n_fine, a.rollout, net, scales, a.late_start)
    gerrs, fired = cl.guarded_rollout(cases[-1], a.n_fine, a.rollout, net, scales,
                                      check_every=a.check_every, warmup=a.warmup)
    log("guarded rollout: %d fallback(s); final plain %.3e corrected %.3e guarded %.3e" % (
        len(fired), gerrs[-1][0], gerrs[-1][1], gerrs[-1][2]))
    # fine step time on the same family member (two fine steps per coarse step)
    cf = cl.CoarseFine(cases[-1], a.n_fine)
    cf.fine_steps(3)
    torch.cuda.synchronize()
    e0v, e1v = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0v.record()
    cf.fine_steps(20)
    e1v.record()
    torch.cuda.synchronize()
    t_fine = e0v.elapsed_time(e1v) / 20
    cf.close()
    # coarse intervals timed the same way: back to back, no host round trip
    t_plain, t_corr = cl.interval_times(cases[-1], a.n_fine, net, scales, 20, a.warmup)
    rates = conv_rates(net, nc)
    line = {
        "workload": "closure: %d^3 coarse (2 dt) vs %d^3 fine, %d trajectories (%d held out), "
                    "%d pairs of %d^3 crops" % (nc, a.n_fine, a.traj, a.held, tr.count, a.crop),
        "pairs_train": tr.count, "pairs_held_out": ho.count,
        "generation_s": round(gen_s, 1), "train_s": round(train_s, 1), "iters": a.iters,
        "loss_first_last": [float(losses[:50].mean()), float(losses[-50:].mean())],
        "held_out_interval_error_ratio": round(e1 / e0, 4),
        "train_interval_error_ratio": round(r1 / r0, 4),
        "rollout_rel_l2_vs_restricted_fine": {
            "steps": a.rollout, "start_fine_step": a.warmup,
            "plain_coarse": [round(e[0], 6) for e in errs],
            "coarse_plus_closure": [round(e[1], 6) for e in errs],
            "coarse_plus_closure_one_interval_training_only": [round(e[1], 6) for e in errs1],
            "intervals_corrected_below_plain": int(sum(e[1] < e[0] for e in errs))},
        "rollout_mid_trajectory": {
            "start_fine_step": a.late_start,
            "plain_coarse": [round(e[0], 6) for e in errs_late],
            "coarse_plus_closure": [round(e[1], 6) for e in errs_late],
            "intervals_corrected_below_plain": int(sum(e[1] < e[0] for e in errs_late))},
        "guarded_rollout": {
            "check_every": a.check_every,
            "note": "the fine solve audits the corrected run every check_every intervals and "
                    "restarts it from the restricted fine state where it has fallen behind "
                    "the plain coarse run",
            "fallback_after_interval": [k + 1 for k in fired],
            "guarded": [round(e[2], 6) for e in gerrs],
            "plain_coarse": [round(e[0], 6) for e in gerrs],
            "coarse_plus_closure_unguarded": [round(e[1], 6) for e in gerrs]},
        "corrected_run_training": dag,
        "ms_per_interval": {"fine_two_steps": round(2 * t_fine, 4),
                            "coarse_plain": round(t_plain, 4),
                            "coarse_plus_closure": round(t_corr, 4)},
        "ms_per_interval_note": "GPU time per interval over 20 intervals (fine: 20 steps) "
                                "enqueued back to back, HIP events",
        "speedup_coarse_plus_closure_vs_fine": round(2 * t_fine / t_corr, 3),
        "speedup_plain_coarse_vs_fine": round(2 * t_fine / t_plain, 3),
        "forward_layers_at_coarse_grid": rates,
        "scales": scales.__dict__,
    }
    l2 = rates[1]
    line["roofline"] = {"bound": "mfma", "kernel": "conv3d 32->32 channels, %d^3 periodic" % nc,
                        "achieved": l2["tflops"], "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(l2["tflops"] / MFMA_BF16_PEAK_TFLOPS, 4), "traffic": None}
    del tr, ho, net, cases
    return line


if __name__ == "__main__":
    print(json.dumps(main()), flush=True)
