"""Train the learned curvature closure on the GPU and measure what it gains.

    python -m paper_1603_02421_amd.train_closure --out DIR [--shapes N] [--epochs E] ...

1. Training data: rotated discs and sinusoidal interfaces with exact labels,
   and jets run at 4x resolution, subsampled to the target spacing and
   labelled by the fine runs' plain curvature (see closure.py), each stencil
   also mirrored about its frame's e1 axis.
2. Training: Adam on the mean squared error with the library's own forward,
   backward and Adam kernels (sph_mlp_train_step).
3. Evaluation on held-out shapes and held-out jets (other seeds, Re, We): the
   relative L2 curvature error against the reference of the plain estimate
   (eq. 23) at the target resolution, of the network alone, and of the
   closure with its fallback, the last taken from the particle update itself
   (sph_evaluate with the closure installed).
4. Cost: particle-steps/s of the plain and closure updates on the same jet,
   and the 4x-resolution run that the reference labels come from.

Writes DIR/closure_weights.npz and DIR/closure_report.json.
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np


def log(*a):
    print(*a, flush=True)


# (nD coarse, Re, We, seed, piston amplitude). The jet of the closure workload:
# D = 20 dx, Re 500, We 20, kD 0.7, labelled by runs at 4x resolution; seeds
# 100-103 are held out.
TRAIN_JETS = [(20, 500.0, 20.0, seed, 0.01) for seed in range(8)]
HELD_OUT_JETS = [(20, 500.0, 20.0, seed, 0.01) for seed in (100, 101, 102, 103)]
# smaller, more varied jets (D = 10-16 dx, other Re/We, stronger inflow perturbation)
SWEEP_JETS = [
    (10, 500.0, 20.0, 11, 0.01), (10, 200.0, 10.0, 12, 0.2), (12, 1000.0, 30.0, 13, 0.01),
    (12, 300.0, 8.0, 14, 0.2), (16, 800.0, 15.0, 15, 0.1), (10, 1500.0, 40.0, 16, 0.2),
    (14, 400.0, 25.0, 17, 0.1), (16, 2000.0, 50.0, 18, 0.01),
]
SWEEP_HELD_OUT = [(10, 700.0, 12.0, 101, 0.1), (12, 250.0, 35.0, 102, 0.2), (16, 1200.0, 20.0, 103, 0.01)]


def fine_runs(spec, snap_steps, n_coarse, free_length, avg_steps):
    """(spec entry, snapshots) of the jets of `spec` run at 4x resolution (the
    fine run has 16 n_coarse particles, so that its tank matches a coarse jet
    of n_coarse); jets whose run fails are skipped."""
    from . import closure as cl
    from .native import SphError
    runs = []
    for (nD, Re, We, seed, amp) in spec:
        t0 = time.time()
        try:
            snaps = cl.fine_jet_snapshots(nD, Re, We, seed, snap_steps, n_fine=16 * n_coarse,
                                          free_length=free_length, piston_amp=amp, avg_steps=avg_steps)
        except SphError as e:
            log(f"[jets] nD={nD} Re={Re} We={We} amp={amp}: skipped ({e})")
            continue
        runs.append(((nD, Re, We, seed, amp), snaps))
        log(f"[jets] nD={nD} Re={Re} We={We} amp={amp}: {len(snaps)} snapshots, {time.time() - t0:.1f} s")
    return runs


def jet_sets(spec, snap_steps, n_coarse, free_length, avg_steps=1, window=1.0):
    """Coarse labelled sets from jets run at 4x resolution (labels: see
    closure.coarse_from_snapshot and fine_jet_snapshots)."""
    from . import closure as cl
    out = []
    for (nD, Re, We, seed, amp), snaps in fine_runs(spec, snap_steps, n_coarse, free_length, avg_steps):
        t0 = time.time()
        for k, sn in enumerate(snaps):
            out.append(cl.coarse_from_snapshot(sn, nD, Re, We, seed * 100 + k, window=window))
        log(f"[jets] nD={nD} Re={Re} We={We} amp={amp}: {len(snaps)} snapshots, "
            f"{sum(s.n for s in out[-len(snaps):])} coarse particles, {time.time() - t0:.1f} s")
    return out


def errors(k_ref, k_plain, k_mlp, k_closure):
    from .closure import rel_l2
    curved = np.abs(k_ref) > 0.05
    r = dict(n=int(len(k_ref)), plain=rel_l2(k_plain, k_ref), mlp=rel_l2(k_mlp, k_ref),
             closure=rel_l2(k_closure, k_ref), n_curved=int(curved.sum()))
    if curved.any():
        r.update(plain_curved=rel_l2(k_plain[curved], k_ref[curved]), mlp_curved=rel_l2(k_mlp[curved], k_ref[curved]),
                 closure_curved=rel_l2(k_closure[curved], k_ref[curved]))
    return r


def throughput(system, params, steps, closure: bool):
    import workloads as wl
    from .sim import Simulation
    s = wl.round_for_dtype(system, 32)
    s.params = dict(s.params, closure=1 if closure else 0)
    with Simulation(s, dtype_bits=32, graph_steps=50) as sim:
        if closure:
            sim.set_closure(params)
        sim.step(100)
        sim.sync()
        tau0 = float(sim.read("time")[0])
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        dt = time.perf_counter() - t0
        tau = float(sim.read("time")[0]) - tau0
        n = int(sim.read("nactive")[0])
    return dict(n=n, steps=steps, seconds=dt, particle_steps_per_s=n * steps / dt, sim_time=tau,
                seconds_per_unit_time=dt / tau)


def _snaps(text):
    return [int(x) for x in text.split(",")]


def main(argv=None):
    from . import closure as cl
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--shapes", type=int, default=4000)
    ap.add_argument("--held-out-shapes", type=int, default=400)
    ap.add_argument("--jets", type=int, default=len(TRAIN_JETS), help="training jets of the D = 20 dx workload")
    ap.add_argument("--jet-n", type=int, default=300_000, help="particles of a coarse D = 20 dx jet")
    ap.add_argument("--jet-free-length", type=float, default=60.0)
    ap.add_argument("--jet-snap-steps", type=str, default="4000,8000,12000,16000,20000,24000,28000,32000",
                    help="steps of the 4x-resolution run after which it is sampled")
    ap.add_argument("--sweep-jets", type=int, default=len(SWEEP_JETS), help="smaller, varied jets to add")
    ap.add_argument("--sweep-n", type=int, default=25_000)
    ap.add_argument("--sweep-free-length", type=float, default=40.0)
    ap.add_argument("--sweep-snap-steps", type=str, default="6000,12000,18000,24000,30000")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--bench-steps", type=int, default=2000)
    ap.add_argument("--cost-n", type=int, default=300_000)
    ap.add_argument("--no-mirror", action="store_true", help="no mirror images of the training stencils")
    ap.add_argument("--skip-eval", action="store_true", help="stop after training")
    ap.add_argument("--eval-only", action="store_true", help="skip data and training; evaluate the weights")
    ap.add_argument("--label-steps", type=int, default=1,
                    help="fine steps each jet label's curvature is averaged over (4: one coarse step; "
                         "measured to leave the labels' noise unchanged)")
    ap.add_argument("--label-window", type=float, default=2.0,
                    help="radius of a jet label's average, in coarse smoothing lengths (2: the kernel's support)")
    ap.add_argument("--label-study", action="store_true",
                    help="only measure the held-out jet labels' split-half noise and the plain estimate's "
                         "error (at the coarse and at twice the coarse resolution) for label variants")
    ap.add_argument("--weights", default="", help="weights file for --eval-only (default: the shipped ones)")
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    rep = dict(args=vars(a))

    if a.label_study:
        label_study(cl, a, rep)
        return
    if a.eval_only:
        w = cl.load(a.weights) if a.weights else cl.load()
        evaluate_and_cost(cl, w, a, rep)
        return
    t0 = time.time()
    shapes = cl.shape_systems(a.shapes, seed=a.seed)
    Xs, Ts, Ps, _ = cl.harvest_shapes(shapes)
    del shapes
    log(f"[data] shapes: {len(Xs)} neighbourhoods ({time.time() - t0:.1f} s)")
    jets = jet_sets(TRAIN_JETS[:a.jets], _snaps(a.jet_snap_steps), a.jet_n, a.jet_free_length,
                    a.label_steps, a.label_window)
    jets += jet_sets(SWEEP_JETS[:a.sweep_jets], _snaps(a.sweep_snap_steps), a.sweep_n, a.sweep_free_length,
                     a.label_steps, a.label_window)
    Xj, Tj, Pj, _, _ = cl.harvest_coarse(jets)
    del jets
    log(f"[data] jets: {len(Xj)} neighbourhoods ({time.time() - t0:.1f} s)")
    X = np.concatenate([Xs, Xj])
    T = np.concatenate([Ts, Tj])
    if not a.no_mirror:
        Xm, Tm = cl.mirror(X, T)
        X, T = np.concatenate([X, Xm]), np.concatenate([T, Tm])
    rep["data"] = dict(shapes=int(len(Xs)), jets=int(len(Xj)), mirrored=not a.no_mirror, samples=int(len(X)),
                       seconds=time.time() - t0)

    t1 = time.time()
    w, hist = cl.train(X, T, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
    rep["train"] = dict(seconds=time.time() - t1, loss=hist, samples=int(len(X)))
    cl.save(w, os.path.join(a.out, "closure_weights.npz"))
    del X, T
    log(f"[train] done in {time.time() - t1:.1f} s, final loss {hist[-1]:.4e}")
    if a.skip_eval:
        with open(os.path.join(a.out, "closure_report.json"), "w") as f:
            json.dump(rep, f, indent=1)
        log("[done]")
        return
    evaluate_and_cost(cl, w, a, rep)


def label_study(cl, a, rep):
    """Split-half noise of the held-out jets' labels, and the plain estimate's
    error against them at the coarse and at twice the coarse resolution, for
    labels from one fine step or averaged over `label_steps`, over one or two
    coarse smoothing lengths. The twice-as-fine subsample is labelled at the
    coarse scale, so both resolutions are measured against the same labels."""
    out = {}
    for name, spec, snaps, n, fl in (("jets_D20", HELD_OUT_JETS, a.jet_snap_steps, a.jet_n, a.jet_free_length),
                                     ("sweep_jets", SWEEP_HELD_OUT, a.sweep_snap_steps, a.sweep_n,
                                      a.sweep_free_length)):
        runs = fine_runs(spec, _snaps(snaps), n, fl, max(a.label_steps, 4))
        # the Poisson radius that keeps one point per dx^2 at twice the coarse
        # resolution (four fine points per cell), from the first snapshot
        (nD0, *_), sn0 = runs[0][0], runs[0][1][-1]
        target = len(sn0["pos"]) / 4.0
        rmin2 = min((0.60, 0.64, 0.68, 0.72, 0.76),
                    key=lambda f: abs(len(cl.poisson_subsample(sn0["pos"], f / (2 * nD0), 1)) - target))
        log(f"[labels] {name}: Poisson radius {rmin2} dx at twice the coarse resolution")
        keeps = {(i, k, fine): cl.poisson_subsample(sn["pos"], (0.78 if fine == 1 else rmin2) / (fine * nD),
                                                    seed * 100 + k)
                 for i, ((nD, Re, We, seed, amp), sn_list) in enumerate(runs)
                 for k, sn in enumerate(sn_list) for fine in (1, 2)}
        for steps in (1, max(a.label_steps, 4)):
            for window in (1.0, 2.0):
                for fine in (1, 2):
                    systems, kept, expect = [], 0, 0.0
                    for i, ((nD, Re, We, seed, amp), sn_list) in enumerate(runs):
                        for k, sn in enumerate(sn_list):
                            snap = sn if steps > 1 else dict(sn, kappa=sn["kappa_first"])
                            systems.append(cl.coarse_from_snapshot(snap, fine * nD, Re, We, seed * 100 + k,
                                                                   window=window, label_h=1.3 / nD,
                                                                   keep=keeps[(i, k, fine)]))
                            kept += systems[-1].n
                            expect += len(sn["pos"]) * (fine / 4.0) ** 2
                    X, T, P, K, F, H, HM = cl.harvest_coarse(systems, halves=True)
                    ref = T[:, 2]
                    # kept points per dx^2 of the subsample's spacing (1 is the target)
                    r = dict(n=int(len(ref)), plain=cl.rel_l2(P, ref), density=kept / expect)
                    if HM.any():
                        d = H[HM, 0] - H[HM, 1]
                        r.update(n_split=int(HM.sum()),
                                 noise=float(0.5 * np.linalg.norm(d) / np.linalg.norm(ref[HM])))
                    key = f"{name} steps={steps} window={window} resolution={fine}x"
                    out[key] = r
                    log(f"[labels] {key}: {r}")
                    del X, T, P, K, F, H, HM, systems
    rep["label_study"] = out
    with open(os.path.join(a.out, "label_study.json"), "w") as f:
        json.dump(rep, f, indent=1)
    log("[done]")


def held_out_jets(cl, w, spec, snaps, n, free_length, avg_steps=1, window=1.0):
    hj = jet_sets(spec, snaps, n, free_length, avg_steps, window)
    X2, T2, P2, K2, F2, H2, HM2 = cl.harvest_coarse(hj, params=w, halves=True)
    Y2 = cl.predict(w, X2)
    nh = Y2[:, :2] / np.linalg.norm(Y2[:, :2], axis=1, keepdims=True)
    ang = np.degrees(np.arccos(np.clip(np.einsum("ij,ij->i", nh, T2[:, :2]), -1, 1)))
    r = errors(T2[:, 2], P2, Y2[:, 2], K2)
    r.update(fallback_fraction=float(F2.mean()), normal_angle_deg_median=float(np.median(ang)))
    # the reference's own noise, split-half: each label recomputed from either
    # half of the fine interface particles; with independent halves the full
    # label's noise is half their difference, a floor for any predictor's error
    if HM2.any():
        ref = T2[HM2, 2]
        d = H2[HM2, 0] - H2[HM2, 1]
        r.update(n_split=int(HM2.sum()), reference_noise_floor=float(0.5 * np.linalg.norm(d) / np.linalg.norm(ref)),
                 mlp_on_split=cl.rel_l2(Y2[HM2, 2], ref), plain_on_split=cl.rel_l2(P2[HM2], ref))
    return r


def evaluate_and_cost(cl, w, a, rep):
    # held-out shapes (exact labels)
    ho = cl.shape_systems(a.held_out_shapes, seed=a.seed + 1000)
    Xh, Th, Ph, Ih = cl.harvest_shapes(ho)
    Yh = cl.predict(w, Xh)
    rep["held_out_shapes"] = errors(Th[:, 2], Ph, Yh[:, 2], cl.apply_fallback(Yh[:, 2], Ph))
    log(f"[eval] held-out shapes: {rep['held_out_shapes']}")
    for name, sel in (("layered", lambda s: s.meta["layered"]), ("lattice", lambda s: not s.meta["layered"]),
                      ("layered_discs", lambda s: s.meta["layered"] and s.name == "circle"),
                      ("layered_no_jitter", lambda s: s.meta["layered"] and s.meta["jitter"] == 0.0)):
        m = np.array([sel(ho[i]) for i in Ih], dtype=bool)
        if m.any():
            rep[f"held_out_shapes_{name}"] = errors(Th[m, 2], Ph[m], Yh[m, 2], cl.apply_fallback(Yh[m, 2], Ph[m]))
            log(f"[eval]   {name}: {rep[f'held_out_shapes_{name}']}")
    # held-out jets (the D = 20 dx workload at seeds 100-103, and varied smaller
    # jets), with the closure's curvature taken from the particle update
    rep["held_out_jets"] = held_out_jets(cl, w, HELD_OUT_JETS, _snaps(a.jet_snap_steps), a.jet_n,
                                         a.jet_free_length, a.label_steps, a.label_window)
    log(f"[eval] held-out jets (D = 20 dx): {rep['held_out_jets']}")
    rep["held_out_sweep_jets"] = held_out_jets(cl, w, SWEEP_HELD_OUT, _snaps(a.sweep_snap_steps), a.sweep_n,
                                               a.sweep_free_length, a.label_steps, a.label_window)
    log(f"[eval] held-out jets (D = 10-16 dx): {rep['held_out_sweep_jets']}")

    # cost: plain vs closure on a jet at D = 20 dx, and the same jet at 4x
    # resolution (D = 80 dx, 16x the particles, plain), per unit simulated time
    import workloads as wl
    base = wl.jet(n_target=a.cost_n, nD=20, Re=500.0, We=20.0, seed=7, free_length=60.0, prefill=20.0)
    rep["cost"] = dict(plain=throughput(base, w, a.bench_steps, False),
                       closure=throughput(base, w, a.bench_steps, True))
    log(f"[cost] D=20dx: {rep['cost']}")
    fine = wl.jet(n_target=16 * a.cost_n, nD=80, Re=500.0, We=20.0, seed=7, free_length=60.0, prefill=20.0)
    rep["cost"]["fine_plain_4x"] = throughput(fine, w, max(a.bench_steps // 4, 100), False)
    rep["cost"]["speedup_vs_4x_resolution"] = (rep["cost"]["fine_plain_4x"]["seconds_per_unit_time"]
                                               / rep["cost"]["closure"]["seconds_per_unit_time"])
    log(f"[cost] {rep['cost']}")
    with open(os.path.join(a.out, "closure_report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    log("[done]")


if __name__ == "__main__":
    main()
