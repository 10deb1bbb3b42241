"""The breakup-length study of Section 3-2 on the HIP update.

    python -m paper_1603_02421_amd.breakup [--nD 20] [--t-max 1.0] [--out DIR]

Jets in the paper's units (workloads.paper_jet: D0 = 0.01 m, water,
c0 = 10 m/s, alpha = 0.3, g along the jet beyond the orifice) for the inflow
speeds of Table 1 (0.07, 0.17, 0.20, 0.25 m/s) with the Wendland and the
cubic-spline kernel run as one batch of systems. Every `check` steps the
breakup criterion (sph_breakup: a gap of more than 1.5 h between particles
consecutive along the jet) is taken on every system. Reported per system:
the first breakup (time and length from the orifice exit) and the intact
length of the established jet, the median over the second half of the run. Each row also carries
the dimensionless groups with the orifice radius (eq. 33-36) and the length
of the correlation of eq. 37. All arithmetic of the update and the criterion
runs in the library; this module only marshals and tabulates.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np

U0 = (0.07, 0.17, 0.20, 0.25)
MU, SIGMA, RHO0, G, D0 = 1e-3, 0.072, 1000.0, 9.81, 0.01


def groups_row(u0: float):
    from workloads import groups
    R = D0 / 2
    We = groups.weber(RHO0, u0, R, SIGMA)
    Re = groups.reynolds(RHO0, u0, R, MU)
    Oh = groups.ohnesorge(We, Re)
    return dict(We=We, Re=Re, Oh=Oh, Fr=groups.froude(u0, G, D0),
                L_corr=groups.breakup_length_correlation(We, Oh))


def run(nD: int = 20, t_max: float = 1.0, check: int = 400, kernels=(0, 1), u0s=U0, seed: int = 0,
        free_length: float = 70.0, log=print):
    """Steps the batch to t_max (every system's own time), taking the breakup
    criterion every `check` steps. Per system: the first breakup (time and
    length), and the intact length L of the established jet -- the median, over
    the checks in the second half of the run, of the length to the first gap
    (checks without a gap count with the jet's full length). The domain reaches
    free_length D0 beyond the orifice: a jet intact to its end is cut there."""
    import workloads as wl
    from . import sim as simmod
    # the tank holds the same volume at every resolution (the piston travels
    # about 3.6 D0 in 1 s at the fastest inflow, of a 14 D0 tank)
    n_target = int(40_000 * (nD / 20.0) ** 2)
    systems = [wl.paper_jet(u0, kernel=k, nD=nD, seed=seed + i, n_target=n_target, free_length=free_length)
               for i, (k, u0) in
               enumerate((k, u0) for k in kernels for u0 in u0s)]
    batch = wl.Batch(systems)
    starts = np.array([s.meta["exit"] for s in systems])
    first = {}
    series = [[] for _ in systems]
    t0 = time.perf_counter()
    steps = 0
    flag_time = None
    with simmod.Simulation(batch, dtype_bits=32) as sim:
        while True:
            sim.step(check)
            steps += check
            # a stretching ligament's density may leave [rho0/2, 2 rho0] (the
            # instability flag): recorded, and the run goes on
            t = sim.read("time", allow_unstable=True)
            if flag_time is None and int(sim.read("flags", allow_unstable=True)[0]) & ~8:
                flag_time = float(t.min())
            L, broken = sim.breakup(starts)
            for i in range(len(systems)):
                series[i].append((float(t[i]), float(L[i]), int(broken[i])))
                if broken[i] and i not in first:
                    first[i] = (float(t[i]), float(L[i]))
            if steps % (25 * check) == 0:
                log(f"[breakup] {steps} steps, t = {t.min():.3f}-{t.max():.3f} s, {time.perf_counter() - t0:.1f} s")
            if t.min() >= t_max:
                flags = int(sim.read("flags", allow_unstable=True)[0])
                rho = sim.read("rho", allow_unstable=True)
                pos = sim.read("pos", allow_unstable=True)
                typ = sim.read("type", allow_unstable=True)
                break
    off = batch.offsets
    low = []   # per system: fluid particles outside [rho0/2, 2 rho0] at the end, nearest one's distance
    for i in range(len(systems)):
        sl = slice(off[i], off[i + 1])
        bad = (typ[sl] == wl.FLUID) & ((rho[sl] < 500.0) | (rho[sl] > 2000.0))
        low.append((int(bad.sum()), float((pos[sl][bad, 0] - starts[i]).min() / D0) if bad.any() else None))
    rows = []
    for i, s in enumerate(systems):
        u0 = s.meta["u0"]
        row = dict(u0=u0, kernel="wendland" if s.params["kernel"] == 0 else "cubic", nD=nD, n=s.n,
                   free_length_over_D0=free_length,
                   **groups_row(u0))
        row.update(t_first=first[i][0] if i in first else None,
                   L_first_over_D0=first[i][1] / D0 if i in first else None)
        late = [(L, b) for (tt, L, b) in series[i] if tt >= 0.5 * t_max]
        row.update(L_over_D0=float(np.median([L for L, _ in late])) / D0,
                   L_q25_over_D0=float(np.percentile([L for L, _ in late], 25)) / D0,
                   L_q75_over_D0=float(np.percentile([L for L, _ in late], 75)) / D0,
                   broken_fraction=float(np.mean([b for _, b in late])), n_checks=len(late),
                   out_of_range=low[i][0], out_of_range_nearest_over_D0=low[i][1])
        rows.append(row)
    return dict(rows=rows, steps=steps, wall_s=time.perf_counter() - t0, flags=flags, flag_time=flag_time,
                check=check, t_max=t_max, series=series)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nD", type=int, default=20)
    ap.add_argument("--t-max", type=float, default=1.0)
    ap.add_argument("--check", type=int, default=400)
    ap.add_argument("--free-length", type=float, default=70.0, help="domain beyond the orifice, in D0")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = run(nD=a.nD, t_max=a.t_max, check=a.check, free_length=a.free_length, log=lambda m: print(m, flush=True))
    for r in res["rows"]:
        first = "none" if r["L_first_over_D0"] is None else f"{r['L_first_over_D0']:.2f} at {r['t_first']:.3f} s"
        print(f"u0 = {r['u0']:.2f} m/s {r['kernel']:8s} nD {r['nD']} We {r['We']:.2f} Re {r['Re']:.0f} Fr {r['Fr']:.2f}: "
              f"L/D0 = {r['L_over_D0']:.2f} [{r['L_q25_over_D0']:.2f}, {r['L_q75_over_D0']:.2f}] "
              f"(broken at {100 * r['broken_fraction']:.0f}% of {r['n_checks']} checks), first breakup {first}; "
              f"eq. 37: {r['L_corr']:.2f}; density out of range: {r['out_of_range']} particles, nearest "
              f"{r['out_of_range_nearest_over_D0']} D0 from the exit", flush=True)
    print(f"steps {res['steps']}, wall {res['wall_s']:.1f} s, flags {res['flags']} (first at t = {res['flag_time']})",
          flush=True)
    if a.out:
        os.makedirs(a.out, exist_ok=True)
        with open(os.path.join(a.out, f"breakup_study_nD{a.nD}.json"), "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
