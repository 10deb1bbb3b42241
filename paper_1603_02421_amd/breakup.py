"""The breakup-length study of Section 3-2 on the HIP update.

    python -m paper_1603_02421_amd.breakup [--nD 20] [--t-max 2.0] [--out DIR]

Jets in the paper's units (workloads.paper_jet: D0 = 0.01 m, water,
c0 = 10 m/s, alpha = 0.3, g along the jet beyond the orifice) for the inflow
speeds of Table 1 (0.07, 0.17, 0.20, 0.25 m/s) with the Wendland and the
cubic-spline kernel run as one batch of systems. Every `check` steps the
breakup criterion (sph_breakup: a gap of more than 1.5 h between particles
consecutive along the jet) is taken on every system; the first breakup gives
the breakup time and length L (from the orifice exit). Each row also carries
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


def run(nD: int = 20, t_max: float = 2.0, check: int = 400, kernels=(0, 1), u0s=U0, seed: int = 0, log=print):
    import workloads as wl
    from . import sim as simmod
    systems = [wl.paper_jet(u0, kernel=k, nD=nD, seed=seed + i) for i, (k, u0) in
               enumerate((k, u0) for k in kernels for u0 in u0s)]
    batch = wl.Batch(systems)
    starts = np.array([s.meta["exit"] for s in systems])
    first = {}
    t0 = time.perf_counter()
    steps = 0
    with simmod.Simulation(batch, dtype_bits=32) as sim:
        while True:
            sim.step(check)
            steps += check
            t = sim.read("time")
            L, broken = sim.breakup(starts)
            for i in range(len(systems)):
                if broken[i] and i not in first:
                    first[i] = (float(t[i]), float(L[i]))
            log(f"[breakup] {steps} steps, t = {t.min():.3f}-{t.max():.3f} s, broken {len(first)}/{len(systems)}, "
                f"{time.perf_counter() - t0:.1f} s")
            if len(first) == len(systems) or t.min() >= t_max:
                flags = int(sim.read("flags", allow_unstable=True)[0])
                break
    rows = []
    for i, s in enumerate(systems):
        u0 = s.meta["u0"]
        row = dict(u0=u0, kernel="wendland" if s.params["kernel"] == 0 else "cubic", nD=nD, n=s.n,
                   **groups_row(u0))
        if i in first:
            row.update(t_break=first[i][0], L_over_D0=first[i][1] / D0)
        else:
            row.update(t_break=None, L_over_D0=None)
        rows.append(row)
    return dict(rows=rows, steps=steps, wall_s=time.perf_counter() - t0, flags=flags, check=check, t_max=t_max)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nD", type=int, default=20)
    ap.add_argument("--t-max", type=float, default=2.0)
    ap.add_argument("--check", type=int, default=400)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    res = run(nD=a.nD, t_max=a.t_max, check=a.check, log=lambda m: print(m, flush=True))
    for r in res["rows"]:
        L = "not broken" if r["L_over_D0"] is None else f"L/D0 = {r['L_over_D0']:.2f} at t = {r['t_break']:.3f} s"
        print(f"u0 = {r['u0']:.2f} m/s {r['kernel']:8s} We {r['We']:.2f} Re {r['Re']:.0f} Fr {r['Fr']:.2f}: {L}; "
              f"eq. 37: {r['L_corr']:.2f}", flush=True)
    if a.out:
        os.makedirs(a.out, exist_ok=True)
        with open(os.path.join(a.out, "breakup_study.json"), "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
