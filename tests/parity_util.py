"""Comparison helpers for the HIP-vs-oracle parity tests.

Tolerances follow one rule: the FP32 path must agree with the FP64 oracle to
1e-5 of each quantity's absolute-sum scale S_a = sum_b |term_ab| (the bound on
rounding error for a sum of terms of mixed sign), the FP64 path to 1e-10 of it.
Particles whose normal magnitude lies within rounding reach of the filter
threshold eps (eq. 20), or that have such a neighbour, take a discrete decision
that either precision may take either way; they are excluded and counted.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("colour", "drhodt", "accel", "normal", "nflag", "curv", "dt")


def gpu_eval(sim):
    sim.evaluate()
    return dict(
        colour=sim.read("colour"), drho=sim.read("drhodt"), acc=sim.read("accel"),
        nrm=sim.read("normal"), nflag=sim.read("nflag"), kappa=sim.read("curv"),
        dt=sim.read("dt"), type=sim.read("type"))


def near_threshold_mask(orc_res, params_per_particle_eps, start, nbr, rel=2e-6):
    """True for particles whose (or whose neighbour's) |n| is within rounding
    reach of eps."""
    m = np.linalg.norm(orc_res["nrm"], axis=1)
    near = np.abs(m - params_per_particle_eps) <= rel * orc_res["s_nrm"] + 1e-7 * params_per_particle_eps
    out = near.copy()
    # a particle is affected if it or any neighbour is near the threshold
    n = len(m)
    counts = np.diff(start)
    owner = np.repeat(np.arange(n), counts)
    hit = near[nbr]
    out[owner[hit]] = True
    return out


def compare_eval(g, o, eps_pp, start, nbr, tol, fluid_mask):
    """Return a dict of (max normalised error, n compared) per field and the
    number of excluded particles; raises AssertionError on a violation."""
    excl = near_threshold_mask(o, eps_pp, start, nbr)
    keep = ~excl
    report = {"excluded": int(excl.sum())}
    tiny = 1e-300

    def chk(name, gv, ov, scale, mask):
        if gv.ndim == 2:
            err = np.linalg.norm(gv - ov, axis=1)
        else:
            err = np.abs(gv - ov)
        r = err / (scale + tiny)
        r = np.where(mask, r, 0.0)
        worst = float(r.max()) if r.size else 0.0
        report[name] = worst
        if worst > tol:
            i = int(np.argmax(r))
            raise AssertionError(f"{name}: particle {i} err {err[i]:.3e} scale {scale[i]:.3e} "
                                 f"(ratio {worst:.3e} > {tol:.1e}); gpu {gv[i]} oracle {ov[i]}")

    act = o["colour"] > 0
    chk("colour", g["colour"], o["colour"], np.abs(o["colour"]), act)
    chk("drhodt", g["drho"], o["drho"], o["s_drho"], act & keep)
    chk("normal", g["nrm"], o["nrm"], o["s_nrm"], fluid_mask & keep)
    chk("accel", g["acc"], o["acc"], o["s_acc"], fluid_mask & keep)
    fl = fluid_mask & keep
    mism = int((g["nflag"][fl] != o["nflag"][fl]).sum())
    report["nflag_mismatch"] = mism
    assert mism == 0, f"{mism} normal-filter flags differ away from the threshold"
    return report
