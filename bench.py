"""Throughput of the SPH particle update on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c2-cubic|c5|c1]

Default workload: the batched Re/We sweep -- 64 independent tank-fed jets
(Re log-uniform in [100, 2000], We uniform in [5, 50], D resolved by 10-40
particles, 20k-400k particles each, about 8M in total, seed 1234), FP32,
Wendland kernel, hipGraph-replayed steps. A step is one predictor-corrector
step of every jet: cell sort, two evaluations of all right-hand sides, the
eq. 30-32 time step and the integrator. value = particle-steps/s over the
timed steps with all inputs resident on the GPU.

After the timed region the same context runs a few eagerly launched steps with
a HIP event pair around every kernel on the context's stream; the kernel with
the largest share of the step gives the roofline object (algorithmic bytes per
active particle x active particles / mean launch time). The same workload then
runs with the learned curvature closure in every system (closure: its
particle-steps/s, listed particles and fallback fraction). The FP64 oracle is
timed on the host cores on a bounded sample of the workload (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes of the method per active particle, FP32, 2-D: each field
# the step needs, counted once per sweep that needs it (neighbour re-reads are
# the reuse the cell order provides and are not counted). Colour sweep: pos 8,
# rho 4, type 4 -> C 4. Main sweep: pos 8, v 8, rho 4, type 4, C 4 -> drho/dt 4,
# a 8, n 8. Surface sweep: pos 8, rho 4, type 4, n 8, a 8 -> a 8. Predictor and
# corrector: state 20 + derivatives 12 -> state 20, each. Neighbour structure
# once per step: key 8 + 4, histogram 4, scan 1.2, scatter 8, permute 2 x 24.
# Per step, with two evaluations: 2 x (20 + 48 + 40) + 104 + 73 = 393, used as
# 400 B per particle-step.
METHOD_BYTES = {"colour": 20, "colour_skin": 20, "main": 48, "surface": 40, "predict": 52, "correct": 52}
METHOD_BYTES_PER_STEP = 400

# This implementation's own bytes per active particle and launch, FP32
# storage: every per-slot array the kernel reads once and every output written
# once. Layout: pos 16 (FP64 pair), vel 8, dens 4, mass 4, tag 4, id 4, cell 4,
# colour 4, drho 4, acc 8, nrm 8, kappa 4, vol 4, eos 16 (P/rho^2, C, rho,
# m/rho), neighbour mask 20 (one word per cell row).
IMPL_BYTES = {
    "colour": 16 + 4 + 4 + 4 + 4 + 16 + 20,               # pos vol cell tag dens -> colour eos skin-mask
    "colour_skin": 16 + 4 + 4 + 4 + 4 + 20 + 4 + 16,      # pos vol cell tag dens skin-mask -> colour eos
    "main": 4 + 16 + 8 + 16 + 20 + 4 + 4 + 8 + 8,         # tag pos vel eos mask cell -> drho acc nrm
    # per filtered particle: list entry tag nrm acc rho vol pos mask cell -> acc kappa kappa_plain
    # (88 B), over active particles at the 2.9% filtered on the 64-jet batch
    "surface": 0.029 * (4 + 4 + 8 + 8 + 4 + 4 + 16 + 20 + 4 + 8 + 4 + 4),
    "predict": 4 + 16 + 8 + 4 + 4 + 8 + 4 + 16 + 8 + 4 + 4,  # tag pos vel dens drho acc mass -> half state, vol
    "correct": 4 + 16 + 8 + 4 + 4 + 8 + 16 + 8 + 4 + 8,   # tag pos vel dens drho acc -> pos vel dens, key slot
    "sort_key": 16 + 4 + 4 + 4,                           # pos tag -> key slot
    "sort_scatter": 4 + 4 + 4 + 4 + 4,                    # key slot id cstart -> cell_ids
    "sort_permute": 4 + 4 + 4 + 40 + 40 + 4 + 4,          # key cstart cell_ids X -> Y cell vol
}


KERNEL_NAMES = {  # device function -> the name the library's profiler gives it
    "k_colour": "colour", "k_colour_skin": "colour_skin", "k_main": "main", "k_surface": "surface",
    "k_permute": "sort_permute", "k_predict": "predict", "k_correct": "correct", "k_key": "sort_key", "k_scatter": "sort_scatter",
    "k_stencil": "closure_stencil", "k_closure_net": "closure_net",
}


def sources_digest() -> str:
    """SHA-256 of the HIP sources: measured traffic applies only to the kernels it was taken on."""
    import hashlib
    d = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1603_02421_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            d.update(f.encode() + b"\0" + fh.read())
    return d.hexdigest()


def traffic_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"traffic_{workload}.json")


def measured_traffic(workload: str, cell_factor: float, block_sweep: int, kernel: str):
    """(HBM bytes per launch of `kernel`, the launch shape they were taken on)
    from the committed rocprofv3 counter summary, when it was taken on these
    sources and this cell size (the bytes a kernel moves follow its cells, not
    its workgroup size); (None, None) otherwise."""
    try:
        with open(traffic_path(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None, None
    if t.get("sources_sha256") != sources_digest():
        return None, None
    if abs(t.get("cell_factor", 0) - cell_factor) > 1e-9:
        return None, None
    k = t.get("kernels", {}).get(kernel)
    if k is None:
        return None, None
    return k["fetch_bytes"] + k["write_bytes"], f"cell size {t['cell_factor']} h, {t['block_sweep']}-thread sweep blocks"


def _pmc(path: str, counter: str):
    import collections
    import csv
    out = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].split("<")[0].replace("void ", "").split("::")[-1]
            out[name].append(float(r["Counter_Value"]))
    return out


def write_traffic(args):
    """Turn four rocprofv3 --pmc counter files (FETCH_SIZE and WRITE_SIZE of
    the workload, and of the 1 GiB copy) into profiles/traffic_<workload>.json."""
    import statistics
    fetch, write, cfetch, cwrite = args.traffic_from
    copy_bytes = float(1 << 30)
    cf = max(v for vals in _pmc(cfetch, "FETCH_SIZE").values() for v in vals) * 1024.0
    cw = max(v for vals in _pmc(cwrite, "WRITE_SIZE").values() for v in vals) * 1024.0
    fs, ws = copy_bytes / cf, copy_bytes / cw
    f, w = _pmc(fetch, "FETCH_SIZE"), _pmc(write, "WRITE_SIZE")
    kernels = {}
    for dev, name in KERNEL_NAMES.items():
        if dev in f and dev in w:
            kernels[name] = dict(fetch_bytes=statistics.median(f[dev]) * 1024.0 * fs,
                                 write_bytes=statistics.median(w[dev]) * 1024.0 * ws, dispatches=len(f[dev]))
    out = dict(workload=args.workload, cell_factor=args.cell_factor, block_sweep=args.block_sweep,
               sources_sha256=sources_digest(), fetch_scale=fs, write_scale=ws,
               note="median HBM bytes per dispatch, rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB) scaled by the "
                    "factors a plain 1 GiB device copy gives (bench.py --copy-calibration)",
               kernels=kernels)
    with open(traffic_path(args.workload), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def make_workload(name: str):
    import workloads as wl
    if name == "c3":
        b = wl.batch_sweep(n_jets=64, seed=1234)
        desc = ("batched Re/We sweep: 64 tank-fed jets, Re logU[100,2000], We U[5,50], D/dx U{10..40}, "
                "N logU[20k,400k] per jet, seed 1234, FP32, Wendland")
        return wl.Batch([wl.round_for_dtype(s, 32) for s in b.systems]), desc, 32
    if name in ("c2", "c2-cubic"):
        cubic = name == "c2-cubic"
        s = wl.round_for_dtype(wl.jet(n_target=300_000, nD=20, Re=500, We=20, kD=0.7, seed=0,
                                      kernel=wl.CUBIC if cubic else wl.WENDLAND), 32)
        return wl.Batch([s]), ("single jet D=20dx, Re=500, We=20, kD=0.7, N~300k, FP32, "
                               + ("cubic spline" if cubic else "Wendland")), 32
    if name == "c5":
        s = wl.round_for_dtype(wl.jet(n_target=4_000_000, nD=80, Re=1000, We=30, seed=0,
                                      free_length=100.0, prefill=50.0), 32)
        return wl.Batch([s]), "large jet D=80dx, 100D domain, N~4M, Re=1000, We=30, FP32, Wendland", 32
    if name == "c1":
        return wl.Batch([wl.dam_break()]), "dam break with obstacle, 1,600 fluid + 668 wall, FP64", 64
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(batch, n_jets: int = 4, steps: int = 20):
    """Oracle particle-steps/s on a bounded sample of the workload: n_jets of its
    jets, at the 1/8, 3/8, 5/8 and 7/8 quantiles of size, each stepped `steps`
    times on all host cores, then the same on one core."""
    import oracle
    import workloads as wl
    oracle.build(force=False)
    systems = sorted(batch.systems, key=lambda s: s.n)
    k = len(systems)
    picks = [systems[min(k - 1, int((2 * i + 1) * k / (2 * n_jets)))] for i in range(n_jets)] if k > n_jets \
        else systems
    all_cores = oracle.threads()

    def run(threads):
        oracle.set_threads(threads)
        total, el = 0.0, 0.0
        for sy in picks:
            st = oracle.State(sy)
            n0 = int((st.type != wl.INACTIVE).sum())
            t0 = time.perf_counter()
            st.step(steps)
            el += time.perf_counter() - t0
            total += steps * 0.5 * (n0 + int((st.type != wl.INACTIVE).sum()))
        return total / el, el

    v_all, t_all = run(all_cores)
    v_one, t_one = run(1)
    oracle.set_threads(all_cores)
    sizes = ", ".join(str(sy.n) for sy in picks)
    return dict(value=v_all, unit="particle-steps/s", cores=all_cores, kind="oracle",
                sample=f"{len(picks)} jets of the workload (N = {sizes}; the 1/8, 3/8, 5/8, 7/8 size quantiles), "
                       f"{steps} steps each, FP64 C oracle with OpenMP: {t_all:.1f} s on {all_cores} threads, "
                       f"{t_one:.1f} s on 1",
                single_core=dict(value=v_one, cores=1))


def closure_leg(sph, batch, bits, block_sweep, cell_factor, args):
    """The same workload and launch shape with the learned closure in every
    system (shipped weights, fallback tolerance 0.2), timed the same way."""
    import torch
    import workloads as wl
    from paper_1603_02421_amd import closure as cl
    systems = []
    for s in batch.systems:
        c = s.copy()
        c.params = dict(s.params, closure=1, closure_tol=0.2)
        systems.append(c)
    cb = wl.Batch(systems)
    sim = sph.Simulation(cb, dtype_bits=bits, block_sweep=block_sweep, xcd_remap=args.xcd, cell_factor=cell_factor)
    sim.set_closure(cl.load())
    sim.step(args.warmup)
    sim.sync()
    n0 = int(sim.read("nactive", allow_unstable=True).sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.step(args.steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    n1 = int(sim.read("nactive", allow_unstable=True).sum())
    prof = sim.profile(args.profile_steps)
    kernels = {k: dict(avg_ms=round(v["avg_ms"], 4), calls=v["calls"])
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["calls"])}
    sim.evaluate()
    listed = sim.read("closure", allow_unstable=True)[:, 3] == 1.0
    fb = sim.read("fallback", allow_unstable=True)
    sim.close()
    value = args.steps * 0.5 * (n0 + n1) / (ms * 1e-3)
    print(f"[bench] closure: {args.steps} steps in {ms:.1f} ms, {value:.4g} particle-steps/s", flush=True)
    return dict(value=value, unit="particle-steps/s", ms_per_step=ms / args.steps, tolerance=0.2,
                listed=int(listed.sum()), fallback_fraction=float(fb[listed].mean()) if listed.any() else 0.0,
                kernels=kernels)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-closure", action="store_true", help="skip the learned-closure leg")
    ap.add_argument("--block-sweep", type=int, default=0)
    ap.add_argument("--xcd", type=int, default=-1)
    ap.add_argument("--cell-factor", type=float, default=0.0,
                    help="override every system's cell size as this multiple of h (skips the autotuner)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (keep the scenario cell size)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic_<workload>.json from rocprofv3 --pmc counter files "
                         "(needs --cell-factor and --block-sweep of the profiled run)")
    args = ap.parse_args()
    if args.traffic_from:
        write_traffic(args)
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": src.numel() * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the batched jets would "
              "shard across GPUs by whole jets; the library runs on one GPU per process).", file=sys.stderr)
        raise SystemExit(2)

    import torch
    import paper_1603_02421_amd as sph

    batch, desc, bits = make_workload(args.workload)
    if args.cell_factor > 0:
        for sy in batch.systems:
            sy.params["cell_size"] = args.cell_factor * sy.params["h"]
        desc += f", cell size {args.cell_factor} h"
    print(f"[bench] workload {args.workload}: {desc}; n={batch.n}", flush=True)
    tune = None
    cell_factor, block_sweep = args.cell_factor, args.block_sweep
    if not args.no_tune and args.cell_factor <= 0 and args.block_sweep == 0:
        t0 = time.perf_counter()
        tune = sph.autotune(batch, dtype_bits=bits, trial_steps=10)
        cell_factor, block_sweep = tune["cell_factor"], tune["block_sweep"]
        print(f"[bench] autotune {time.perf_counter() - t0:.1f} s: {tune}", flush=True)
        desc += f", autotuned cell size {cell_factor} h, {block_sweep}-thread sweep blocks"
    t0 = time.perf_counter()
    sim = sph.Simulation(batch, dtype_bits=bits, block_sweep=block_sweep, xcd_remap=args.xcd,
                         cell_factor=cell_factor)
    print(f"[bench] init {time.perf_counter() - t0:.1f} s, workspace {sim.workspace_bytes / 2**30:.2f} GiB",
          flush=True)
    sim.step(args.warmup)
    sim.sync()
    n0 = int(sim.read("nactive", allow_unstable=True).sum())
    st = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    w0 = time.perf_counter()
    sim.step(args.steps)
    e1.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    n1 = int(sim.read("nactive", allow_unstable=True).sum())
    flags = int(sim.read("flags", allow_unstable=True)[0])
    psteps = args.steps * 0.5 * (n0 + n1)
    value = psteps / (ms * 1e-3)
    print(f"[bench] {args.steps} steps in {ms:.1f} ms (wall {wall * 1e3:.1f} ms), active {n0} -> {n1}, "
          f"flags {flags}", flush=True)

    prof = sim.profile(args.profile_steps)
    n_act = int(sim.read("nactive", allow_unstable=True).sum())
    step_ms = sum(v["avg_ms"] * v["calls"] for v in prof.values()) / max(args.profile_steps, 1)
    dom = max((k for k in prof if k in METHOD_BYTES), key=lambda k: prof[k]["avg_ms"] * prof[k]["calls"])
    avg = prof[dom]["avg_ms"]
    bytes_launch = METHOD_BYTES[dom] * n_act
    achieved = bytes_launch / (avg * 1e-3) / 1e9
    kernels = {k: dict(avg_ms=round(v["avg_ms"], 4), calls=v["calls"],
                       share=round(v["avg_ms"] * v["calls"] / args.profile_steps / step_ms, 4))
               for k, v in sorted(prof.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["calls"])}
    impl_step_bytes = sum(IMPL_BYTES.get(k, 0) * v["calls"] for k, v in prof.items()) / args.profile_steps
    traffic_bytes, traffic_launch = measured_traffic(args.workload, cell_factor, block_sweep, dom)
    out = {
        "metric": "particle-steps/s (plain vs learned closure, batched jets); % HBM roofline",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if bits == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n_particles": batch.n, "n_systems": len(batch.systems),
                   "n_active": n_act, "closure": "plain", "graph": True, "instability_flags": flags,
                   "autotune": tune},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_bytes, "traffic_launch": traffic_launch,
                     "algo_bytes_per_particle": METHOD_BYTES[dom], "avg_launch_ms": avg,
                     "impl_bytes_per_particle": IMPL_BYTES[dom],
                     "impl_frac": IMPL_BYTES[dom] * n_act / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "step_model": {"algo_bytes_per_particle_step": METHOD_BYTES_PER_STEP,
                       "hbm_frac": METHOD_BYTES_PER_STEP * value / (HBM_PEAK_GBS * 1e9),
                       "impl_bytes_per_particle_step": impl_step_bytes,
                       "impl_hbm_frac": impl_step_bytes * value / (HBM_PEAK_GBS * 1e9)},
        "kernels": kernels,
    }
    sim.close()
    if not args.no_closure:
        out["closure"] = closure_leg(sph, batch, bits, block_sweep, cell_factor, args)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", flush=True)
        out["cpu_baseline"] = cpu_baseline(batch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
