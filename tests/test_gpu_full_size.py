"""Parity at the benchmark's full size: the batch of 64 jets, 7.88M particles in
FP32, that bench.py times, in the launch shape its autotuner picks there (cell
size 1.05 h, 256-thread sweep blocks) and with graph-replayed steps.

Every particle of every jet is compared with the FP64 oracle: one evaluation to
1e-5 of each quantity's absolute-sum scale (the bound of the small cases), and
a three-step trajectory to 1e-4 (positions in units of the jet's dx, density
of rho0 = 1, velocities of the largest speed). The jets are independent
systems, so the oracle runs them as one batch as well. The closure leg is
checked on the same batch with the closure bounds of the small cases.
"""
import numpy as np
import pytest

import workloads as wl
from parity_util import compare_eval, gpu_eval

pytestmark = pytest.mark.gpu

CELL_FACTOR, BLOCK_SWEEP = 1.05, 256


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c3():
    import bench
    batch, _, bits = bench.make_workload("c3")
    assert bits == 32 and len(batch.systems) == 64
    for sy in batch.systems:
        sy.params["cell_size"] = CELL_FACTOR * sy.params["h"]
    return batch


def _per_particle(batch, f):
    return np.concatenate([np.full(s.n, f(s)) for s in batch.systems])


def test_full_batch_single_evaluation(gpu, orc, c3):
    say(f"[full size] evaluation: 64 jets, n={c3.n}, cell {CELL_FACTOR} h, block {BLOCK_SWEEP}")
    with gpu.Simulation(c3, dtype_bits=32, block_sweep=BLOCK_SWEEP) as sim:
        g = gpu_eval(sim)
    o = orc.evaluate(c3)
    start, nbr = orc.neighbors(c3)
    say(f"   oracle: {len(nbr)} neighbour pairs")
    eps = _per_particle(c3, lambda s: s.params["eps_h"] / s.params["h"])
    rep = compare_eval(g, o, eps, start, nbr, 1e-5, c3.cat("type") == wl.FLUID)
    say("  ", rep)
    ok = np.isfinite(o["dt"]) & (o["dt"] > 0)
    assert ok.sum() == 64
    assert np.allclose(g["dt"][ok], o["dt"][ok], rtol=1e-5, atol=0)


def test_full_batch_trajectory(gpu, orc, c3):
    n_steps = 3
    say(f"[full size] trajectory: 64 jets, n={c3.n}, {n_steps} graph-replayed steps")
    st = orc.State(c3)
    with gpu.Simulation(c3, dtype_bits=32, block_sweep=BLOCK_SWEEP, use_graph=1, graph_steps=2) as sim:
        sim.step(n_steps)
        pos, vel, rho = sim.read("pos"), sim.read("vel"), sim.read("rho")
        typ, flags, t = sim.read("type"), sim.read("flags")[0], sim.read("time")
    st.step(n_steps)
    assert flags == 0
    assert np.array_equal(typ, st.type)
    assert np.allclose(t, st.time, rtol=1e-5)
    act = st.type != wl.INACTIVE
    dx = _per_particle(c3, lambda s: s.meta["dx"])
    ep = (np.linalg.norm(pos - st.pos, axis=1) / dx)[act].max()
    er = np.abs(rho - st.rho)[act].max()
    ev = np.linalg.norm(vel - st.vel, axis=1)[act].max() / np.linalg.norm(st.vel, axis=1)[act].max()
    say(f"   after {n_steps} steps: pos {ep:.2e} dx, rho {er:.2e}, vel {ev:.2e}")
    assert ep <= 1e-4 and er <= 1e-4 and ev <= 1e-4


def test_large_single_jet_evaluation_and_steps(gpu, orc):
    """The largest single-jet workload (D = 80 dx, 100 D domain, 4.0M particles,
    FP32, cell size 1.05 h): one evaluation to 1e-5 of scale and two
    graph-replayed steps to 1e-4, every particle compared."""
    import bench
    batch, _, bits = bench.make_workload("c5")
    s = batch.systems[0]
    s.params["cell_size"] = CELL_FACTOR * s.params["h"]
    say(f"[full size] one jet D = 80 dx: n={s.n}, cell {CELL_FACTOR} h")
    with gpu.Simulation(s, dtype_bits=bits, block_sweep=BLOCK_SWEEP) as sim:
        g = gpu_eval(sim)
    o = orc.evaluate(s)
    start, nbr = orc.neighbors(s)
    rep = compare_eval(g, o, np.full(s.n, s.params["eps_h"] / s.params["h"]), start, nbr, 1e-5,
                       s.type == wl.FLUID)
    say("  ", rep)
    assert np.allclose(g["dt"], o["dt"], rtol=1e-5, atol=0)
    del g, o, start, nbr
    st = orc.State(s)
    with gpu.Simulation(s, dtype_bits=bits, block_sweep=BLOCK_SWEEP, use_graph=1, graph_steps=2) as sim:
        sim.step(2)
        pos, vel, rho = sim.read("pos"), sim.read("vel"), sim.read("rho")
        flags = sim.read("flags")[0]
    st.step(2)
    assert flags == 0
    act = st.type != wl.INACTIVE
    ep = np.abs(pos - st.pos)[act].max() / s.meta["dx"]
    er = np.abs(rho - st.rho)[act].max() / s.params["rho0"]
    ev = np.abs(vel - st.vel)[act].max() / np.abs(st.vel)[act].max()
    say(f"   after 2 steps: pos {ep:.2e} dx, rho {er:.2e}, vel {ev:.2e}")
    assert ep <= 1e-4 and er <= 1e-4 and ev <= 1e-4


def test_full_batch_closure_evaluation(gpu, orc, c3):
    """The closure leg of the benchmark: the same batch with the learned closure
    in every jet (random network weights). The listed particles, network
    outputs, fallback decisions, accelerations and dt are compared everywhere;
    the stencils of 4,000 listed particles one by one, the others by a check
    that they hold the oracle's points in its order."""
    from test_gpu_closure import check_closure_evaluation
    batch = wl.Batch([s.copy() for s in c3.systems])
    for s in batch.systems:
        s.params["closure"] = 1
    say(f"[full size] closure evaluation: 64 jets, n={batch.n}")
    check_closure_evaluation(gpu, orc, batch, 32, 0.2, sim_kw=dict(block_sweep=BLOCK_SWEEP), sample=4000)


def test_surface_lane_split_matches_one_lane(gpu, c3):
    """The surface sweep gives each entry of a short list (at most 65,536
    entries) four lanes that split its neighbours by mask bit, and each entry of
    a long list one lane. One jet evaluated alone (a list of a few thousand
    entries: four lanes) and inside the 64-jet batch (about 230k entries: one
    lane) has the same cells, order and masks, so the colour, continuity and
    normal sweeps agree bit for bit, and the curvature and the accelerations
    it sets agree to the rounding of the sum's order."""
    j = 0
    one = c3.systems[j]
    say(f"[surface lanes] jet {j} alone (n={one.n}) and in the batch (n={c3.n})")
    with gpu.Simulation(one, dtype_bits=32, block_sweep=BLOCK_SWEEP) as sim:
        a = gpu_eval(sim)
    with gpu.Simulation(c3, dtype_bits=32, block_sweep=BLOCK_SWEEP) as sim:
        b = gpu_eval(sim)
    n = one.n
    b = {k: (v[:n] if k != "dt" else v[j:j + 1]) for k, v in b.items()}
    for k in ("colour", "drho", "nrm", "nflag", "type"):
        assert np.array_equal(a[k], b[k]), k
    listed = a["nflag"] == 1
    say(f"   {int(listed.sum())} filtered particles")
    assert listed.sum() > 100
    ek = np.abs(a["kappa"] - b["kappa"])[listed].max() / np.abs(b["kappa"][listed]).max()
    ea = np.linalg.norm(a["acc"] - b["acc"], axis=1).max() / np.linalg.norm(b["acc"], axis=1).max()
    say(f"   curvature {ek:.2e}, acceleration {ea:.2e} of their largest magnitudes")
    assert ek < 1e-5 and ea < 1e-5
    assert np.array_equal(a["acc"][~listed], b["acc"][~listed])
    assert np.allclose(a["dt"], b["dt"], rtol=1e-6, atol=0)
