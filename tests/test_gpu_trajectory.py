"""An FP32 jet trajectory against the oracle out to its divergence horizon.

The horizon (the reading of the tolerance for trajectories) is where two
oracle runs whose fluid positions start one FP64 ulp apart separate by 1e-5 dx.
The FP32 path rounds velocities, densities and accelerations to FP32 at every
step, about 1e8 times an FP64 ulp, so the jet's chaotic episodes amplify its
deviation long before they amplify an FP64 ulp. Two things are checked:

- up to the last checkpoint at which an oracle run started one FP32 ulp away
  (velocities and rho - rho0 of the fluid nudged by one float ulp) is still
  within 1e-5 dx of the unperturbed one, the GPU is within 1e-4 of the oracle
  (dx, rho0 and the largest speed);
- at every checkpoint to the end, the GPU is no farther from the oracle than
  20 times that FP32-ulp pair is from each other (1e-6 dx floor): the HIP path
  behaves like one more realisation of the same FP32 state.
"""
import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

STEPS, EVERY = 3000, 100


def say(*a):
    print(*a, flush=True)


def test_fp32_jet_to_the_divergence_horizon(gpu, orc):
    s = wl.round_for_dtype(wl.jet(n_target=12_000, nD=12, Re=400, We=15, seed=0, free_length=8.0, prefill=4.0), 32)
    dx, rho0 = s.meta["dx"], s.params["rho0"]
    fl = s.type == wl.FLUID
    ulp64 = s.copy()
    ulp64.pos = np.where(fl[:, None], np.nextafter(s.pos, np.inf), s.pos)
    ulp32 = s.copy()
    ulp32.vel = np.where(fl[:, None], np.nextafter(s.vel.astype(np.float32), np.float32(np.inf)).astype(np.float64),
                         s.vel)
    d32 = (s.rho - rho0).astype(np.float32)
    ulp32.rho = np.where(fl, rho0 + np.nextafter(d32, np.float32(np.inf)).astype(np.float64), s.rho)
    ref, a64, a32 = orc.State(s), orc.State(ulp64), orc.State(ulp32)
    horizon64, within32 = None, 0
    say(f"[horizon] jet n={s.n}, {STEPS} steps")
    with gpu.Simulation(s) as sim:
        for k in range(EVERY, STEPS + 1, EVERY):
            sim.step(EVERY)
            for st in (ref, a64, a32):
                st.step(EVERY)
            pos, vel, rho = sim.read("pos"), sim.read("vel"), sim.read("rho")
            act = ref.type != wl.INACTIVE
            ep = np.abs(pos[act] - ref.pos[act]).max() / dx
            ev = np.abs(vel[act] - ref.vel[act]).max() / np.abs(ref.vel[act]).max()
            er = np.abs(rho[act] - ref.rho[act]).max() / rho0
            s64 = np.abs(a64.pos - ref.pos).max() / dx
            s32 = np.abs(a32.pos - ref.pos).max() / dx
            say(f"   {k}: gpu pos {ep:.2e} vel {ev:.2e} rho {er:.2e} | oracle pairs fp64-ulp {s64:.2e} fp32-ulp {s32:.2e}")
            if horizon64 is None and s64 > 1e-5:
                horizon64 = k
            if s32 <= 1e-5 and within32 == k - EVERY:
                within32 = k
                assert ep <= 1e-4 and ev <= 1e-4 and er <= 1e-4
            assert ep <= 20.0 * max(s32, 1e-6)
    say(f"   FP64 1-ulp horizon: {'beyond ' + str(STEPS) if horizon64 is None else horizon64} steps; "
        f"GPU within 1e-4 through step {within32}")
    assert within32 >= 500
