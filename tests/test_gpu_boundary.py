"""The C-ABI's state handling on the GPU: checkpoint and resume, instability
detection with the state still readable, and the half step of a system whose
particles outrun the cell skin (scanned again, exactly).

Resumed runs must equal straight runs bit for bit (the blob holds the stored
values and the cell order is (cell, id) whatever order a state arrives in).
The rescanned half step is held to the same trajectory bounds against the
oracle as any other step: the oracle builds fresh neighbour lists at every
evaluation, so it has no skin at all.
"""
import math

import numpy as np
import pytest

import workloads as wl
from paper_1603_02421_amd import native

pytestmark = pytest.mark.gpu

STRAIGHT = ("pos", "vel", "rho", "type", "time", "dt", "accel", "drhodt", "colour", "normal")


def say(*a):
    print(*a, flush=True)


def _jet(seed=0, **kw):
    args = dict(n_target=12_000, nD=12, Re=400, We=15, seed=seed, free_length=8.0, prefill=4.0)
    args.update(kw)
    return wl.round_for_dtype(wl.jet(**args), 32)


def _cases():
    return dict(
        jet=(_jet(), 32),
        dam_break=(wl.dam_break(), 64),
        batch=(wl.Batch([_jet(1, n_target=5_000, nD=10), _jet(2, n_target=6_000, nD=11, kernel=wl.CUBIC),
                         wl.round_for_dtype(wl.circle(7.0, jitter=0.02, seed=3), 32)]), 32),
    )


@pytest.mark.parametrize("name", ["jet", "dam_break", "batch"])
def test_checkpoint_then_resume_equals_straight_run(gpu, name):
    obj, bits = _cases()[name]
    say(f"[checkpoint] case={name} n={obj.n} bits={bits}")
    with gpu.Simulation(obj, dtype_bits=bits) as a:
        a.step(10)
        blob = a.checkpoint()
        at10 = {f: a.read(f) for f in ("pos", "vel", "rho", "type", "time")}
        a.step(10)
        straight = {f: a.read(f) for f in STRAIGHT}
    with gpu.Simulation(obj, dtype_bits=bits) as b:
        b.step(3)                       # a different state, overwritten by the blob
        b.restore(blob)
        for f, x in at10.items():
            assert np.array_equal(b.read(f), x), f"restored {f} differs"
        assert np.all(b.read("accel") == 0.0)   # derived fields are cleared
        b.step(10)
        for f in STRAIGHT:
            assert np.array_equal(b.read(f), straight[f]), f"resumed {f} differs from the straight run"


def test_restore_into_a_context_with_a_smaller_courant_number(gpu):
    """Recovery: the same state in a context whose systems use Cr = 0.1 steps
    with half the dt of Cr = 0.2 (eq. 32), from the same time."""
    obj = _jet(4)
    with gpu.Simulation(obj) as a:
        a.step(4)
        blob = a.checkpoint()
        t4 = a.read("time")
        a.step(1)
        dt_a = a.read("dt")
    slow = obj.copy()
    slow.params["courant"] = 0.1
    with gpu.Simulation(slow) as b:
        b.restore(blob)
        assert np.array_equal(b.read("time"), t4)
        b.step(1)
        assert np.array_equal(b.read("dt"), 0.5 * dt_a)


def test_restore_rejects_blobs_of_another_shape(gpu):
    a_obj, b_obj = _jet(5), _jet(6, n_target=9_000)
    with gpu.Simulation(a_obj) as a, gpu.Simulation(b_obj) as b, gpu.Simulation(a_obj, dtype_bits=64) as c:
        blob = a.checkpoint()
        for target, data in ((b, blob), (c, blob), (a, blob[:-4]), (a, b"XXXX" + blob[4:])):
            with pytest.raises(native.SphError) as e:
                target.restore(data)
            assert e.value.status == native.SPH_EINVAL
        a.restore(blob)                 # the right blob still loads


def test_non_finite_position_is_rejected_at_init(gpu):
    s = _jet(7)
    s.pos[17, 0] = math.nan
    with pytest.raises(native.SphError) as e:
        gpu.Simulation(s)
    assert e.value.status == native.SPH_EINVAL


def test_non_finite_velocity_is_flagged_with_the_state_readable(gpu):
    s = _jet(8)
    fluid = np.nonzero(s.type == wl.FLUID)[0]
    bad = int(fluid[len(fluid) // 2])
    s.vel[bad] = [math.nan, 0.0]
    say(f"[unstable] NaN velocity at id {bad}")
    with gpu.Simulation(s) as sim:
        sim.step(1)
        with pytest.raises(native.SphError) as e:
            sim.read("pos")
        assert e.value.status == native.SPH_EUNSTABLE
        flags = int(sim.read("flags", allow_unstable=True)[0])
        assert flags & 1
        pos = sim.read("pos", allow_unstable=True)
        # the data still comes back: far from the bad particle nothing changed kind
        far = np.linalg.norm(s.pos - s.pos[bad], axis=1) > 10 * s.params["h"]
        assert np.all(np.isfinite(pos[far]))


def test_overdense_input_is_flagged_with_the_state_readable(gpu):
    s = _jet(9)
    fluid = np.nonzero(s.type == wl.FLUID)[0][:50]
    s.rho[fluid] = 3.0 * s.params["rho0"]
    with gpu.Simulation(s) as sim:
        sim.step(1)
        with pytest.raises(native.SphError) as e:
            sim.read("rho")
        assert e.value.status == native.SPH_EUNSTABLE
        assert int(sim.read("flags", allow_unstable=True)[0]) & 2
        rho = sim.read("rho", allow_unstable=True)
        assert rho.shape == (s.n,) and np.all(np.isfinite(rho))


def _fast_jet(cell_factor, seed):
    """A jet stepped with a fixed dt so long that its free jet (speed 1) moves
    about twice half the cell skin within half a step; c0 = 3 keeps the step
    acoustically stable."""
    s = _jet(seed, nD=12)
    h = s.params["h"]
    s.params.update(cell_size=cell_factor * h, c0=3.0)
    skin = (1 if cell_factor > 2 else 2) * cell_factor * h - 2 * h
    s.params["dt_fixed"] = 2.0 * skin          # half step: displacement ~ skin > skin / 2
    return s


@pytest.mark.parametrize("cell_factor", [1.05, 2.2])
def test_half_step_outrunning_the_skin_is_rescanned_exactly(gpu, orc, cell_factor):
    s = _fast_jet(cell_factor, seed=10)
    say(f"[rescan] cell {cell_factor} h, dt_fixed {s.params['dt_fixed']:.4g}, n={s.n}")
    st = orc.State(s)
    with gpu.Simulation(s) as sim:
        sim.step(4)
        flags = int(sim.read("flags")[0])      # no instability: SPH_OK
        assert flags == 8                      # the rescan ran
        pos, vel, rho = sim.read("pos"), sim.read("vel"), sim.read("rho")
    st.step(4)
    dx = s.meta["dx"]
    vmax = np.abs(st.vel).max()
    assert np.abs(pos - st.pos).max() / dx <= 1e-4
    assert np.abs(vel - st.vel).max() / vmax <= 1e-4
    assert np.abs(rho - st.rho).max() / s.params["rho0"] <= 1e-4


def test_half_step_beyond_the_widest_rescan_is_flagged(gpu):
    s = _fast_jet(1.05, seed=11)
    s.params["dt_fixed"] = 6.0 * s.params["h"]   # half step ~ 3h: reach above 6 cells
    with gpu.Simulation(s) as sim:
        sim.step(1)
        with pytest.raises(native.SphError) as e:
            sim.read("pos")
        assert e.value.status == native.SPH_EUNSTABLE
        assert int(sim.read("flags", allow_unstable=True)[0]) & 4
        assert sim.read("pos", allow_unstable=True).shape == (s.n, 2)
