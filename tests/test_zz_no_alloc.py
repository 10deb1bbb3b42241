"""sph_init_static, the entry point for callers that cannot allocate device
memory, against sph_init on a caller-supplied workspace: the same systems give
the same results bit for bit (same kernels, same launch shapes), on two
contexts in a row, the second smaller than the first, from the one static
array of the device."""
import numpy as np
import pytest

import workloads as wl
from paper_1603_02421_amd import native

pytestmark = pytest.mark.gpu

EVAL = ("colour", "drhodt", "accel", "normal", "curv", "nflag", "dt")
STATE = ("pos", "vel", "rho", "type", "time", "dt")


def say(*a):
    print(*a, flush=True)


def _run(sph, obj, static, steps):
    out = {}
    with sph.Simulation(obj, dtype_bits=32, use_graph=0, static_workspace=static) as sim:
        sim.evaluate()
        out.update({"eval_" + f: sim.read(f) for f in EVAL})
        sim.step(steps)
        out.update({"step_" + f: sim.read(f) for f in STATE})
    return out


def test_static_workspace_matches_caller_workspace(gpu):
    big = wl.round_for_dtype(wl.jet(n_target=30_000, nD=14, Re=400, We=15, seed=11, free_length=12.0,
                                    prefill=6.0), 32)
    small = wl.round_for_dtype(wl.jet(n_target=7_000, nD=10, Re=800, We=25, seed=12, kernel=wl.CUBIC,
                                      free_length=6.0, prefill=3.0), 32)
    for name, obj in (("big", big), ("small", small)):
        say(f"[no-alloc] case={name} n={obj.n}")
        ref = _run(gpu, obj, False, 5)
        got = _run(gpu, obj, True, 5)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), f"{name}: {k} differs"


def test_one_static_context_per_device(gpu):
    a = wl.round_for_dtype(wl.lattice_block(20, 20), 32)
    say("[no-alloc] second context while the first holds the array")
    with gpu.Simulation(a, static_workspace=True) as sim:
        sim.step(2)
        with pytest.raises(native.SphError) as e:
            gpu.Simulation(a, static_workspace=True)
        assert e.value.status == native.SPH_ESTATE
        pos = sim.read("pos")
    # freed: the array is available again, and a new context starts clean
    with gpu.Simulation(a, static_workspace=True) as sim2:
        sim2.step(2)
        assert np.array_equal(sim2.read("pos"), pos)
