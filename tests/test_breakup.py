"""The breakup criterion of Section 3-2 (a gap of more than 1.5h between two
particles consecutive along the jet) in the oracle, on particle sets whose
answer is known by construction; the same sets, and jets, check the HIP
detector bit for bit (tests marked gpu)."""
import numpy as np
import pytest

import workloads as wl
from workloads import scenarios

GAP = 1.5


def _row(xs, ys=None, h=1.3, types=None):
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.zeros_like(xs) if ys is None else np.asarray(ys, dtype=np.float64)
    pos = np.stack([xs, ys], axis=1)
    p = scenarios.default_params(h, 1.0, 10.0, box_lo=(-50.0, -50.0), box_hi=(400.0, 50.0))
    s = scenarios._assemble(p, [(pos, (0.0, 0.0), 1.0, wl.FLUID)])
    if types is not None:
        s.type[:] = types
    return s


def _strip(nx, ny, cut=None):
    """A lattice strip along x (ny particles across), optionally with the columns
    in [cut[0], cut[1]) removed."""
    s = wl.lattice_block(nx, ny, dx=1.0)
    if cut is not None:
        keep = ~((s.pos[:, 0] >= cut[0]) & (s.pos[:, 0] < cut[1]))
        s = scenarios._assemble(s.params, [(s.pos[keep], (0.0, 0.0), 1.0, wl.FLUID)])
    return s


def cases():
    h = 1.3
    d = GAP * h
    line = np.arange(40, dtype=np.float64)
    return {
        # (system, xi_start, axis, expected length, expected broken)
        "intact": (_row(line), 0.0, (1.0, 0.0), 39.0, 0),
        "one_gap": (_row(np.r_[line[:11], line[11:] + 2.0]), 0.0, (1.0, 0.0), 10.0, 1),
        "gap_exactly_1.5h": (_row(np.r_[0.0, d, d + 1.0]), 0.0, (1.0, 0.0), d + 1.0, 0),
        "gap_just_above": (_row(np.r_[0.0, np.nextafter(d, 10.0), d + 1.0]), 0.0, (1.0, 0.0), 0.0, 1),
        "two_gaps_first_counts": (_row(np.r_[0.0, 1.0, 5.0, 6.0, 11.0]), 0.0, (1.0, 0.0), 1.0, 1),
        "gap_before_start": (_row(np.r_[-10.0, -9.0, 0.0, 1.0, 2.0]), -0.5, (1.0, 0.0), 2.5, 0),
        "wall_does_not_bridge": (_row(np.r_[0.0, 1.0, 2.5, 4.0, 5.0], types=[0, 0, 1, 0, 0]), 0.0, (1.0, 0.0),
                                 1.0, 1),
        "unsorted_input": (_row(np.r_[6.0, 0.0, 2.0, 1.0, 3.0]), 0.0, (1.0, 0.0), 3.0, 1),
        "nothing_beyond_start": (_row(np.r_[0.0, 1.0]), 5.0, (1.0, 0.0), 0.0, 0),
        "along_y": (_row(np.zeros(6), ys=np.r_[0.0, 1.0, 2.0, 6.0, 7.0, 8.0]), 0.0, (0.0, 1.0), 2.0, 1),
        "strip_intact": (_strip(60, 5), 0.0, (1.0, 0.0), 59.5, 0),
        "strip_cut": (_strip(60, 5, cut=(30.0, 33.0)), 0.0, (1.0, 0.0), 29.5, 1),
        "strip_one_column_out": (_strip(60, 5, cut=(30.0, 31.0)), 0.0, (1.0, 0.0), 29.5, 1),   # gap 2.0 > 1.95
    }


@pytest.mark.parametrize("name", list(cases()))
def test_oracle_breakup_known_answers(orc, name):
    s, start, axis, want, brk = cases()[name]
    length, broken = orc.breakup(s, start, axis=axis, gap_h=GAP)
    assert broken[0] == brk
    assert length[0] == pytest.approx(want, abs=1e-12)


def test_oracle_breakup_per_system(orc):
    c = cases()
    batch = wl.Batch([c["one_gap"][0], c["intact"][0], c["gap_before_start"][0]])
    length, broken = orc.breakup(batch, [0.0, 0.0, -0.5], gap_h=GAP)
    assert list(broken) == [1, 0, 0]
    assert np.allclose(length, [10.0, 39.0, 2.5])


# ---------------------------------------------------------------- GPU detector

def _gpu_breakup(gpu, obj, start, axis=(1.0, 0.0), steps=0):
    with gpu.Simulation(obj, dtype_bits=32) as sim:
        if steps:
            sim.step(steps)
        length, broken = sim.breakup(start, axis=axis, gap_h=GAP)
        pos, typ = sim.read("pos", allow_unstable=True), sim.read("type", allow_unstable=True)
    return length, broken, pos, typ


def _with_state(obj, pos, typ):
    """obj with the positions and types a GPU run reached."""
    if hasattr(obj, "systems"):
        out = wl.Batch([sy.copy() for sy in obj.systems])
        off = out.offsets
        for k, sy in enumerate(out.systems):
            sy.pos, sy.type = pos[off[k]:off[k + 1]].copy(), typ[off[k]:off[k + 1]].copy()
        return out
    out = obj.copy()
    out.pos, out.type = pos, typ
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(cases()))
def test_gpu_breakup_known_answers(gpu, orc, name):
    s, start, axis, want, brk = cases()[name]
    s = wl.round_for_dtype(s, 32)
    print(f"[breakup] case={name} n={s.n}", flush=True)
    length, broken, _, _ = _gpu_breakup(gpu, s, start, axis)
    o_len, o_brk = orc.breakup(s, start, axis=axis, gap_h=GAP)
    assert broken[0] == o_brk[0] == brk
    assert length[0] == o_len[0]                  # bit for bit
    assert length[0] == pytest.approx(want, abs=1e-12)


@pytest.mark.gpu
@pytest.mark.parametrize("steps", [0, 40])
def test_gpu_breakup_on_jets_bit_exact(gpu, orc, steps):
    """A batch of jets (with a few fluid particles moved downstream, so that
    some are broken) after `steps` steps: the GPU detector and the oracle's
    sort agree bit for bit at the state the GPU reached."""
    jets = [wl.round_for_dtype(wl.jet(n_target=6_000 + 1_000 * k, nD=10 + k, Re=300, We=10, seed=20 + k,
                                      free_length=10.0, prefill=5.0), 32) for k in range(4)]
    for k, j in enumerate(jets[:2]):               # detached drops beyond a gap
        tip = np.argmax(np.where(j.type == wl.FLUID, j.pos[:, 0], -np.inf))
        j.pos[tip, 0] += 0.6 + 0.2 * k
    batch = wl.Batch(jets)
    starts = np.array([j.meta["exit"] for j in jets])
    print(f"[breakup] jets n={batch.n} steps={steps}", flush=True)
    length, broken, pos, typ = _gpu_breakup(gpu, batch, starts, steps=steps)
    o_len, o_brk = orc.breakup(_with_state(batch, pos, typ), starts, gap_h=GAP)
    assert np.array_equal(broken, o_brk)
    assert np.array_equal(length, o_len)
    assert broken[:2].all()
