"""The C-ABI library builds for gfx950, loads, exports every entry point that
include/sph.h declares, and validates its arguments on the host (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sph.h")).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(sph_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_expected_entry_points():
    from paper_1603_02421_amd import native
    assert sorted(native.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_1603_02421_amd import native
    L = native.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.sph_abi_version() == 2


def _ws(params_list, n_list, **opt):
    from paper_1603_02421_amd import native
    L = native.load()
    P = (native.SphParams * len(params_list))()
    for i, d in enumerate(params_list):
        P[i] = native.params_struct(d)
    off = np.zeros(len(n_list) + 1, dtype=np.int64)
    off[1:] = np.cumsum(n_list)
    o = native.SphOptions()
    for k, v in opt.items():
        setattr(o, k, v)
    out = C.c_size_t(0)
    st = L.sph_workspace_bytes(C.byref(o), len(params_list), P, off.ctypes.data_as(C.c_void_p), C.byref(out))
    return st, out.value, L.sph_last_error(None).decode()


def test_workspace_bytes_scales_with_particles():
    s = wl.dam_break()
    st1, b1, _ = _ws([s.params], [s.n])
    st2, b2, _ = _ws([s.params], [4 * s.n])
    st3, b3, _ = _ws([s.params], [s.n], dtype_bits=64)
    assert st1 == st2 == st3 == 0
    assert b2 > b1 and b3 > b1
    assert b1 > 100 * s.n


@pytest.mark.parametrize("field,value,msg", [
    ("h", -1.0, "h must"), ("courant", 1.5, "courant"), ("cell_size", 0.5, "cell_size"),
    ("kernel", 7, "kernel"), ("c0", 0.0, "c0"),
])
def test_workspace_bytes_rejects_bad_parameters(field, value, msg):
    s = wl.dam_break()
    p = dict(s.params)
    if field == "cell_size":
        value = 0.5 * p["h"]
    p[field] = value
    st, _, err = _ws([p], [s.n])
    assert st == -1 and msg in err


def test_workspace_bytes_rejects_bad_options():
    s = wl.dam_break()
    assert _ws([s.params], [s.n], dtype_bits=16)[0] == -1
    assert _ws([s.params], [s.n], block_sweep=100)[0] == -1


def test_init_rejects_null_workspace_without_touching_the_gpu():
    from paper_1603_02421_amd import native
    L = native.load()
    s = wl.dam_break()
    P = (native.SphParams * 1)()
    P[0] = native.params_struct(s.params)
    off = np.array([0, s.n], dtype=np.int64)
    ctx = C.c_void_p()
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    st = L.sph_init(None, 1, P, vp(off), vp(s.pos), vp(s.vel), vp(s.rho), vp(s.mass), vp(s.type),
                    None, 0, None, C.byref(ctx))
    assert st == -1 and ctx.value is None


def test_trainer_workspace_and_argument_checks_without_the_gpu():
    from paper_1603_02421_amd import native
    L = native.load()
    out = C.c_size_t(0)
    assert L.sph_mlp_workspace_bytes(0, C.byref(out)) == -1
    sizes = []
    for m in (16, 4096, 16 * 1024, 16 * 1024 * 8):
        assert L.sph_mlp_workspace_bytes(m, C.byref(out)) == 0
        sizes.append(out.value)
    # the per-wave gradient partials grow with the batch up to 1024 waves, then stop
    assert sizes[0] < sizes[1] < sizes[2] == sizes[3]
    assert sizes[2] >= 1024 * native.MLP_NPARAMS * 4
    h = C.c_void_p()
    w = np.zeros(native.MLP_NPARAMS, dtype=np.float32)
    assert L.sph_mlp_create(None, 16, None, 0, None, C.byref(h)) == -1 and h.value is None
    assert L.sph_mlp_create(w.ctypes.data_as(C.c_void_p), 0, None, 0, None, C.byref(h)) == -1
    assert L.sph_mlp_gradient(None, None, None, 16, None, None) == -1
    assert L.sph_mlp_train_step(None, None, None, 16, C.c_float(1e-3), None) == -1
    assert L.sph_mlp_forward(None, None, 16, None) == -1
    assert "bad arguments" in L.sph_last_error(None).decode()


def test_static_init_rejects_systems_beyond_its_array_without_the_gpu():
    """sph_init_static checks the workspace the systems need against
    SPH_STATIC_WORKSPACE_BYTES on the host, before any device call."""
    from paper_1603_02421_amd import native
    L = native.load()
    s = wl.lattice_block(1500, 1000)            # 1.5M particles: several hundred MB
    P = (native.SphParams * 1)()
    P[0] = native.params_struct(s.params)
    off = np.array([0, s.n], dtype=np.int64)
    arrs = [np.ascontiguousarray(a) for a in (s.pos, s.vel, s.rho, s.mass, s.type.astype(np.int32))]
    out = C.c_void_p()
    st = L.sph_init_static(None, 1, P, off.ctypes.data_as(C.c_void_p),
                           *[a.ctypes.data_as(C.c_void_p) for a in arrs], None, C.byref(out))
    assert st == native.SPH_ENOMEM
    assert b"static workspace holds" in L.sph_last_error(None)
    assert out.value is None
