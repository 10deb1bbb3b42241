"""ctypes declarations of libsphjet's C-ABI (include/sph.h).

The shared library is built in-tree (``python -m paper_1603_02421_amd.build``)
into ``paper_1603_02421_amd/lib/libsphjet.so``. There is no fallback: if the
library is missing, :func:`load` raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsphjet.so")

SPH_OK, SPH_EINVAL, SPH_ENOMEM, SPH_EDEVICE, SPH_EUNSTABLE, SPH_ECAPACITY, SPH_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SPH_OK", -1: "SPH_EINVAL", -2: "SPH_ENOMEM", -3: "SPH_EDEVICE", -4: "SPH_EUNSTABLE",
                -5: "SPH_ECAPACITY", -6: "SPH_ESTATE"}

FIELDS = {
    "pos": 0, "vel": 1, "rho": 2, "pressure": 3, "mass": 4, "type": 5, "drhodt": 6, "accel": 7,
    "colour": 8, "normal": 9, "curv": 10, "nflag": 11, "dt": 12, "time": 13, "nactive": 14,
    "sort_keys": 15, "sort_perm": 16, "flags": 17, "curv_plain": 18, "stencil": 19, "closure": 20,
    "fallback": 21, "all_state": 22,
}
MLP_NPARAMS = 8515
STATIC_WORKSPACE_BYTES = 128 << 20   # SPH_STATIC_WORKSPACE_BYTES

# Exported entry points, as declared in include/sph.h.
EXPORTS = [
    "sph_workspace_bytes", "sph_init", "sph_init_static", "sph_step", "sph_evaluate", "sph_read", "sph_neighbors",
    "sph_sync", "sph_profile", "sph_autotune", "sph_state_bytes", "sph_restore", "sph_breakup",
    "sph_set_wall_normals", "sph_free", "sph_last_error", "sph_abi_version",
    "sph_set_closure", "sph_mlp_workspace_bytes", "sph_mlp_create", "sph_mlp_forward", "sph_mlp_gradient",
    "sph_mlp_train_step", "sph_mlp_params", "sph_mlp_free",
]


class SphParams(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32), ("closure", C.c_int32),
        ("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double), ("gamma", C.c_double),
        ("alpha", C.c_double), ("eta2_h2", C.c_double), ("sigma", C.c_double), ("eps_h", C.c_double),
        ("gravity", C.c_double * 2), ("courant", C.c_double), ("dt_fixed", C.c_double),
        ("box_lo", C.c_double * 2), ("box_hi", C.c_double * 2), ("cell_size", C.c_double),
        ("piston_dir", C.c_double * 2), ("piston_u", C.c_double), ("piston_amp", C.c_double),
        ("piston_omega", C.c_double), ("closure_tol", C.c_double),
        ("density", C.c_int32), ("boundary", C.c_int32), ("wall_spacing", C.c_double),
        ("gravity_plane", C.c_int32), ("pad_", C.c_int32), ("gravity_from", C.c_double),
    ]


class SphOptions(C.Structure):
    _fields_ = [
        ("dtype_bits", C.c_int32), ("block_sweep", C.c_int32), ("block_stream", C.c_int32),
        ("use_graph", C.c_int32), ("xcd_remap", C.c_int32), ("graph_steps", C.c_int32),
        ("reserved", C.c_int32 * 2),
    ]


class SphTuneResult(C.Structure):
    _fields_ = [
        ("cell_factor", C.c_double), ("block_sweep", C.c_int32), ("n_tried", C.c_int32),
        ("ms_per_step", C.c_double), ("from_cache", C.c_int32), ("pad_", C.c_int32),
    ]


_lib = None


class SphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libsphjet.so from the package tree; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsphjet.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_1603_02421_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    L.sph_workspace_bytes.argtypes = [vp, i32, vp, vp, C.POINTER(sz)]
    L.sph_init.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, C.POINTER(vp)]
    L.sph_init_static.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.sph_step.argtypes = [vp, i32]
    L.sph_evaluate.argtypes = [vp]
    L.sph_read.argtypes = [vp, i32, vp, sz]
    L.sph_neighbors.argtypes = [vp, vp, vp, i64, C.POINTER(i64)]
    L.sph_sync.argtypes = [vp]
    L.sph_state_bytes.argtypes = [vp, C.POINTER(sz)]
    L.sph_restore.argtypes = [vp, vp, sz]
    L.sph_breakup.argtypes = [vp, vp, vp, C.c_double, vp, vp]
    L.sph_set_wall_normals.argtypes = [vp, vp]
    L.sph_profile.argtypes = [vp, i32, i32, C.POINTER(C.c_char_p), vp, vp, C.POINTER(i32)]
    L.sph_autotune.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, i32, vp]
    L.sph_free.argtypes = [vp]
    L.sph_free.restype = None
    L.sph_set_closure.argtypes = [vp, vp]
    L.sph_mlp_workspace_bytes.argtypes = [i64, C.POINTER(sz)]
    L.sph_mlp_create.argtypes = [vp, i64, vp, sz, vp, C.POINTER(vp)]
    L.sph_mlp_forward.argtypes = [vp, vp, i64, vp]
    L.sph_mlp_gradient.argtypes = [vp, vp, vp, i64, vp, vp]
    L.sph_mlp_train_step.argtypes = [vp, vp, vp, i64, C.c_float, vp]
    L.sph_mlp_params.argtypes = [vp, vp]
    L.sph_mlp_free.argtypes = [vp]
    L.sph_mlp_free.restype = None
    L.sph_last_error.argtypes = [vp]
    L.sph_last_error.restype = C.c_char_p
    L.sph_abi_version.restype = i32
    for name in ("sph_workspace_bytes", "sph_init", "sph_init_static", "sph_step", "sph_evaluate", "sph_read",
                 "sph_neighbors", "sph_sync", "sph_profile", "sph_autotune", "sph_set_closure",
                 "sph_state_bytes", "sph_restore", "sph_breakup", "sph_set_wall_normals",
                 "sph_mlp_workspace_bytes", "sph_mlp_create", "sph_mlp_forward", "sph_mlp_gradient",
                 "sph_mlp_train_step", "sph_mlp_params"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def check(status: int, ctx=None):
    if status != SPH_OK:
        msg = load().sph_last_error(ctx).decode(errors="replace")
        raise SphError(status, msg)


def params_struct(d) -> SphParams:
    p = SphParams()
    p.kernel = int(d["kernel"])
    p.closure = int(d.get("closure", 0))
    for k in ("h", "rho0", "c0", "gamma", "alpha", "eta2_h2", "sigma", "eps_h", "courant",
              "dt_fixed", "cell_size", "piston_u", "piston_amp", "piston_omega"):
        setattr(p, k, float(d[k]))
    p.closure_tol = float(d.get("closure_tol", 0.2))
    p.density = int(d.get("density", 0))
    p.boundary = int(d.get("boundary", 0))
    p.wall_spacing = float(d.get("wall_spacing", 0.0))
    p.gravity_plane = int(d.get("gravity_plane", 0))
    p.gravity_from = float(d.get("gravity_from", 0.0))
    for k in ("gravity", "box_lo", "box_hi", "piston_dir"):
        arr = getattr(p, k)
        arr[0], arr[1] = float(d[k][0]), float(d[k][1])
    return p
