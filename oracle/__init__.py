"""FP64 CPU oracle for the SPH particle update (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the HIP library:
the C source beside this file is compiled with gcc into ``liborc.so`` and called
through ctypes with its own parameter struct.

Every array is in particle-id order; the functions take a workloads ``System``
or ``Batch`` (or raw arrays) and return plain numpy arrays.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def compile_source(src: str, out: str) -> str:
    """gcc the oracle source `src` into the shared library `out` (FP64, no FMA
    contraction, OpenMP)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-I", _HERE, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into liborc.so beside its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        compile_source(_SRC, _LIB)
    return _LIB


@contextlib.contextmanager
def using(path: str):
    """Route every function of this module to the oracle library at `path`
    for the duration of the block (the mutation tests load deliberately
    broken copies of the oracle this way)."""
    global _lib
    saved = _lib
    _lib = _declare(C.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


class Params(C.Structure):
    _fields_ = [
        ("kernel", C.c_int32), ("density", C.c_int32),
        ("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double), ("gamma", C.c_double),
        ("alpha", C.c_double), ("eta2_h2", C.c_double), ("sigma", C.c_double), ("eps_h", C.c_double),
        ("gravity", C.c_double * 2), ("courant", C.c_double), ("dt_fixed", C.c_double),
        ("box_lo", C.c_double * 2), ("box_hi", C.c_double * 2), ("cell_size", C.c_double),
        ("piston_dir", C.c_double * 2), ("piston_u", C.c_double), ("piston_amp", C.c_double),
        ("piston_omega", C.c_double),
        ("boundary", C.c_int32), ("gravity_plane", C.c_int32), ("wall_spacing", C.c_double),
        ("gravity_from", C.c_double),
    ]


class EvalOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in (
        "colour", "drho", "apv", "nrm", "nflag", "kappa", "asurf", "acc", "vsig", "nnb",
        "s_drho", "s_acc", "s_nrm", "dt_f", "dt_cv", "dt", "rho")]


def _params(d: Dict) -> Params:
    p = Params()
    p.kernel = int(d["kernel"])
    p.density = int(d.get("density", 0))
    p.boundary = int(d.get("boundary", 0))
    p.gravity_plane = int(d.get("gravity_plane", 0))
    p.wall_spacing = float(d.get("wall_spacing", 0.0))
    p.gravity_from = float(d.get("gravity_from", 0.0))
    for k in ("h", "rho0", "c0", "gamma", "alpha", "eta2_h2", "sigma", "eps_h", "courant",
              "dt_fixed", "cell_size", "piston_u", "piston_amp", "piston_omega"):
        setattr(p, k, float(d[k]))
    for k in ("gravity", "box_lo", "box_hi", "piston_dir"):
        arr = getattr(p, k)
        arr[0], arr[1] = float(d[k][0]), float(d[k][1])
    return p


def _declare(L):
    """Declare the C signatures of an oracle library handle."""
    vp = C.c_void_p
    L.orc_kernel_w.restype = C.c_double
    L.orc_kernel_w.argtypes = [C.c_int, C.c_double, C.c_double]
    L.orc_kernel_f.restype = C.c_double
    L.orc_kernel_f.argtypes = [C.c_int, C.c_double, C.c_double]
    L.orc_eos.argtypes = [vp, C.c_int64, vp, vp, vp]
    L.orc_grid.argtypes = [vp, vp, vp]
    L.orc_neighbors.restype = C.c_int64
    L.orc_neighbors.argtypes = [C.c_int, vp, vp, vp, vp, C.c_int, vp, vp, C.c_int64]
    L.orc_sort.argtypes = [C.c_int, vp, vp, vp, vp, vp, vp]
    L.orc_eval.argtypes = [C.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.orc_step.argtypes = [C.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int, vp]
    L.orc_breakup.argtypes = [C.c_int, vp, vp, vp, vp, vp, vp, C.c_double, vp, vp]
    L.orc_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_set_threads.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _declare(C.CDLL(_LIB))
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _wall_normals(obj):
    """The boundary particles' unit normals (meta["wall_normal"], n x 2) of a
    System or of every System of a Batch, or None if none carries them."""
    systems = obj.systems if hasattr(obj, "systems") else [obj]
    if not any("wall_normal" in s.meta for s in systems):
        return None
    return np.ascontiguousarray(np.concatenate(
        [s.meta.get("wall_normal", np.zeros((s.n, 2))) for s in systems]), dtype=np.float64)


def _unpack(obj):
    """Accept a workloads System or Batch; return (params list, offsets, arrays)."""
    if hasattr(obj, "systems"):
        plist = [s.params for s in obj.systems]
        off = obj.offsets
        pos, vel, rho, mass, typ = (obj.cat(f) for f in ("pos", "vel", "rho", "mass", "type"))
    else:
        plist = [obj.params]
        off = np.array([0, obj.n], dtype=np.int64)
        pos, vel, rho, mass, typ = obj.pos, obj.vel, obj.rho, obj.mass, obj.type
    arr = (np.ascontiguousarray(pos, dtype=np.float64), np.ascontiguousarray(vel, dtype=np.float64),
           np.ascontiguousarray(rho, dtype=np.float64), np.ascontiguousarray(mass, dtype=np.float64),
           np.ascontiguousarray(typ, dtype=np.int32))
    return plist, np.ascontiguousarray(off, dtype=np.int64), arr


def _param_array(plist: Sequence[Dict]):
    arr = (Params * len(plist))()
    for i, d in enumerate(plist):
        arr[i] = _params(d)
    return arr


def kernel_w(kernel: int, r: float, h: float) -> float:
    return lib().orc_kernel_w(int(kernel), float(r), float(h))


def kernel_f(kernel: int, r: float, h: float) -> float:
    return lib().orc_kernel_f(int(kernel), float(r), float(h))


def eos(params: Dict, rho: np.ndarray):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    P = np.empty_like(rho)
    c = np.empty_like(rho)
    p = _params(params)
    lib().orc_eos(C.byref(p), rho.size, _ptr(rho), _ptr(P), _ptr(c))
    return P, c


def grid(params: Dict):
    nx = np.zeros(1, dtype=np.int64)
    ny = np.zeros(1, dtype=np.int64)
    p = _params(params)
    lib().orc_grid(C.byref(p), _ptr(nx), _ptr(ny))
    return int(nx[0]), int(ny[0])


def neighbors(obj, brute: bool = False):
    """CSR neighbour lists (start[n+1], nbr) in id order, ascending ids."""
    plist, off, (pos, vel, rho, mass, typ) = _unpack(obj)
    n = int(off[-1])
    P = _param_array(plist)
    start = np.zeros(n + 1, dtype=np.int64)
    total = lib().orc_neighbors(len(plist), P, _ptr(off), _ptr(pos), _ptr(typ), int(brute),
                                _ptr(start), None, 0)
    nbr = np.zeros(max(total, 1), dtype=np.int32)
    lib().orc_neighbors(len(plist), P, _ptr(off), _ptr(pos), _ptr(typ), int(brute),
                        _ptr(start), _ptr(nbr), total)
    return start, nbr[:total]


def sort(obj):
    """(keys_sorted uint64, perm int64) ordered by (cell key, id)."""
    plist, off, (pos, vel, rho, mass, typ) = _unpack(obj)
    n = int(off[-1])
    keys = np.zeros(n, dtype=np.uint64)
    perm = np.zeros(n, dtype=np.int64)
    lib().orc_sort(len(plist), _param_array(plist), _ptr(off), _ptr(pos), _ptr(typ),
                   _ptr(keys), _ptr(perm))
    return keys, perm


def evaluate(obj) -> Dict[str, np.ndarray]:
    """Every right-hand side at the given state (see sph_oracle.h)."""
    plist, off, (pos, vel, rho, mass, typ) = _unpack(obj)
    n = int(off[-1])
    ns = len(plist)
    res = dict(
        colour=np.zeros(n), drho=np.zeros(n), apv=np.zeros((n, 2)), nrm=np.zeros((n, 2)),
        nflag=np.zeros(n, dtype=np.int32), kappa=np.zeros(n), asurf=np.zeros((n, 2)),
        acc=np.zeros((n, 2)), vsig=np.zeros(n), nnb=np.zeros(n, dtype=np.int32),
        s_drho=np.zeros(n), s_acc=np.zeros(n), s_nrm=np.zeros(n),
        dt_f=np.zeros(ns), dt_cv=np.zeros(ns), dt=np.zeros(ns), rho=np.zeros(n))
    out = EvalOut(**{k: _ptr(v).value if v is not None else None for k, v in res.items()})
    wn = _wall_normals(obj)
    lib().orc_eval(ns, _param_array(plist), _ptr(off), _ptr(pos), _ptr(vel), _ptr(rho),
                   _ptr(mass), _ptr(typ), _ptr(wn), C.byref(out))
    return res


def breakup(obj, xi_start, axis=(1.0, 0.0), gap_h: float = 1.5):
    """(length, broken) per system: the breakup criterion of Section 3-2 (see
    orc_breakup in sph_oracle.h). xi_start: the start coordinate along the axis
    (the nozzle exit), one per system or one for all."""
    plist, off, (pos, vel, rho, mass, typ) = _unpack(obj)
    ns = len(plist)
    ax = np.ascontiguousarray(axis, dtype=np.float64)
    xs = np.ascontiguousarray(np.broadcast_to(np.asarray(xi_start, dtype=np.float64), (ns,)))
    length = np.zeros(ns)
    broken = np.zeros(ns, dtype=np.int32)
    lib().orc_breakup(ns, _param_array(plist), _ptr(off), _ptr(pos), _ptr(typ), _ptr(ax), _ptr(xs),
                      float(gap_h), _ptr(length), _ptr(broken))
    return length, broken


class State:
    """Mutable FP64 state for multi-step oracle runs."""

    def __init__(self, obj):
        self.plist, self.off, (self.pos, self.vel, self.rho, self.mass, self.type) = _unpack(obj)
        self.pos = self.pos.copy(); self.vel = self.vel.copy(); self.rho = self.rho.copy()
        self.type = self.type.copy()
        self.time = np.zeros(len(self.plist))
        self.dt = np.zeros(len(self.plist))
        self._P = _param_array(self.plist)
        self.wall_normal = _wall_normals(obj)

    def step(self, nsteps: int = 1):
        lib().orc_step(len(self.plist), self._P, _ptr(self.off), _ptr(self.pos), _ptr(self.vel),
                       _ptr(self.rho), _ptr(self.mass), _ptr(self.type), _ptr(self.wall_normal),
                       _ptr(self.time), int(nsteps), _ptr(self.dt))
        return self


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Number of OpenMP threads for the following oracle calls."""
    lib().orc_set_threads(int(n))
