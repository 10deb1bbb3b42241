"""Python handle on a libsphjet context (argument marshalling only).

PyTorch supplies the device workspace and the stream; every step of the
particle update runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence

import numpy as np

from . import native

_VEC = {"pos", "vel", "accel", "normal"}
_WIDE = {"stencil": 64, "closure": 4}
_I32 = {"type", "nflag", "flags", "fallback"}
_I64 = {"nactive", "sort_perm"}
_U64 = {"sort_keys"}
_PER_SYS = {"dt", "time", "nactive"}


def _unpack(obj):
    if hasattr(obj, "systems"):
        plist = [s.params for s in obj.systems]
        off = obj.offsets
        arrs = [obj.cat(f) for f in ("pos", "vel", "rho", "mass", "type")]
    elif isinstance(obj, (list, tuple)):
        plist = [s.params for s in obj]
        off = np.zeros(len(obj) + 1, dtype=np.int64)
        off[1:] = np.cumsum([s.n for s in obj])
        arrs = [np.concatenate([getattr(s, f) for s in obj]) for f in ("pos", "vel", "rho", "mass", "type")]
    else:
        plist = [obj.params]
        off = np.array([0, obj.n], dtype=np.int64)
        arrs = [obj.pos, obj.vel, obj.rho, obj.mass, obj.type]
    pos, vel, rho, mass, typ = arrs
    return (plist, np.ascontiguousarray(off, dtype=np.int64),
            np.ascontiguousarray(pos, dtype=np.float64), np.ascontiguousarray(vel, dtype=np.float64),
            np.ascontiguousarray(rho, dtype=np.float64), np.ascontiguousarray(mass, dtype=np.float64),
            np.ascontiguousarray(typ, dtype=np.int32))


def _wall_normals(obj):
    """meta["wall_normal"] (n x 2) of a System, or of a Batch's systems."""
    systems = obj.systems if hasattr(obj, "systems") else (list(obj) if isinstance(obj, (list, tuple)) else [obj])
    if not any("wall_normal" in getattr(s, "meta", {}) for s in systems):
        return None
    return np.concatenate([s.meta.get("wall_normal", np.zeros((s.n, 2))) for s in systems])


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Simulation:
    """A set of particle systems resident on one GPU.

    systems: a workloads System, Batch or list of Systems (params dicts plus FP64
    host arrays). Options map to sph_options (dtype_bits, block_sweep,
    block_stream, use_graph, xcd_remap). static_workspace=True creates the
    context with sph_init_static (no device allocation; one per device).
    """

    def __init__(self, systems, dtype_bits: int = 32, block_sweep: int = 0, block_stream: int = 0,
                 use_graph: int = -1, xcd_remap: int = -1, graph_steps: int = 0, cell_factor: float = 0.0,
                 device: str = "cuda:0", stream=None, static_workspace: bool = False):
        import torch

        L = native.load()
        self._L = L
        plist, off, pos, vel, rho, mass, typ = _unpack(systems)
        if cell_factor > 0:
            plist = [dict(d, cell_size=cell_factor * d["h"]) for d in plist]
        self.n = int(off[-1])
        self.n_sys = len(plist)
        self.params = plist
        self.offsets = off
        P = (native.SphParams * self.n_sys)()
        for i, d in enumerate(plist):
            P[i] = native.params_struct(d)
        self._P = P
        opt = native.SphOptions()
        opt.dtype_bits, opt.block_sweep, opt.block_stream = dtype_bits, block_sweep, block_stream
        opt.use_graph, opt.xcd_remap, opt.graph_steps = use_graph, xcd_remap, graph_steps
        self._opt = opt
        self.dtype_bits = dtype_bits
        self.device = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        handle = C.c_void_p(stream.cuda_stream)
        ctx = C.c_void_p()
        if static_workspace:
            self.workspace_bytes = native.STATIC_WORKSPACE_BYTES
            self.workspace = None
            with torch.cuda.device(self.device):
                native.check(L.sph_init_static(C.byref(opt), self.n_sys, P, _ptr(off), _ptr(pos), _ptr(vel),
                                               _ptr(rho), _ptr(mass), _ptr(typ), handle, C.byref(ctx)))
        else:
            nbytes = C.c_size_t(0)
            native.check(L.sph_workspace_bytes(C.byref(opt), self.n_sys, P, _ptr(off), C.byref(nbytes)))
            self.workspace_bytes = int(nbytes.value)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            native.check(L.sph_init(C.byref(opt), self.n_sys, P, _ptr(off), _ptr(pos), _ptr(vel), _ptr(rho),
                                    _ptr(mass), _ptr(typ), C.c_void_p(self.workspace.data_ptr()),
                                    self.workspace_bytes, handle, C.byref(ctx)))
        self._ctx = ctx
        normals = _wall_normals(systems)
        if normals is not None and any(int(d.get("boundary", 0)) == 1 for d in plist):
            self.set_wall_normals(normals)

    def set_wall_normals(self, normals: np.ndarray) -> "Simulation":
        """Unit normals of the boundary particles of repulsive-force systems (n x 2)."""
        w = np.ascontiguousarray(normals, dtype=np.float64)
        assert w.shape == (self.n, 2)
        native.check(self._L.sph_set_wall_normals(self._ctx, _ptr(w)), self._ctx)
        return self

    # -- stepping -------------------------------------------------------
    def step(self, n: int = 1) -> "Simulation":
        native.check(self._L.sph_step(self._ctx, int(n)), self._ctx)
        return self

    def evaluate(self) -> "Simulation":
        native.check(self._L.sph_evaluate(self._ctx), self._ctx)
        return self

    def sync(self):
        native.check(self._L.sph_sync(self._ctx), self._ctx)

    # -- reading --------------------------------------------------------
    def read(self, field: str, allow_unstable: bool = False) -> np.ndarray:
        fid = native.FIELDS[field]
        if field in _PER_SYS:
            count = self.n_sys
        elif field == "flags":
            count = 1
        else:
            count = self.n
        if field in _VEC:
            out = np.zeros((count, 2), dtype=np.float64)
        elif field in _WIDE:
            out = np.zeros((count, _WIDE[field]), dtype=np.float64)
        elif field in _I32:
            out = np.zeros(count, dtype=np.int32)
        elif field in _I64:
            out = np.zeros(count, dtype=np.int64)
        elif field in _U64:
            out = np.zeros(count, dtype=np.uint64)
        else:
            out = np.zeros(count, dtype=np.float64)
        st = self._L.sph_read(self._ctx, fid, _ptr(out), out.nbytes)
        if not (allow_unstable and st == native.SPH_EUNSTABLE):
            native.check(st, self._ctx)
        return out

    def checkpoint(self, allow_unstable: bool = False) -> bytes:
        """The state blob (sph_read of SPH_F_ALL_STATE)."""
        nbytes = C.c_size_t(0)
        native.check(self._L.sph_state_bytes(self._ctx, C.byref(nbytes)), self._ctx)
        buf = np.zeros(int(nbytes.value), dtype=np.uint8)
        st = self._L.sph_read(self._ctx, native.FIELDS["all_state"], _ptr(buf), buf.nbytes)
        if not (allow_unstable and st == native.SPH_EUNSTABLE):
            native.check(st, self._ctx)
        return buf.tobytes()

    def restore(self, blob: bytes) -> "Simulation":
        """Load a state blob from checkpoint() (sph_restore)."""
        buf = np.frombuffer(blob, dtype=np.uint8)
        native.check(self._L.sph_restore(self._ctx, _ptr(buf), buf.nbytes), self._ctx)
        return self

    def breakup(self, xi_start, axis=(1.0, 0.0), gap_h: float = 1.5):
        """(length, broken) per system: the breakup criterion (sph_breakup)."""
        ax = np.ascontiguousarray(axis, dtype=np.float64)
        xs = np.ascontiguousarray(np.broadcast_to(np.asarray(xi_start, dtype=np.float64), (self.n_sys,)))
        length = np.zeros(self.n_sys)
        broken = np.zeros(self.n_sys, dtype=np.int32)
        native.check(self._L.sph_breakup(self._ctx, _ptr(ax), _ptr(xs), float(gap_h), _ptr(length), _ptr(broken)),
                     self._ctx)
        return length, broken

    def read_all(self, fields: Sequence[str] = ("pos", "vel", "rho", "type")) -> Dict[str, np.ndarray]:
        return {f: self.read(f) for f in fields}

    def neighbors(self):
        """CSR neighbour lists at the current state, in id order (ascending ids)."""
        start = np.zeros(self.n + 1, dtype=np.int64)
        total = C.c_int64(0)
        st = self._L.sph_neighbors(self._ctx, _ptr(start), None, 0, C.byref(total))
        if st not in (native.SPH_OK, native.SPH_ECAPACITY):
            native.check(st, self._ctx)
        nbr = np.zeros(max(int(total.value), 1), dtype=np.int32)
        native.check(self._L.sph_neighbors(self._ctx, _ptr(start), _ptr(nbr), nbr.size, C.byref(total)),
                     self._ctx)
        return start, nbr[: int(total.value)]

    def set_closure(self, params: np.ndarray) -> "Simulation":
        """Install closure network parameters (flat FP32, SPH_MLP_NPARAMS)."""
        w = np.ascontiguousarray(params, dtype=np.float32)
        assert w.size == native.MLP_NPARAMS
        native.check(self._L.sph_set_closure(self._ctx, _ptr(w)), self._ctx)
        return self

    def profile(self, n_steps: int) -> Dict[str, Dict[str, float]]:
        """Per-kernel average time (ms) over n_steps eager steps (advances the state)."""
        maxk = 64
        names = (C.c_char_p * maxk)()
        avg = np.zeros(maxk, dtype=np.float64)
        calls = np.zeros(maxk, dtype=np.int64)
        nk = C.c_int32(0)
        native.check(self._L.sph_profile(self._ctx, int(n_steps), maxk, names, _ptr(avg), _ptr(calls),
                                         C.byref(nk)), self._ctx)
        return {names[i].decode(): dict(avg_ms=float(avg[i]), calls=int(calls[i]))
                for i in range(min(nk.value, maxk))}

    def close(self):
        if getattr(self, "_ctx", None):
            self._L.sph_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def autotune(systems, dtype_bits: int = 32, trial_steps: int = 5, device: str = "cuda:0", stream=None,
             **opts) -> Dict:
    """Time the candidate cell sizes and sweep block shapes on a copy of the
    initial state (sph_autotune) and return the winner."""
    import torch

    L = native.load()
    plist, off, pos, vel, rho, mass, typ = _unpack(systems)
    n_sys = len(plist)
    opt = native.SphOptions()
    opt.dtype_bits = dtype_bits
    for k, v in opts.items():
        setattr(opt, k, v)
    fine = (native.SphParams * n_sys)()
    P = (native.SphParams * n_sys)()
    for i, d in enumerate(plist):
        P[i] = native.params_struct(d)
        fine[i] = native.params_struct(dict(d, cell_size=1.05 * d["h"]))
    nbytes = C.c_size_t(0)
    native.check(L.sph_workspace_bytes(C.byref(opt), n_sys, fine, _ptr(off), C.byref(nbytes)))
    dev = torch.device(device)
    ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    res = native.SphTuneResult()
    native.check(L.sph_autotune(C.byref(opt), n_sys, P, _ptr(off), _ptr(pos), _ptr(vel), _ptr(rho), _ptr(mass),
                                _ptr(typ), C.c_void_p(ws.data_ptr()), int(nbytes.value),
                                C.c_void_p(stream.cuda_stream), int(trial_steps), C.byref(res)))
    del ws
    return dict(cell_factor=res.cell_factor, block_sweep=res.block_sweep, ms_per_step=res.ms_per_step,
                n_tried=res.n_tried, from_cache=bool(res.from_cache))
