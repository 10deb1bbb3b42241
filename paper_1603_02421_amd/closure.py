"""Learned curvature closure: training data, training loop and accuracy.

The network and its kernels live in the library (sph_mlp_* and the closure
path of the particle update, include/sph.h); this module marshals data:

* training stencils come from the library's own stencil kernel, run on
  particle sets whose interface is known: discs (radius 3-50 dx) and
  sinusoidal interfaces (amplitude 0.5-5 dx, wavelength 10-60 dx), on a
  jittered lattice and randomly rotated, labelled with the exact unit normal
  and curvature; and jet snapshots subsampled from a run at 4x resolution,
  labelled with that run's plain estimate (eq. 18-23) at the kept particles;
* targets are (n_x, n_y, kappa h) with the normal pointing into the liquid
  (the direction of grad C) and kappa = div n_hat (negative on a convex
  liquid surface);
* training runs sph_mlp_train_step (forward, backward and Adam on the GPU).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Tuple

import numpy as np

from . import native

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "closure_weights.npz")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Trainer:
    """Device-resident closure network with its Adam state (sph_mlp_*)."""

    def __init__(self, params: np.ndarray, max_batch: int, device: str = "cuda:0", stream=None):
        import torch
        self.torch = torch
        L = native.load()
        self._L = L
        self.max_batch = int(max_batch)
        nbytes = C.c_size_t(0)
        native.check(L.sph_mlp_workspace_bytes(self.max_batch, C.byref(nbytes)))
        self.device = torch.device(device)
        self.ws = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        w = np.ascontiguousarray(params, dtype=np.float32)
        h = C.c_void_p()
        native.check(L.sph_mlp_create(w.ctypes.data_as(C.c_void_p), self.max_batch, _ptr(self.ws),
                                      int(nbytes.value), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.loss_dev = torch.zeros(4, dtype=torch.float32, device=self.device)

    def forward(self, X):
        torch = self.torch
        Y = torch.empty((X.shape[0], 3), dtype=torch.float32, device=self.device)
        native.check(self._L.sph_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(Y)))
        return Y

    def gradient(self, X, T):
        torch = self.torch
        g = torch.empty(native.MLP_NPARAMS, dtype=torch.float32, device=self.device)
        native.check(self._L.sph_mlp_gradient(self._h, _ptr(X), _ptr(T), X.shape[0], _ptr(g), _ptr(self.loss_dev)))
        return g, self.loss_dev[0]

    def step(self, X, T, lr: float):
        native.check(self._L.sph_mlp_train_step(self._h, _ptr(X), _ptr(T), X.shape[0], float(lr),
                                                _ptr(self.loss_dev)))
        return self.loss_dev[0]

    def params(self) -> np.ndarray:
        w = np.zeros(native.MLP_NPARAMS, dtype=np.float32)
        native.check(self._L.sph_mlp_params(self._h, w.ctypes.data_as(C.c_void_p)))
        return w

    def close(self):
        if getattr(self, "_h", None):
            self._L.sph_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def xavier_params(seed: int = 0) -> np.ndarray:
    """Seeded Xavier-uniform weights, zero biases, in the flat layout of sph.h."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def xav(fi, fo):
        lim = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-lim, lim, size=(fi, fo))

    parts = [xav(64, 64).ravel(), np.zeros(64), xav(64, 64).ravel(), np.zeros(64), xav(64, 3).ravel(), np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)


# ----------------------------------------------------------------- data

def _rotate(xy, th, c=(0.0, 0.0)):
    cs, sn = math.cos(th), math.sin(th)
    R = np.array([[cs, -sn], [sn, cs]])
    return (xy - c) @ R.T


def _jittered_lattice(x0, y0, nx, ny, dx, jitter, rng):
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    p = np.stack([x0 + (i.ravel() + 0.5) * dx, y0 + (j.ravel() + 0.5) * dx], axis=1)
    if jitter > 0:
        p = p + rng.uniform(-jitter * dx, jitter * dx, size=p.shape)
    return p


def shape_systems(n_shapes: int, seed: int, dx: float = 1.0):
    """Discs and sinusoidal slabs with their exact interface geometry.

    Returns (systems, label functions): label(pos) -> (n_hat (k, 2), kappa (k,),
    keep mask (k,)) in the system's own coordinates."""
    import workloads as wl
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_shapes):
        jitter = float(rng.choice([0.0, 0.05, 0.1, 0.2]))
        th = float(rng.uniform(0, 2 * math.pi))
        if k % 2 == 0:
            R = float(rng.uniform(3.0, 50.0))
            n = int(math.ceil(R / dx)) + 1
            p = _jittered_lattice(-n * dx, -n * dx, 2 * n, 2 * n, dx, jitter, rng)
            p = p[np.hypot(p[:, 0], p[:, 1]) < R]

            def label(q, R=R):
                r = np.hypot(q[:, 0], q[:, 1])
                nh = -q / np.maximum(r, 1e-12)[:, None]
                return nh, np.full(len(q), -1.0 / R), r > R - 3.0 * dx
        else:
            A = float(rng.uniform(0.5, 5.0)) * dx
            lam = float(rng.uniform(10.0, 60.0)) * dx
            kk = 2 * math.pi / lam
            L = 4 * lam
            depth = 10.0 * dx
            base = _jittered_lattice(0.0, -depth - A, int(L / dx), int((depth + 2 * A) / dx) + 2, dx, jitter, rng)
            p = base[base[:, 1] < A * np.sin(kk * base[:, 0])]

            def label(q, A=A, kk=kk, lam=lam, dx=dx):
                x = q[:, 0]
                s = A * kk * np.cos(kk * x)
                den = np.sqrt(1 + s * s)
                nh = np.stack([s / den, -1.0 / den], axis=1)
                kap = -A * kk * kk * np.sin(kk * x) / den ** 3
                keep = (x > lam) & (x < 3 * lam) & (np.abs(q[:, 1] - A * np.sin(kk * x)) < 3.0 * dx)
                return nh, kap, keep
        # rotate the particle set; labels are evaluated in the unrotated frame
        sysm = wl.scenarios._assemble(wl.scenarios.default_params(1.3 * dx, 1.0, 10.0, sigma=1.0, alpha=0.05,
                                                                   closure=1),
                                      [(_rotate(p, th), (0.0, 0.0), 1.0, wl.FLUID)])
        lo = sysm.pos.min(0) - 4 * dx
        hi = sysm.pos.max(0) + 4 * dx
        sysm.params.update(box_lo=tuple(lo), box_hi=tuple(hi), cell_size=2.2 * 1.3 * dx)
        sysm.meta = dict(theta=th, label=label)
        out.append(sysm)
    return out


def harvest(systems, device="cuda:0", chunk_particles: int = 1_500_000):
    """Run the closure's stencil kernel on the systems (GPU) and return, for
    every listed particle, (stencil, target (n_x, n_y, kappa h), plain kappa h)."""
    from .sim import Simulation
    X, T, P = [], [], []
    i = 0
    while i < len(systems):
        grp, n = [], 0
        while i < len(systems) and (n + systems[i].n <= chunk_particles or not grp):
            grp.append(systems[i])
            n += systems[i].n
            i += 1
        with Simulation(grp, dtype_bits=32, device=device) as sim:
            sim.evaluate()
            st = sim.read("stencil")
            listed = np.any(st != 0, axis=1)
            kplain = sim.read("curv_plain")
            pos = sim.read("pos")
        o = 0
        for s in grp:
            sl = slice(o, o + s.n)
            o += s.n
            h = s.params["h"]
            th = s.meta["theta"]
            q = _rotate(pos[sl], -th)
            nh, kap, keep = s.meta["label"](q)
            m = listed[sl] & keep
            nh_rot = _rotate(nh, th)
            X.append(st[sl][m])
            T.append(np.concatenate([nh_rot[m], (kap[m] * h)[:, None]], axis=1))
            P.append(kplain[sl][m] * h)
    return np.concatenate(X), np.concatenate(T), np.concatenate(P)


def poisson_subsample(pos: np.ndarray, rmin: float, seed: int) -> np.ndarray:
    """Indices of a greedy Poisson-disk subset: visited in seeded random order,
    a point is kept when no kept point lies closer than rmin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(pos))
    cs = rmin / math.sqrt(2.0)
    lo = pos.min(0)
    grid: Dict[Tuple[int, int], int] = {}
    kept = []
    r2 = rmin * rmin
    for i in order:
        gx, gy = int((pos[i, 0] - lo[0]) / cs), int((pos[i, 1] - lo[1]) / cs)
        ok = True
        for ax in range(gx - 2, gx + 3):
            for ay in range(gy - 2, gy + 3):
                j = grid.get((ax, ay))
                if j is not None:
                    d = pos[j] - pos[i]
                    if d[0] * d[0] + d[1] * d[1] < r2:
                        ok = False
                        break
            if not ok:
                break
        if ok:
            grid[(gx, gy)] = i
            kept.append(i)
    return np.array(sorted(kept), dtype=np.int64)


def jet_harvest(nD_coarse: int = 10, seeds=(0,), steps: int = 300, n_fine: int = 300_000, Re: float = 500.0,
                We: float = 20.0, window: float = 25.0, device="cuda:0"):
    """Jet neighbourhoods at resolution D/nD_coarse labelled by the plain
    estimate of a run at 4x resolution (D/(4 nD_coarse)).

    The fine jet runs `steps` steps; its particles within `window` D of the
    orifice are Poisson-disk subsampled to the coarse spacing and re-evaluated
    at the coarse h. Targets: the fine run's unit normal and curvature at the
    kept particles that the fine run also filtered as interface (N = 1)."""
    import workloads as wl
    from .sim import Simulation
    Xs, Ts, Ps = [], [], []
    for seed in seeds:
        fine = wl.round_for_dtype(wl.jet(n_target=n_fine, nD=4 * nD_coarse, Re=Re, We=We, seed=seed,
                                         free_length=window + 5.0, prefill=window), 32)
        with Simulation(fine, dtype_bits=32, device=device) as sim:
            sim.step(steps)
            sim.evaluate()
            pos = sim.read("pos")
            typ = sim.read("type")
            nrm = sim.read("normal")
            kap = sim.read("curv")
            nfl = sim.read("nflag")
        dxc = 1.0 / nD_coarse
        region = (typ != wl.INACTIVE) & (pos[:, 0] > -2.0) & (pos[:, 0] < window)
        idx = np.nonzero(region)[0]
        keep = idx[poisson_subsample(pos[idx], 1.05 * dxc, seed)]
        hc = 1.3 * dxc
        p = wl.scenarios.jet_params(nD_coarse, Re, We)
        p.update(closure=1, box_lo=tuple(pos[keep].min(0) - 4 * dxc), box_hi=tuple(pos[keep].max(0) + 4 * dxc),
                 cell_size=2.2 * hc)
        coarse = wl.System(p, pos[keep].copy(), np.zeros((len(keep), 2)), np.ones(len(keep)),
                           np.full(len(keep), dxc * dxc), typ[keep].astype(np.int32).copy(), name="jet_coarse")
        with Simulation(coarse, dtype_bits=32, device=device) as sim:
            sim.evaluate()
            st = sim.read("stencil")
            kpc = sim.read("curv_plain")
        listed = np.any(st != 0, axis=1)
        ok = listed & (nfl[keep] == 1) & (typ[keep] == wl.FLUID)
        nf = nrm[keep][ok]
        nh = nf / np.linalg.norm(nf, axis=1, keepdims=True)
        Xs.append(st[ok])
        Ts.append(np.concatenate([nh, (kap[keep][ok] * hc)[:, None]], axis=1))
        Ps.append(kpc[ok] * hc)
    return np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Ps)


# ----------------------------------------------------------------- training

def to_device_bf16(X: np.ndarray, device="cuda:0"):
    import torch
    return torch.tensor(np.asarray(X, dtype=np.float32), device=device).to(torch.bfloat16).contiguous()


def train(X: np.ndarray, T: np.ndarray, epochs: int = 40, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          params: np.ndarray = None, device="cuda:0", log=print) -> np.ndarray:
    """Adam on the mean squared error with the library's training kernels; the
    learning rate decays by 10x over the run (cosine)."""
    import torch
    Xd = to_device_bf16(X, device)
    Td = torch.tensor(np.asarray(T, dtype=np.float32), device=device)
    w0 = xavier_params(seed) if params is None else params
    tr = Trainer(w0, batch, device)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    nb = n // batch
    total = epochs * nb
    it = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(device)
        tot = 0.0
        for b in range(nb):
            rows = perm[b * batch:(b + 1) * batch]
            xb = Xd.index_select(0, rows).contiguous()
            tb = Td.index_select(0, rows).contiguous()
            f = 0.1 + 0.9 * 0.5 * (1 + math.cos(math.pi * it / max(total, 1)))
            loss = tr.step(xb, tb, lr * f)
            it += 1
            if b == nb - 1:
                tot = float(loss)
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"[closure] epoch {ep} loss {tot:.3e}")
    w = tr.params()
    tr.close()
    return w


def predict(params: np.ndarray, X: np.ndarray, device="cuda:0") -> np.ndarray:
    Xd = to_device_bf16(X, device)
    tr = Trainer(params, max(1, X.shape[0]), device)
    Y = tr.forward(Xd).cpu().numpy().astype(np.float64)
    tr.close()
    return Y


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def save(params: np.ndarray, path: str = WEIGHTS, **meta):
    np.savez(path, params=np.asarray(params, dtype=np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def load(path: str = WEIGHTS) -> np.ndarray:
    return np.load(path, allow_pickle=False)["params"].astype(np.float32)
