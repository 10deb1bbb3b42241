"""Learned curvature closure: training data, training loop and accuracy.

The network and its kernels live in the library (sph_mlp_* and the closure
path of the particle update, include/sph.h); this module marshals data.

Training neighbourhoods come from the library's own stencil kernel, run on
two kinds of particle sets whose interface geometry is known:

* discs (radius 3-50 dx) and sinusoidal interfaces (amplitude 0.5-5 dx,
  wavelength 10-60 dx), with particles in layers that follow the interface
  or cut from the square lattice, jittered and randomly rotated, labelled
  with the exact unit normal and curvature of the interface at the
  particle's nearest interface point (particles within 2h of the interface);
* jets: a jet run at 4x the target resolution is Poisson-disk subsampled to
  the target spacing; the coarse set is labelled by the fine run's plain
  estimate (eq. 18-23), averaged with Wendland weights of the coarse h over
  the fine interface particles around each coarse particle.

Only interface particles (see INTERFACE_NH) enter the training sets and the
accuracy figures.

Targets are (n_1, n_2, kappa h): the unit normal pointing into the liquid (the
direction of grad C) written in the particle's frame (e1 = its unit colour
gradient, e2 = e1 turned by +90 degrees), and kappa = div n_hat (negative on a
convex liquid surface), as in eq. 23. Training runs sph_mlp_train_step (forward, backward
and Adam on the GPU).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import native

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS = os.path.join(HERE, "closure_weights.npz")

# Interface particles for labels and accuracy figures: |n| h >= INTERFACE_NH.
# The colour gradient (eq. 18) is about 0.1-0.15/h in the two outer particle
# layers of a free surface and at most a few hundredths of 1/h deeper, where the filter of eq. 20
# (|n| > 0.01/h) still passes particles whose stencil does not see the surface.
INTERFACE_NH = 0.05


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
        assert w.size == native.MLP_NPARAMS
        h = C.c_void_p()
        native.check(L.sph_mlp_create(w.ctypes.data_as(C.c_void_p), self.max_batch, _ptr(self.ws),
                                      int(nbytes.value), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h
        self.loss_dev = torch.zeros(4, dtype=torch.float32, device=self.device)

    def forward(self, X):
        Y = self.torch.empty((X.shape[0], 3), dtype=self.torch.float32, device=self.device)
        native.check(self._L.sph_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(Y)))
        return Y

    def gradient(self, X, T):
        g = self.torch.empty(native.MLP_NPARAMS, dtype=self.torch.float32, device=self.device)
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


# ----------------------------------------------------------------- shapes

def _rotate(xy, th):
    cs, sn = math.cos(th), math.sin(th)
    return xy @ np.array([[cs, sn], [-sn, cs]])


def _jittered_lattice(x0, y0, nx, ny, dx, jitter, rng):
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    p = np.stack([x0 + (i.ravel() + 0.5) * dx, y0 + (j.ravel() + 0.5) * dx], axis=1)
    if jitter > 0:
        p = p + rng.uniform(-jitter * dx, jitter * dx, size=p.shape)
    return p


def _disc_label(q, R, dx):
    r = np.hypot(q[:, 0], q[:, 1])
    nh = -q / np.maximum(r, 1e-12)[:, None]
    return nh, np.full(len(q), -1.0 / R), r > R - 2.6 * dx


def _sine_label(q, A, kk, lam, dx):
    """Normal and curvature of y = A sin(kk x) at the interface point nearest
    to each particle (Newton on the squared distance), liquid below."""
    x = q[:, 0].copy()
    for _ in range(20):
        f = A * np.sin(kk * x)
        f1 = A * kk * np.cos(kk * x)
        f2 = -A * kk * kk * np.sin(kk * x)
        g = (x - q[:, 0]) + (f - q[:, 1]) * f1
        g1 = 1.0 + f1 * f1 + (f - q[:, 1]) * f2
        x = x - g / g1
    f1 = A * kk * np.cos(kk * x)
    den = np.sqrt(1 + f1 * f1)
    nh = np.stack([f1 / den, -1.0 / den], axis=1)
    kap = -A * kk * kk * np.sin(kk * x) / den ** 3
    dist = np.hypot(x - q[:, 0], A * np.sin(kk * x) - q[:, 1])
    keep = (q[:, 0] > lam) & (q[:, 0] < 3 * lam) & (dist < 2.6 * dx)
    return nh, kap, keep


def shape_systems(n_shapes: int, seed: int, dx: float = 1.0, conforming: float = 0.8):
    """Discs and sinusoidal slabs with their exact interface geometry, each
    randomly rotated and jittered (0-0.1 dx). A fraction `conforming` of them
    has particles in layers that follow the interface (rings, columns), as a
    relaxed free surface does; the rest is cut from the square lattice, with
    its staircase. meta["label"](unrotated positions) returns (unit normal,
    kappa, keep mask)."""
    import workloads as wl
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_shapes):
        jitter = float(rng.choice([0.0, 0.02, 0.05, 0.1]))
        th = float(rng.uniform(0, 2 * math.pi))
        layered = bool(rng.uniform() < conforming)
        sub = int(rng.integers(0, 2**31 - 1))
        if k % 2 == 0:
            R = float(math.exp(rng.uniform(math.log(3.0), math.log(50.0)))) * dx
            s = wl.circle(R, dx=dx, jitter=jitter, seed=sub, layout="rings" if layered else "lattice")
            label = (lambda q, R=R: _disc_label(q, R, dx))
        else:
            A = float(rng.uniform(0.5, 5.0)) * dx
            lam = float(rng.uniform(10.0, 60.0)) * dx
            s = wl.sinusoid(A, lam, dx=dx, periods=4, depth=12.0 * dx, jitter=jitter, seed=sub,
                            layout="columns" if layered else "lattice")
            label = (lambda q, A=A, kk=2 * math.pi / lam, lam=lam: _sine_label(q, A, kk, lam, dx))
        pr = _rotate(s.pos, th)
        s.pos = pr
        s.params.update(closure=1, box_lo=tuple(pr.min(0) - 4 * dx), box_hi=tuple(pr.max(0) + 4 * dx),
                        cell_size=2.2 * 1.3 * dx)
        s.meta = dict(theta=th, label=label, layered=layered, jitter=jitter)
        out.append(s)
    return out


def _chunks(systems, max_particles):
    i = 0
    while i < len(systems):
        grp, n = [], 0
        while i < len(systems) and (n + systems[i].n <= max_particles or not grp):
            grp.append(systems[i])
            n += systems[i].n
            i += 1
        yield grp


def _listed_rows(sim, hpp):
    """Stencils, plain curvature, the listed interface particles
    (|n| h >= INTERFACE_NH) and the unit colour gradients e1 of a closure
    evaluation; hpp: h per particle."""
    sim.evaluate()
    st = sim.read("stencil")
    listed = sim.read("closure")[:, 3] == 1.0
    n = sim.read("normal")
    mag = np.linalg.norm(n, axis=1)
    e1 = n / np.maximum(mag, 1e-300)[:, None]
    return st, sim.read("curv_plain"), listed & (mag * hpp >= INTERFACE_NH), e1


def to_frame(v: np.ndarray, e1: np.ndarray) -> np.ndarray:
    """Vectors v (k x 2) in the frames (e1, e2 = e1 turned by +90 degrees)."""
    return np.stack([v[:, 0] * e1[:, 0] + v[:, 1] * e1[:, 1], v[:, 1] * e1[:, 0] - v[:, 0] * e1[:, 1]], axis=1)


def _hpp(grp):
    return np.concatenate([np.full(s.n, s.params["h"]) for s in grp])


def harvest_shapes(systems, device="cuda:0", chunk_particles: int = 2_000_000):
    """(stencils, targets (n_1, n_2, kappa h), plain kappa h, index of the
    shape) of every listed particle near the interface of the shapes."""
    from .sim import Simulation
    X, T, P, I = [], [], [], []
    k = 0
    for grp in _chunks(systems, chunk_particles):
        with Simulation(grp, dtype_bits=32, device=device) as sim:
            st, kplain, listed, e1 = _listed_rows(sim, _hpp(grp))
        o = 0
        for s in grp:
            sl = slice(o, o + s.n)
            o += s.n
            h = s.params["h"]
            th = s.meta["theta"]
            nh, kap, keep = s.meta["label"](_rotate(s.pos, -th))
            m = listed[sl] & keep
            X.append(st[sl][m])
            T.append(np.concatenate([to_frame(_rotate(nh, th)[m], e1[sl][m]), (kap[m] * h)[:, None]], axis=1))
            P.append(kplain[sl][m] * h)
            I.append(np.full(int(m.sum()), k))
            k += 1
    return np.concatenate(X), np.concatenate(T), np.concatenate(P), np.concatenate(I)


# ----------------------------------------------------------------- jets

def poisson_subsample(pos: np.ndarray, rmin: float, seed: int) -> np.ndarray:
    """Indices of a greedy Poisson-disk subset: points are visited in seeded
    random order and kept when no kept point lies closer than rmin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    order = rng.permutation(len(pos))
    cs = rmin / math.sqrt(2.0)   # at most one kept point per grid cell
    lo = pos.min(0)
    g = np.floor((pos - lo) / cs).astype(np.int64)
    ny = int(g[:, 1].max()) + 5
    occ: Dict[int, int] = {}
    kept = []
    r2 = rmin * rmin
    offs = [(a, b) for a in range(-2, 3) for b in range(-2, 3)]
    for i in order:
        gx, gy = int(g[i, 0]), int(g[i, 1])
        px, py = pos[i, 0], pos[i, 1]
        ok = True
        for a, b in offs:
            j = occ.get((gx + a) * ny + gy + b)
            if j is not None:
                dx, dy = pos[j, 0] - px, pos[j, 1] - py
                if dx * dx + dy * dy < r2:
                    ok = False
                    break
        if ok:
            occ[gx * ny + gy] = i
            kept.append(i)
    return np.array(sorted(kept), dtype=np.int64)


def _wendland(q):
    return np.where(q < 2.0, (1 - q / 2) ** 4 * (1 + 2 * q), 0.0)


def fine_jet_snapshots(nD_coarse: int, Re: float, We: float, seed: int, steps: Sequence[int],
                       n_fine: int = 300_000, free_length: float = 30.0, piston_amp: float = 0.01,
                       avg_steps: int = 1, device="cuda:0"):
    """Run a jet at 4 nD_coarse particles per D (piston velocity amplitude
    `piston_amp`) and return snapshots (fluid positions, unit normals, plain
    curvature and filter flags) after each step count in `steps` (ascending).

    With avg_steps = K > 1 the curvature of each snapshot is the mean over the
    K fine steps that start at it (K = 4 spans about one step of the coarse
    run, whose dt is four times the fine one), taken over the steps at which
    the particle is an interface particle; positions, normals and the
    interface flag are the first step's."""
    import workloads as wl
    from .sim import Simulation
    fine = wl.round_for_dtype(wl.jet(n_target=n_fine, nD=4 * nD_coarse, Re=Re, We=We, seed=seed,
                                     free_length=free_length, prefill=free_length / 3), 32)
    fine.params["piston_amp"] = float(piston_amp)
    t_plate = 3 * fine.meta["dx"]
    snaps = []
    done = 0
    h = fine.params["h"]

    def interface(sim):
        nrm = sim.read("normal")
        mag = np.linalg.norm(nrm, axis=1)
        return nrm, mag, (sim.read("nflag") == 1) & (mag * h >= INTERFACE_NH)

    with Simulation(fine, dtype_bits=32, device=device, graph_steps=50) as sim:
        for st in steps:
            if st > done:
                sim.step(st - done)
                done = st
            sim.evaluate()
            typ = sim.read("type")
            pos = sim.read("pos")
            sel = (typ == wl.FLUID) & (pos[:, 0] > t_plate + 0.5)
            nrm, mag, iface = interface(sim)
            nh = np.where(mag[:, None] > 0, nrm / np.maximum(mag, 1e-300)[:, None], 0.0)
            k1 = sim.read("curv")
            ksum = np.where(iface, k1, 0.0)
            kcnt = iface.astype(np.int64)
            for _ in range(avg_steps - 1):
                sim.step(1)
                done += 1
                sim.evaluate()
                _, _, fi = interface(sim)
                ksum += np.where(fi, sim.read("curv"), 0.0)
                kcnt += fi
            kappa = ksum / np.maximum(kcnt, 1)
            snaps.append(dict(pos=pos[sel], nhat=nh[sel], kappa=kappa[sel], kappa_first=k1[sel],
                              iface=iface[sel], step=st, h_fine=h, avg_steps=avg_steps))
    return snaps


def coarse_from_snapshot(snap, nD_coarse: int, Re: float, We: float, seed: int, window: float = 1.0,
                         label_h: float = 0.0, rmin: float = 0.78, keep=None):
    """Poisson-disk subsample of a fine snapshot at the coarse spacing (number
    density 1/dx^2) with reference labels; returns a closure System whose
    meta holds (nhat_ref, kappa_ref, has_ref).

    A label is the Wendland-weighted mean, W(r / h_l), of the fine interface
    particles' normals and curvatures within window * h_l of the kept
    particle, h_l the coarse smoothing length (or label_h, so that a finer
    subsample can be labelled at the same physical scale); window = 2 is the
    whole support of the coarse kernel.

    The meta also holds kappa_halves (n x 2) and has_halves: the same label
    computed from each half of a seeded random split of the fine interface
    particles. Their spread measures the label's own noise (split-half).
    `keep` (indices into the snapshot) replaces the subsample when given."""
    import workloads as wl
    from scipy.spatial import cKDTree
    dxc = 1.0 / nD_coarse
    # one greedy pass over the fine points (16 per coarse cell) with
    # rmin = 0.78 dx keeps one point per dx^2 (measured on a jittered lattice;
    # a subsample at half the fine run's spacing needs its own rmin)
    if keep is None:
        keep = poisson_subsample(snap["pos"], rmin * dxc, seed)
    pc = snap["pos"][keep]
    hc = label_h if label_h > 0 else 1.3 * dxc
    surf = snap["iface"]
    sp = snap["pos"][surf]
    sn = snap["nhat"][surf]
    sk = snap["kappa"][surf]
    tree = cKDTree(sp)
    nbrs = tree.query_ball_point(pc, r=window * hc)
    nref = np.zeros((len(pc), 2))
    kref = np.zeros(len(pc))
    has = np.zeros(len(pc), dtype=bool)
    half = np.random.default_rng(seed + 7).integers(0, 2, size=len(sp))
    khalf = np.zeros((len(pc), 2))
    has_half = np.zeros(len(pc), dtype=bool)
    for i, lst in enumerate(nbrs):
        if len(lst) < 3:
            continue
        idx = np.asarray(lst)
        w = _wendland(np.linalg.norm(sp[idx] - pc[i], axis=1) / hc)
        v = (w[:, None] * sn[idx]).sum(0)
        if np.linalg.norm(v) <= 0.5 * w.sum():   # normals disagree: no clean label
            continue
        nref[i] = v / np.linalg.norm(v)
        kref[i] = (w * sk[idx]).sum() / w.sum()
        has[i] = True
        hs = half[idx]
        wa, wb = w[hs == 0], w[hs == 1]
        if (hs == 0).sum() >= 2 and (hs == 1).sum() >= 2 and wa.sum() > 0 and wb.sum() > 0:
            khalf[i, 0] = (wa * sk[idx][hs == 0]).sum() / wa.sum()
            khalf[i, 1] = (wb * sk[idx][hs == 1]).sum() / wb.sum()
            has_half[i] = True
    p = wl.scenarios.jet_params(nD_coarse, Re, We)
    p.update(closure=1, box_lo=tuple(pc.min(0) - 4 * dxc), box_hi=tuple(pc.max(0) + 4 * dxc))
    n = len(pc)
    return wl.System(p, pc.copy(), np.zeros((n, 2)), np.ones(n), np.full(n, dxc * dxc), np.zeros(n, np.int32),
                     name="jet_coarse", meta=dict(nhat_ref=nref, kappa_ref=kref, has_ref=has, nD=nD_coarse,
                                                  kappa_halves=khalf, has_halves=has_half))


def harvest_coarse(systems, device="cuda:0", chunk_particles: int = 2_000_000, params=None, halves=False):
    """(stencils, targets, plain kappa h, closure kappa h, fallback flags) of
    the listed particles of coarse jet sets that carry a reference label; with
    `params` the closure runs in the same evaluation (else its kappa is 0).
    With `halves` also the split-half labels (kappa h, n x 2) and their mask."""
    from .sim import Simulation
    X, T, P, K, F, H, HM = [], [], [], [], [], [], []
    for grp in _chunks(systems, chunk_particles):
        with Simulation(grp, dtype_bits=32, device=device) as sim:
            if params is not None:
                sim.set_closure(params)
            st, kplain, listed, e1 = _listed_rows(sim, _hpp(grp))
            kfin = sim.read("curv")
            fb = sim.read("fallback")
        o = 0
        for s in grp:
            sl = slice(o, o + s.n)
            o += s.n
            h = s.params["h"]
            m = listed[sl] & s.meta["has_ref"]
            X.append(st[sl][m])
            T.append(np.concatenate([to_frame(s.meta["nhat_ref"][m], e1[sl][m]),
                                     (s.meta["kappa_ref"][m] * h)[:, None]], axis=1))
            P.append(kplain[sl][m] * h)
            K.append(kfin[sl][m] * h)
            F.append(fb[sl][m])
            if halves:
                H.append(s.meta["kappa_halves"][m] * h)
                HM.append(s.meta["has_halves"][m])
    cat = np.concatenate
    if halves:
        return cat(X), cat(T), cat(P), cat(K), cat(F), cat(H), cat(HM)
    return cat(X), cat(T), cat(P), cat(K), cat(F)


# ----------------------------------------------------------------- training

def mirror(X: np.ndarray, T: np.ndarray):
    """Mirror images of stencils and targets about e1 (e2 -> -e2): entries
    (x, y) become (x, -y), re-ordered by angle (ties: nearer first), padding
    kept last; targets (n_1, n_2, kappa h) become (n_1, -n_2, kappa h)."""
    P = X.reshape(len(X), -1, 2).copy()
    P[:, :, 1] = -P[:, :, 1]
    pad = ~np.any(P != 0, axis=2)
    ang = np.arctan2(P[:, :, 1], P[:, :, 0])
    ang[ang == -np.pi] = np.pi
    ang[pad] = np.inf
    r2 = (P ** 2).sum(2)
    order = np.lexsort((r2, ang), axis=1)
    P = np.take_along_axis(P, order[:, :, None], axis=1)
    Tm = T.copy()
    Tm[:, 1] = -Tm[:, 1]
    return P.reshape(len(X), -1), Tm


def to_device_bf16(X: np.ndarray, device="cuda:0"):
    import torch
    return torch.tensor(np.asarray(X, dtype=np.float32), device=device).to(torch.bfloat16).contiguous()


def train(X: np.ndarray, T: np.ndarray, epochs: int = 40, batch: int = 4096, lr: float = 1e-3, seed: int = 0,
          params: np.ndarray = None, device="cuda:0", log=print) -> Tuple[np.ndarray, List[float]]:
    """Adam on the mean squared error with the library's training kernels, on
    seeded shuffled mini-batches; the learning rate follows a cosine from lr
    down to lr / 10. Returns the FP32 parameters and the mean loss per epoch."""
    import torch
    Xd = to_device_bf16(X, device)
    Td = torch.tensor(np.asarray(T, dtype=np.float32), device=device)
    w0 = xavier_params(seed) if params is None else params
    tr = Trainer(w0, batch, device)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    nb = max(n // batch, 1)
    total = epochs * nb
    it = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(device)
        acc = torch.zeros((), dtype=torch.float32, device=device)
        for b in range(nb):
            rows = perm[b * batch:(b + 1) * batch]
            xb = Xd.index_select(0, rows)
            tb = Td.index_select(0, rows)
            f = 0.1 + 0.9 * 0.5 * (1 + math.cos(math.pi * it / max(total, 1)))
            acc += tr.step(xb, tb, lr * f)
            it += 1
        hist.append(float(acc) / nb)
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"[closure] epoch {ep} loss {hist[-1]:.4e}")
    w = tr.params()
    tr.close()
    return w, hist


def predict(params: np.ndarray, X: np.ndarray, device="cuda:0") -> np.ndarray:
    Xd = to_device_bf16(X, device)
    tr = Trainer(params, max(1, X.shape[0]), device)
    Y = tr.forward(Xd).cpu().numpy().astype(np.float64)
    tr.close()
    return Y


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def apply_fallback(k_mlp: np.ndarray, k_plain: np.ndarray, tol: float = 0.2) -> np.ndarray:
    """Curvature the closure uses: the network's, or the plain one where the two
    differ by more than tol times the plain magnitude."""
    return np.where(np.abs(k_mlp - k_plain) > tol * np.abs(k_plain), k_plain, k_mlp)


def save(params: np.ndarray, path: str = WEIGHTS, **meta):
    np.savez(path, params=np.asarray(params, dtype=np.float32), **{k: np.asarray(v) for k, v in meta.items()})


def load(path: str = WEIGHTS) -> np.ndarray:
    return np.load(path, allow_pickle=False)["params"].astype(np.float32)
