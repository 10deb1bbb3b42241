"""FP64 reference for the learned curvature closure (test infrastructure only).

Stencil of a surface particle a: the relative positions (r_b - r_a)/h of its
fluid neighbours (r_ab < 2h, b != a); at most the 32 nearest are kept (ties by
particle id). Each is written in the particle's frame: e1 = n_a/|n_a|, the
unit colour gradient of eq. 18 (pointing into the liquid), and e2 = e1 turned
by +90 degrees, so the entry is (d.e1, d.e2) for d = (r_b - r_a)/h. Entries are
ordered by their angle atan2(d.e2, d.e1) in (-pi, pi] (ties: nearer first,
then lower id) and zero-padded to 32; the network input is
(x0, y0, x1, y1, ...), 64 numbers.

Network: 64 -> 64 -> 64 -> 3, tanh on both hidden layers, linear output
(n_1, n_2, kappa h): the interface normal in the frame (e1, e2) and the
curvature. Loss: mean squared error over the batch and the three outputs,
equal weights. Training: Adam on FP32 master weights whose BF16 copies feed
the forward pass.

Everything here is plain numpy in float64: definitions written out, no
blocking, so it can be read against the description above.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

K_STENCIL = 32
N_IN, N_H, N_OUT = 64, 64, 3


# ----------------------------------------------------------------- stencils

def frame(n_a) -> Tuple[np.ndarray, np.ndarray]:
    """(e1, e2): the unit colour gradient and its +90 degree turn."""
    e1 = np.asarray(n_a, dtype=np.float64) / math.hypot(float(n_a[0]), float(n_a[1]))
    return e1, np.array([-e1[1], e1[0]])


def stencil_of(a: int, pos: np.ndarray, nbrs, types: np.ndarray, h: float, n_a) -> np.ndarray:
    """64-vector stencil of particle a from its neighbour list (ids b != a with
    r_ab < 2h) and its colour gradient n_a. Only fluid neighbours enter."""
    e1, e2 = frame(n_a)
    cand = [b for b in nbrs if types[b] == 0]
    d = [(float((pos[b, 0] - pos[a, 0]) ** 2 + (pos[b, 1] - pos[a, 1]) ** 2), int(b)) for b in cand]
    d.sort()
    keep = [b for _, b in d[:K_STENCIL]]
    items = []
    for b in keep:
        dx = (pos[b, 0] - pos[a, 0]) / h
        dy = (pos[b, 1] - pos[a, 1]) / h
        x = dx * e1[0] + dy * e1[1]
        y = dx * e2[0] + dy * e2[1]
        ang = math.atan2(y, x)
        if ang == -math.pi:
            ang = math.pi
        items.append((ang, dx * dx + dy * dy, b, x, y))
    items.sort(key=lambda t: (t[0], t[1], t[2]))
    out = np.zeros(2 * K_STENCIL)
    for i, (_, _, _, x, y) in enumerate(items):
        out[2 * i] = x
        out[2 * i + 1] = y
    return out


def stencils(pos, start, nbr, types, h, which, nrm) -> np.ndarray:
    """Stencils of the particles `which` (ids) from CSR neighbour lists and
    colour gradients nrm (n x 2)."""
    return np.stack([stencil_of(int(a), pos, nbr[start[a]:start[a + 1]], types, h, nrm[a]) for a in which]) \
        if len(which) else np.zeros((0, 2 * K_STENCIL))


# ----------------------------------------------------------------- network

def init_params(seed: int = 0) -> Dict[str, np.ndarray]:
    """Xavier-uniform weights, zero biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))

    def xavier(fan_in, fan_out):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_in, fan_out))

    return dict(W1=xavier(N_IN, N_H), b1=np.zeros(N_H), W2=xavier(N_H, N_H), b2=np.zeros(N_H),
                W3=xavier(N_H, N_OUT), b3=np.zeros(N_OUT))


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (round to nearest even on the float32
    bit pattern), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p: Dict[str, np.ndarray], X: np.ndarray):
    """Returns (Y, cache) with Y = W3^T tanh(W2^T tanh(W1^T x + b1) + b2) + b3 per row."""
    Z1 = X @ p["W1"] + p["b1"]
    H1 = np.tanh(Z1)
    Z2 = H1 @ p["W2"] + p["b2"]
    H2 = np.tanh(Z2)
    Y = H2 @ p["W3"] + p["b3"]
    return Y, (X, H1, H2)


def loss(Y: np.ndarray, T: np.ndarray) -> float:
    return float(np.mean((Y - T) ** 2))


def backward(p: Dict[str, np.ndarray], cache, Y: np.ndarray, T: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of the mean squared error (chain rule, layer by layer)."""
    X, H1, H2 = cache
    B = Y.shape[0]
    dY = 2.0 * (Y - T) / (B * Y.shape[1])
    g = {}
    g["W3"] = H2.T @ dY
    g["b3"] = dY.sum(0)
    dH2 = dY @ p["W3"].T
    dZ2 = dH2 * (1.0 - H2 ** 2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(0)
    dH1 = dZ2 @ p["W2"].T
    dZ1 = dH1 * (1.0 - H1 ** 2)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(0)
    return g


def adam_step(p, g, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1) of params p in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def flat_params(p) -> np.ndarray:
    """Parameter order of the packed buffers: W1 (row-major 64x64), b1, W2, b2,
    W3 (64x3), b3."""
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]])


def unflat_params(w: np.ndarray) -> Dict[str, np.ndarray]:
    w = np.asarray(w, dtype=np.float64)
    o = 0
    out = {}
    for k, shp in (("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
                   ("W3", (N_H, N_OUT)), ("b3", (N_OUT,))):
        n = int(np.prod(shp))
        out[k] = w[o:o + n].reshape(shp)
        o += n
    return out


N_PARAMS = N_IN * N_H + N_H + N_H * N_H + N_H + N_H * N_OUT + N_OUT


# ----------------------------------------------------------------- closure

def closure_curvature(Y: np.ndarray, h, n_a: np.ndarray):
    """Network output and the particles' colour gradients -> (unit normal in
    x, y, kappa)."""
    e1 = n_a / np.linalg.norm(n_a, axis=1, keepdims=True)
    e2 = np.stack([-e1[:, 1], e1[:, 0]], axis=1)
    nrm = Y[:, :1] * e1 + Y[:, 1:2] * e2
    m = np.linalg.norm(nrm, axis=1, keepdims=True)
    nh = np.where(m > 0, nrm / np.where(m > 0, m, 1.0), 0.0)
    return nh, Y[:, 2] / h


def fallback(kappa_mlp: np.ndarray, kappa_plain: np.ndarray, tol: float = 0.2) -> np.ndarray:
    """True where the plain estimate replaces the network's: a relative
    deviation above tol."""
    return np.abs(kappa_mlp - kappa_plain) > tol * np.abs(kappa_plain)


def closure_evaluate(obj, params, tol=None) -> Dict[str, np.ndarray]:
    """Right-hand sides with the learned closure in the surface-tension term.

    Every fluid particle of a closure system (params["closure"] = 1) that
    passes the normal filter of eq. 20 gets a stencil; the network, with its
    weights and the stencil rounded to BF16 and everything else in FP64, gives
    (n_1, n_2, kappa h) in the frame of the colour gradient. Its curvature and
    unit normal enter eq. 24 as
    a_s = -(sigma / rho_a) kappa |n_a| n_hat, unless the network's curvature
    differs from the plain one (eq. 23) by more than tol |kappa_plain| (default:
    the system's closure_tol, else 0.2) or its normal is zero; then the plain
    term stays. Returns the plain evaluation's dict with acc, kappa, asurf,
    dt_f and dt replaced, plus: kappa_plain (eq. 23), listed (bool), X (stencils of the listed
    particles, in id order), Y (network outputs), fallback (bool per particle).
    """
    import oracle
    res = oracle.evaluate(obj)
    start, nbr = oracle.neighbors(obj)
    systems = obj.systems if hasattr(obj, "systems") else [obj]
    off = np.zeros(len(systems) + 1, dtype=np.int64)
    off[1:] = np.cumsum([s.n for s in systems])
    pos = np.concatenate([s.pos for s in systems])
    rho = np.concatenate([s.rho for s in systems])
    typ = np.concatenate([s.type for s in systems])
    pb = {k: (bf16_round(v) if k.startswith("W") else np.asarray(v, dtype=np.float32).astype(np.float64))
          for k, v in unflat_params(params).items()}
    n = len(typ)
    listed = np.zeros(n, dtype=bool)
    fb = np.zeros(n, dtype=bool)
    Xs, Ys = [], []
    acc = res["acc"].copy()
    asurf = res["asurf"].copy()
    kappa = res["kappa"].copy()
    for s, sysm in enumerate(systems):
        p = sysm.params
        if not p.get("closure", 0):
            continue
        lo, hi = int(off[s]), int(off[s + 1])
        ids = np.nonzero((typ[lo:hi] == 0) & (res["nflag"][lo:hi] == 1))[0] + lo
        if len(ids) == 0:
            continue
        h = float(p["h"])
        X = bf16_round(stencils(pos, start, nbr, typ, h, ids, res["nrm"]))
        Y, _ = forward(pb, X)
        nh, k_mlp = closure_curvature(Y, h, res["nrm"][ids])
        t = tol if tol is not None else (p.get("closure_tol", 0.0) or 0.2)
        k_plain = res["kappa"][ids]
        bad = fallback(k_mlp, k_plain, t) | ~np.any(nh != 0, axis=1)
        nv = res["nrm"][ids]
        mag = np.linalg.norm(nv, axis=1)
        use_k = np.where(bad, k_plain, k_mlp)
        use_n = np.where(bad[:, None], nv / mag[:, None], nh)
        a_s = (-float(p["sigma"]) / rho[ids] * use_k * mag)[:, None] * use_n
        acc[ids] = res["apv"][ids] + a_s + np.asarray(p["gravity"], dtype=np.float64)
        asurf[ids] = a_s
        kappa[ids] = use_k
        listed[ids] = True
        fb[ids] = bad
        Xs.append(X)
        Ys.append(Y)
        # the acceleration limit of eq. 30 over the system's fluid particles
        fl = np.nonzero(typ[lo:hi] == 0)[0] + lo
        am = np.linalg.norm(acc[fl], axis=1)
        am = am[am > 0]
        dtf = float(np.min(np.sqrt(h / am))) if am.size else math.inf
        res["dt_f"][s] = dtf
        d = p["dt_fixed"] if p.get("dt_fixed", 0.0) > 0 else p["courant"] * min(dtf, res["dt_cv"][s])
        res["dt"][s] = d if math.isfinite(d) else 0.0
    res.update(kappa_plain=res["kappa"], acc=acc, asurf=asurf, kappa=kappa, listed=listed, fallback=fb,
               X=np.concatenate(Xs) if Xs else np.zeros((0, 64)), Y=np.concatenate(Ys) if Ys else np.zeros((0, 3)))
    return res
