"""Pins of the FP64 closure reference (stencil definition and MLP)."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import mlp


def test_gradients_match_central_differences():
    rng = np.random.Generator(np.random.PCG64(1))
    p = mlp.init_params(3)
    for k in p:
        p[k] = p[k] + rng.normal(0, 0.1, size=p[k].shape)
    X = rng.normal(0, 1, size=(7, 64))
    T = rng.normal(0, 1, size=(7, 3))
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, Y, T)
    e = 1e-6
    for k in p:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + e
            lp = mlp.loss(mlp.forward(p, X)[0], T)
            flat[i] = old - e
            lm = mlp.loss(mlp.forward(p, X)[0], T)
            flat[i] = old
            fd = (lp - lm) / (2 * e)
            an = g[k].ravel()[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, i, fd, an)


def test_zero_network_outputs_bias():
    p = mlp.init_params(0)
    for k in ("W1", "W2", "W3"):
        p[k][:] = 0.0
    p["b3"][:] = [0.5, -1.0, 2.0]
    Y, _ = mlp.forward(p, np.ones((4, 64)))
    assert np.all(Y == [[0.5, -1.0, 2.0]])


def test_adam_first_step_moves_by_lr_sign():
    p = {"w": np.array([1.0, -2.0])}
    g = {"w": np.array([0.3, -5.0])}
    m = {"w": np.zeros(2)}
    v = {"w": np.zeros(2)}
    mlp.adam_step(p, g, m, v, 1, lr=1e-2)
    # m_hat = g, v_hat = g^2 after one step: the move is lr * g / (|g| + eps)
    assert np.allclose(p["w"], [1.0 - 1e-2, -2.0 + 1e-2], atol=1e-9)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.Generator(np.random.PCG64(2))
    x = np.concatenate([rng.normal(0, 3, 5000), [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -0.0, 1e-30, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_flat_params_round_trip():
    p = mlp.init_params(5)
    w = mlp.flat_params(p)
    assert w.size == mlp.N_PARAMS == 64 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
    q = mlp.unflat_params(w)
    for k in p:
        assert np.array_equal(p[k], q[k])


def _lattice_stencil(angle=0.0, shift=(0.0, 0.0), jitter=0.0, normal=(1.0, 0.0)):
    s = wl.lattice_block(11, 11, dx=1.0)
    if jitter:
        rng = np.random.Generator(np.random.PCG64(4))
        s.pos = s.pos + rng.uniform(-jitter, jitter, size=s.pos.shape)
    c, sn = math.cos(angle), math.sin(angle)
    R = np.array([[c, sn], [-sn, c]])        # row vectors turned by +angle
    s.pos = s.pos @ R + np.array(shift)
    n_a = np.asarray(normal) @ R
    import oracle
    start, nbr = oracle.neighbors(s)
    a = 5 * 11 + 5  # the centre of the block
    return mlp.stencil_of(a, s.pos, nbr[start[a]:start[a + 1]], s.type, s.params["h"], n_a), s.params["h"]


def test_lattice_stencil_geometry(orc):
    st, h = _lattice_stencil()
    xy = st.reshape(-1, 2) * h
    nz = np.any(xy != 0, axis=1)
    # within 2h = 2.6 dx of a lattice site: rings at 1, sqrt 2, 2, sqrt 5 -> 4 + 4 + 4 + 8
    assert nz.sum() == 20
    assert np.all(~nz[20:])
    pts = np.rint(xy[:20]).astype(int)
    assert np.allclose(xy[:20], pts, atol=1e-12)
    assert sorted(map(tuple, pts)) == sorted((i, j) for i in range(-2, 3) for j in range(-2, 3)
                                             if 0 < i * i + j * j <= 5)
    ang = np.arctan2(pts[:, 1], pts[:, 0])
    ang[ang == -np.pi] = np.pi
    assert np.all(np.diff(ang) >= 0)
    same = np.diff(ang) == 0
    r2 = (pts ** 2).sum(1)
    assert np.all(np.diff(r2)[same] > 0)    # collinear neighbours: nearer first


def test_stencil_translation_and_rotation_invariance(orc):
    base, _ = _lattice_stencil()
    moved, _ = _lattice_stencil(shift=(123.25, -7.5))
    assert np.allclose(base, moved, atol=1e-9)
    # turning the particles and the colour gradient together leaves the stencil
    # (written in the gradient's frame) unchanged, order included
    j0, _ = _lattice_stencil(jitter=0.1, normal=(0.6, 0.8))
    for ang in (0.3, math.pi / 2 + 1e-3, 2.5, -1.9):
        jr, _ = _lattice_stencil(angle=ang, jitter=0.1, normal=(0.6, 0.8))
        assert np.allclose(j0, jr, atol=1e-9), ang
    # a frame turned against the particles turns every entry the other way
    c, s = math.cos(0.7), math.sin(0.7)
    fr, _ = _lattice_stencil(normal=(c, s))
    want = base.reshape(-1, 2)[:20] @ np.array([[c, -s], [s, c]])
    got = fr.reshape(-1, 2)[:20]
    match = [int(np.argmin(np.linalg.norm(got - x, axis=1))) for x in want]
    assert sorted(match) == list(range(20))
    assert all(np.linalg.norm(got[m] - x) < 1e-9 for m, x in zip(match, want))


def test_fallback_rule():
    km = np.array([1.0, 1.3, -2.0, 0.1, 0.0])
    kp = np.array([1.1, 1.0, -2.3, 0.0, 0.0])
    assert list(mlp.fallback(km, kp, 0.2)) == [False, True, False, True, False]


def _closure_disc():
    d = wl.circle(10.0, dx=1.0, layout="rings")
    d.params["closure"] = 1
    return d


def test_closure_with_zero_network_falls_back_to_plain(orc):
    d = _closure_disc()
    r = mlp.closure_evaluate(d, np.zeros(mlp.N_PARAMS))
    o = orc.evaluate(d)
    listed = (d.type == wl.FLUID) & (o["nflag"] == 1)
    assert listed.sum() > 50 and np.array_equal(r["listed"], listed)
    # kappa_mlp = 0 and a zero normal: every listed particle keeps eq. 23-24
    assert np.all(r["fallback"][listed])
    scale = np.abs(o["acc"]).max()
    assert np.allclose(r["acc"], o["acc"], rtol=0, atol=1e-12 * scale)
    assert np.array_equal(r["kappa"], o["kappa"])


def test_closure_replaces_the_surface_term(orc):
    # a network that always answers "flat" (kappa = 0, normal e1) with no
    # fallback removes the surface-tension term of the listed particles and
    # nothing else
    d = _closure_disc()
    w = np.zeros(mlp.N_PARAMS)
    w[-3:] = [1.0, 0.0, 0.0]
    r = mlp.closure_evaluate(d, w, tol=np.inf)
    o = orc.evaluate(d)
    L = r["listed"]
    assert not r["fallback"].any()
    assert np.allclose(r["acc"][L], o["apv"][L] + np.asarray(d.params["gravity"]), rtol=0, atol=1e-15)
    assert np.array_equal(r["acc"][~L], o["acc"][~L])
    assert np.all(r["kappa"][L] == 0.0)
    # the plain surface force on the disc rim points to the centre
    rim = L & (np.hypot(d.pos[:, 0], d.pos[:, 1]) > 9.0)
    assert np.all(np.einsum("ij,ij->i", o["asurf"][rim], d.pos[rim]) < 0)


def test_rim_stencils_lean_inward(orc):
    d = _closure_disc()
    r = mlp.closure_evaluate(d, np.zeros(mlp.N_PARAMS))
    ids = np.nonzero(r["listed"])[0]
    rim = np.hypot(d.pos[ids, 0], d.pos[ids, 1]) > 9.0
    X = r["X"].reshape(len(ids), 32, 2)
    mean = X.sum(1)
    assert rim.sum() > 30
    # in the colour-gradient frame the liquid lies along +e1
    assert np.all(mean[rim, 0] > 0)
    # and the stencils of the rim particles, all seen from their own frame, are
    # nearly mirror-symmetric about e1 on the ring layout
    assert np.all(np.abs(mean[rim, 1]) < 0.5 * mean[rim, 0])
    # every stencil entry is a fluid neighbour inside the support, in BF16
    rr = np.linalg.norm(X, axis=2)
    assert np.all(rr <= 2.0 + 2 ** -7)
    assert np.array_equal(mlp.bf16_round(r["X"]), r["X"])
