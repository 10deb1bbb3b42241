"""Host-side logic of the closure's training data (no GPU)."""
import math

import numpy as np

import workloads as wl
from oracle import mlp
from paper_1603_02421_amd import closure as cl


def test_mirror_matches_stencil_of_mirrored_particles(orc):
    s = wl.lattice_block(11, 11, dx=1.0)
    rng = np.random.Generator(np.random.PCG64(4))
    s.pos = s.pos + rng.uniform(-0.1, 0.1, size=s.pos.shape)
    a = 60
    n = np.array([0.6, 0.8])
    start, nbr = orc.neighbors(s)
    X = mlp.stencil_of(a, s.pos, nbr[start[a]:start[a + 1]], s.type, s.params["h"], n)
    e1 = n / np.linalg.norm(n)
    P = s.pos - s.pos[a]
    m = s.copy()
    m.pos = 2 * np.outer(P @ e1, e1) - P + s.pos[a]   # reflection about the line along e1
    start2, nbr2 = orc.neighbors(m)
    Xm = mlp.stencil_of(a, m.pos, nbr2[start2[a]:start2[a + 1]], m.type, m.params["h"], n)
    Xa, Ta = cl.mirror(X[None], np.array([[0.9, 0.1, -0.2]]))
    assert np.abs(Xa[0] - Xm).max() < 1e-12
    assert np.array_equal(Ta, [[0.9, -0.1, -0.2]])


def test_to_frame_is_the_stencil_frame():
    rng = np.random.Generator(np.random.PCG64(1))
    v = rng.normal(size=(50, 2))
    n = rng.normal(size=(50, 2))
    e1 = n / np.linalg.norm(n, axis=1, keepdims=True)
    got = cl.to_frame(v, e1)
    for i in range(50):
        f1, f2 = mlp.frame(n[i])
        assert np.allclose(got[i], [v[i] @ f1, v[i] @ f2], atol=1e-14)


def test_shape_labels():
    # disc: inward normal and -1/R; sinusoid: nearest-point geometry
    nh, k, keep = cl._disc_label(np.array([[3.0, 4.0], [0.0, 1.0]]), 5.0, 1.0)
    assert np.allclose(nh[0], [-0.6, -0.8]) and np.allclose(k, -0.2)
    assert list(keep) == [True, False]
    A, kk, lam = 2.0, 2 * math.pi / 20.0, 20.0
    x0 = np.array([25.0, 27.0, 33.0])
    q = np.stack([x0, A * np.sin(kk * x0)], axis=1)          # points on the curve
    nh, kap, keep = cl._sine_label(q, A, kk, lam, 1.0)
    s = A * kk * np.cos(kk * x0)
    assert np.allclose(nh, np.stack([s, -np.ones(3)], 1) / np.sqrt(1 + s * s)[:, None])
    assert np.allclose(kap, -A * kk * kk * np.sin(kk * x0) / (1 + s * s) ** 1.5)
    # a point below the crest: its nearest interface point is the crest
    nh2, kap2, _ = cl._sine_label(np.array([[25.0, 1.0]]), A, kk, lam, 1.0)
    assert np.allclose(nh2, [[0.0, -1.0]], atol=1e-9) and np.isclose(kap2[0], -A * kk * kk)


def test_poisson_subsample_spacing_and_density():
    rng = np.random.Generator(np.random.PCG64(0))
    i, j = np.meshgrid(np.arange(160), np.arange(160), indexing="ij")
    pos = np.stack([(i.ravel() + 0.5) * 0.025, (j.ravel() + 0.5) * 0.025], 1)
    pos = pos + rng.uniform(-0.0025, 0.0025, size=pos.shape)
    k = cl.poisson_subsample(pos, 0.078, 3)
    from scipy.spatial import cKDTree
    d, _ = cKDTree(pos[k]).query(pos[k], k=2)
    assert d[:, 1].min() >= 0.078
    assert 0.9 * 1600 <= len(k) <= 1.1 * 1600   # about one point per 0.1 x 0.1 cell of the 4 x 4 square


def _disc_snapshot(R, dxf, noise, seed):
    """A fine lattice disc whose outer two rows are interface particles with
    the exact outward normal and curvature -1/R, the curvature perturbed by
    relative Gaussian noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(R / dxf) + 2
    i, j = np.meshgrid(np.arange(-n, n + 1), np.arange(-n, n + 1), indexing="ij")
    pos = np.stack([i.ravel() * dxf, j.ravel() * dxf], 1)
    r = np.hypot(pos[:, 0], pos[:, 1])
    pos = pos[r < R]
    r = r[r < R]
    iface = r > R - 2.0 * dxf
    nhat = pos / np.maximum(r, 1e-12)[:, None]
    kappa = -1.0 / R * (1.0 + noise * rng.normal(size=len(pos)))
    return dict(pos=pos, iface=iface, nhat=nhat, kappa=kappa)


def test_split_half_labels_measure_the_reference_noise():
    """Coarse labels from a fine snapshot: with exact fine curvature both
    half-labels equal the label; with noisy fine curvature, half the spread of
    the two halves estimates the noise left in the full (averaged) label."""
    R, dxc = 1.0, 0.1
    s0 = cl.coarse_from_snapshot(_disc_snapshot(R, dxc / 4, 0.0, 1), 10, 500.0, 20.0, seed=3)
    m = s0.meta["has_halves"]
    assert m.sum() > 20 and np.all(s0.meta["has_ref"][m])
    kh = s0.meta["kappa_halves"][m]
    assert np.allclose(kh[:, 0], -1.0 / R, rtol=1e-12) and np.allclose(kh[:, 1], -1.0 / R, rtol=1e-12)
    assert np.allclose(s0.meta["kappa_ref"][m], -1.0 / R, rtol=1e-12)
    s1 = cl.coarse_from_snapshot(_disc_snapshot(R, dxc / 4, 0.5, 2), 10, 500.0, 20.0, seed=3)
    m = s1.meta["has_halves"]
    ref = s1.meta["kappa_ref"][m]
    kh = s1.meta["kappa_halves"][m]
    floor = 0.5 * np.linalg.norm(kh[:, 0] - kh[:, 1]) / np.linalg.norm(ref)
    actual = np.linalg.norm(ref + 1.0 / R) / np.linalg.norm(ref)
    assert 0.02 < actual < 0.5
    assert 0.6 * actual < floor < 1.6 * actual


def test_wider_label_window_averages_out_more_noise():
    """A label averaged over the whole support of the coarse kernel (window
    2 h) holds more fine interface particles than one over h, so independent
    noise in the fine curvature leaves less in it (compared on the particles
    that carry both labels: the wider window also labels particles farther
    from the interface); label_h sets the scale."""
    R, dxc = 1.0, 0.1
    snap = _disc_snapshot(R, dxc / 4, 0.5, 2)
    s1 = cl.coarse_from_snapshot(snap, 10, 500.0, 20.0, seed=3, window=1.0)
    s2 = cl.coarse_from_snapshot(snap, 10, 500.0, 20.0, seed=3, window=2.0)
    assert np.array_equal(s1.pos, s2.pos)
    m = s1.meta["has_ref"] & s2.meta["has_ref"]
    assert m.sum() > 20 and np.all(s2.meta["has_ref"][s1.meta["has_ref"]])

    def err(s):
        ref = s.meta["kappa_ref"][m]
        return np.linalg.norm(ref + 1.0 / R) / np.linalg.norm(ref)
    assert err(s2) < 0.9 * err(s1)
    # twice the coarse resolution labelled on the coarse scale: the same fine
    # particles enter the labels, so the noise is that of the coarse labels
    s3 = cl.coarse_from_snapshot(snap, 20, 500.0, 20.0, seed=3, window=2.0, label_h=1.3 * dxc, rmin=0.7)
    near = np.hypot(s3.pos[:, 0], s3.pos[:, 1]) > R - 1.3 * dxc
    m3 = s3.meta["has_ref"] & near
    ref = s3.meta["kappa_ref"][m3]
    assert m3.sum() > 20 and np.linalg.norm(ref + 1.0 / R) / np.linalg.norm(ref) < err(s1)
