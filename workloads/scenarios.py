"""Seeded initial conditions for the 2-D weakly-compressible SPH update.

Every generator returns a :class:`System`: FP64 host arrays (positions,
velocities, densities, masses, particle types) and a parameter dict whose keys
are the names both the HIP binding and the oracle marshal from. Particle types:
0 fluid, 1 fixed wall, 2 piston (a moving wall), 3 inactive.

Physical setting (Sections 2-1 to 2-8 and 3 of Pourabdian, Omidvar & Morad):
h = 1.3 dx for every run (Section 2-1); viscosity coefficient eta^2 = 0.01 h^2
(eq. 10); normal filter eps = 0.01/h (eq. 20-21); Tait exponent 7 for a liquid
and B = rho0 c0^2 / gamma (eq. 26); Courant number 0.2 (eq. 32).

The jets are nondimensional (rho0 = D = U = 1), with sigma = 1/We and the
artificial-viscosity coefficient set from the kinematic viscosity nu = 1/Re by
nu = alpha h c0 / 16, the shear viscosity of eq. 10 in 2-D: the term applied to
every pair would give alpha h c0 / 8, and eq. 10 acts on approaching pairs
only, which in a shear is half of them. The momentum equation only ever sees
alpha (eq. 9-10). The paper feeds its jet from a particle-filled tank (Section
3-2); here that tank is driven by a piston so that the particle count stays
fixed, the inflow carrying a 1 % sinusoidal perturbation.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

FLUID, WALL, PISTON, INACTIVE = 0, 1, 2, 3
WENDLAND, CUBIC = 0, 1


def default_params(h: float, rho0: float, c0: float, **kw) -> Dict:
    """Parameter record shared by all scenarios (plain dict of floats/ints)."""
    p = dict(
        kernel=WENDLAND,
        h=float(h),
        rho0=float(rho0),
        c0=float(c0),
        gamma=7.0,
        alpha=0.3,
        eta2_h2=0.01,
        sigma=0.0,
        eps_h=0.01,
        gravity=(0.0, 0.0),
        courant=0.2,
        dt_fixed=0.0,
        box_lo=(-1e3, -1e3),
        box_hi=(1e3, 1e3),
        cell_size=2.2 * float(h),
        piston_dir=(1.0, 0.0),
        piston_u=0.0,
        piston_amp=0.0,
        piston_omega=0.0,
        density=0,
        boundary=0,
        wall_spacing=0.0,
        gravity_plane=0,
        gravity_from=0.0,
    )
    p.update(kw)
    return p


@dataclasses.dataclass
class System:
    """One independent particle system (a tank, a jet, a test shape)."""

    params: Dict
    pos: np.ndarray   # (n, 2) float64
    vel: np.ndarray   # (n, 2) float64
    rho: np.ndarray   # (n,) float64
    mass: np.ndarray  # (n,) float64
    type: np.ndarray  # (n,) int32
    name: str = ""
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def copy(self) -> "System":
        return System(dict(self.params), self.pos.copy(), self.vel.copy(), self.rho.copy(),
                      self.mass.copy(), self.type.copy(), self.name, dict(self.meta))


@dataclasses.dataclass
class Batch:
    """Several independent systems laid end to end (offsets has n_sys+1 entries)."""

    systems: List[System]

    @property
    def offsets(self) -> np.ndarray:
        o = np.zeros(len(self.systems) + 1, dtype=np.int64)
        o[1:] = np.cumsum([s.n for s in self.systems])
        return o

    def cat(self, field: str) -> np.ndarray:
        return np.concatenate([getattr(s, field) for s in self.systems], axis=0)

    @property
    def params(self) -> List[Dict]:
        return [s.params for s in self.systems]

    @property
    def n(self) -> int:
        return int(sum(s.n for s in self.systems))


def _lattice(x0: float, y0: float, nx: int, ny: int, dx: float) -> np.ndarray:
    """Cell-centred square lattice ((i+1/2)dx, (j+1/2)dx) offset by (x0, y0)."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    return np.stack([x0 + (i.ravel() + 0.5) * dx, y0 + (j.ravel() + 0.5) * dx], axis=1)


def _assemble(params, parts, name="", meta=None) -> System:
    """parts: list of (positions, velocity (2,), density array or scalar, type)."""
    pos = np.concatenate([p[0] for p in parts], axis=0).astype(np.float64)
    n = pos.shape[0]
    vel = np.concatenate([np.broadcast_to(np.asarray(p[1], dtype=np.float64), (p[0].shape[0], 2))
                          for p in parts], axis=0).copy()
    rho = np.concatenate([np.broadcast_to(np.asarray(p[2], dtype=np.float64), (p[0].shape[0],))
                          for p in parts], axis=0).copy()
    typ = np.concatenate([np.full(p[0].shape[0], p[3], dtype=np.int32) for p in parts])
    dx = params["h"] / 1.3
    mass = np.full(n, params["rho0"] * dx * dx, dtype=np.float64)
    return System(params, pos, vel, rho, mass, typ, name, meta or {})


def hydrostatic_density(y: np.ndarray, surface_y: float, rho0: float, c0: float, g: float,
                        gamma: float = 7.0) -> np.ndarray:
    """Initial density for a column at rest: rho0 (1 + rho0 g (H - y)/B)^(1/gamma).

    This is the initial condition of a tank in hydrostatic balance under the Tait
    equation (eq. 26) with B = rho0 c0^2/gamma; it is input data, evaluated once.
    """
    B = rho0 * c0 * c0 / gamma
    depth = np.maximum(surface_y - y, 0.0)
    return rho0 * (1.0 + rho0 * g * depth / B) ** (1.0 / gamma)


# ---------------------------------------------------------------------------
# Dam break with an obstacle (Section 3-1, Fig. 2 geometry class)
# ---------------------------------------------------------------------------

def dam_break(dx: float = 0.01, column=(0.4, 0.4), tank=(1.6, 0.6), obstacle=(1.0, 0.1, 0.1),
              wall_layers: int = 2, kernel: int = WENDLAND, alpha: float = 0.3,
              sigma: float = 0.072, repulsive: bool = False) -> System:
    """Water column in a tank with a square obstacle on the floor.

    Fluid on ((i+1/2)dx, (j+1/2)dx); `wall_layers` layers of fixed boundary
    particles below the floor and outside both side walls; the obstacle is filled
    on the same lattice. At dx = 0.01 this gives 1,600 fluid and 668 boundary
    particles. c0 = 10 sqrt(g H), hydrostatic initial density, alpha = 0.3 and
    sigma = 0.072 N/m (the paper's water values). repulsive: the walls exert
    the repulsive force of eq. 29 instead of acting as dynamic particles
    (meta["wall_normal"] holds their normals).
    """
    W, Hc = column
    L, Ht = tank
    g = 9.81
    rho0 = 1000.0
    c0 = 10.0 * math.sqrt(g * Hc)
    h = 1.3 * dx
    nfx, nfy = int(round(W / dx)), int(round(Hc / dx))
    fluid = _lattice(0.0, 0.0, nfx, nfy, dx)
    nl = wall_layers
    ntx = int(round(L / dx))
    nty = int(round(Ht / dx))
    bottom = _lattice(-nl * dx, -nl * dx, ntx + 2 * nl, nl, dx)
    left = _lattice(-nl * dx, 0.0, nl, nty, dx)
    right = _lattice(L, 0.0, nl, nty, dx)
    ox, ow, oh = obstacle
    obs = _lattice(ox, 0.0, int(round(ow / dx)), int(round(oh / dx)), dx)
    walls = np.concatenate([bottom, left, right, obs], axis=0)
    rho_f = hydrostatic_density(fluid[:, 1], Hc, rho0, c0, g)
    rho_w = hydrostatic_density(walls[:, 1], Hc, rho0, c0, g)
    params = default_params(h, rho0, c0, kernel=kernel, alpha=alpha, sigma=sigma,
                            gravity=(0.0, -g), box_lo=(-0.1, -0.1), box_hi=(L + 0.1, 1.2))
    s = _assemble(params, [(fluid, (0.0, 0.0), rho_f, FLUID), (walls, (0.0, 0.0), rho_w, WALL)],
                  name="dam_break", meta=dict(dx=dx, H=Hc))
    if repulsive:
        # walls of force particles (eq. 29): one layer on each face, normals
        # into the fluid; the obstacle's top and sides likewise
        s.params.update(boundary=1, wall_spacing=dx)
        s.rho[s.type == WALL] = rho0
        nrm = np.zeros((s.n, 2))
        wp = s.pos
        w = s.type == WALL
        near = lambda x, v: np.abs(x - v) < 0.25 * dx
        floor = w & near(wp[:, 1], -0.5 * dx)                        # the inner layer of each face
        nrm[floor] = [0.0, 1.0]
        nrm[w & near(wp[:, 0], -0.5 * dx) & (wp[:, 1] > 0)] = [1.0, 0.0]
        nrm[w & near(wp[:, 0], L + 0.5 * dx) & (wp[:, 1] > 0)] = [-1.0, 0.0]
        o = w & (wp[:, 0] > 0) & (wp[:, 0] < L) & (wp[:, 1] > 0)    # the obstacle: its outer particles
        nrm[o & near(wp[:, 0], ox + 0.5 * dx)] = [-1.0, 0.0]
        nrm[o & near(wp[:, 0], ox + ow - 0.5 * dx)] = [1.0, 0.0]
        nrm[o & near(wp[:, 1], oh - 0.5 * dx)] = [0.0, 1.0]
        s.meta["wall_normal"] = nrm
    return s


def rest_tank(dx: float = 0.02, width: float = 0.4, depth: float = 0.3, wall_layers: int = 3,
              kernel: int = WENDLAND, alpha: float = 0.1) -> System:
    """Fully filled tank at rest under gravity (sigma = 0): the hydrostatic special case."""
    g = 9.81
    rho0 = 1000.0
    c0 = 10.0 * math.sqrt(g * depth)
    h = 1.3 * dx
    nfx, nfy = int(round(width / dx)), int(round(depth / dx))
    fluid = _lattice(0.0, 0.0, nfx, nfy, dx)
    nl = wall_layers
    wall_h = int(round(1.5 * depth / dx))
    bottom = _lattice(-nl * dx, -nl * dx, nfx + 2 * nl, nl, dx)
    left = _lattice(-nl * dx, 0.0, nl, wall_h, dx)
    right = _lattice(width, 0.0, nl, wall_h, dx)
    walls = np.concatenate([bottom, left, right], axis=0)
    rho_f = hydrostatic_density(fluid[:, 1], depth, rho0, c0, g)
    rho_w = hydrostatic_density(walls[:, 1], depth, rho0, c0, g)
    params = default_params(h, rho0, c0, kernel=kernel, alpha=alpha, sigma=0.0, gravity=(0.0, -g),
                            box_lo=(-0.2, -0.2), box_hi=(width + 0.2, 2.0 * depth))
    return _assemble(params, [(fluid, (0.0, 0.0), rho_f, FLUID), (walls, (0.0, 0.0), rho_w, WALL)],
                     name="rest_tank", meta=dict(dx=dx, H=depth, g=g))


# ---------------------------------------------------------------------------
# Tank-fed planar jet (Section 3-2; nondimensional rho0 = D = U = 1)
# ---------------------------------------------------------------------------

def jet_params(nD: int, Re: float, We: float, kD: float = 0.7, kernel: int = WENDLAND,
               mach_inv: float = 10.0) -> Dict:
    """Nondimensional jet parameters: dx = D/nD, h = 1.3 dx, c0 = 10 U, sigma = 1/We,
    alpha from nu = 1/Re through nu = alpha h c0 / 16 (eq. 10 in a shear), g = 0."""
    dx = 1.0 / nD
    h = 1.3 * dx
    c0 = mach_inv
    nu = 1.0 / Re
    alpha = 16.0 * nu / (h * c0)
    return default_params(h, 1.0, c0, kernel=kernel, alpha=alpha, sigma=1.0 / We,
                          gravity=(0.0, 0.0), piston_omega=kD)


def jet(n_target: int = 300_000, nD: int = 20, Re: float = 500.0, We: float = 20.0,
        kD: float = 0.7, kernel: int = WENDLAND, seed: int = 0, free_length: float = 60.0,
        prefill: float = 30.0, tank_aspect: float = 2.0, wall_layers: int = 3,
        jitter: float = 0.01) -> System:
    """Piston-driven tank feeding a width-D orifice and a free-jet region.

    Geometry (x along the jet): tank interior [-Lt, 0] x [-W/2, W/2]; a front plate
    of `wall_layers` particle layers at x in [0, t] with an opening |y| < D/2; a
    free region x in [t, t + free_length]. The tank is sized so the total particle
    count is about `n_target` (aspect Lt/W = tank_aspect, W >= 2D). A column of
    fluid up to `prefill` D long (at most a quarter of the particles) already
    leaves the orifice at speed U. The piston moves
    at U (D/W)(1 + 0.01 sin(k U t)), k = kD/D, so the mean orifice speed is U.
    Fluid positions carry seeded uniform jitter in [-jitter dx, jitter dx].
    """
    p = jet_params(nD, Re, We, kD, kernel)
    dx = 1.0 / nD
    nl = wall_layers
    t_plate = nl * dx
    # the pre-formed column takes at most a quarter of the particles: the tank
    # keeps the rest, so the piston stays far from the orifice plate
    n_pre = min(int(round(prefill / dx)), int(0.25 * n_target / nD))
    # tank width in lattice units, same parity as nD so the orifice is symmetric
    area_particles = max(n_target - n_pre * nD, 4 * nD * nD)
    ny = int(math.sqrt(area_particles / tank_aspect))
    ny = max(ny, 2 * nD)
    if (ny - nD) % 2:
        ny += 1
    W = ny * dx
    # solve for the tank length so that the total count is about n_target
    # Piston and front plate span the tank interior only and the side walls start
    # at the piston face, so no two boundary particles coincide and no wall is
    # left behind the moving piston.
    def count(nx):
        walls = nl * ny + 2 * nl * (nx + nl) + nl * (ny - nD)
        return nx * ny + walls + nl * nD + n_pre * nD
    nx = max(int((n_target - count(0)) / (ny + 2 * nl)), 4)
    while count(nx) < n_target and nx < 10_000_000:
        nx += 1
    Lt = nx * dx
    tank = _lattice(-Lt, -W / 2, nx, ny, dx)
    piston = _lattice(-Lt - nl * dx, -W / 2, nl, ny, dx)
    side_lo = _lattice(-Lt, -W / 2 - nl * dx, nx + nl, nl, dx)
    side_hi = _lattice(-Lt, W / 2, nx + nl, nl, dx)
    plate_all = _lattice(0.0, -W / 2, nl, ny, dx)
    hole = np.abs(plate_all[:, 1]) < 0.5
    plate = plate_all[~hole]
    channel = plate_all[hole]
    pre = _lattice(t_plate, -0.5, n_pre, nD, dx)
    rng = np.random.Generator(np.random.PCG64(seed))
    fluid_parts = [tank, channel, pre]
    jit = [rng.uniform(-jitter * dx, jitter * dx, size=f.shape) for f in fluid_parts]
    tank, channel, pre = [f + j for f, j in zip(fluid_parts, jit)]
    Up = 1.0 * (1.0 / W)
    margin = (nl + 2) * dx
    p.update(box_lo=(-Lt - margin - 1.0, -W / 2 - margin), box_hi=(t_plate + free_length, W / 2 + margin),
             piston_dir=(1.0, 0.0), piston_u=Up, piston_amp=0.01, piston_omega=kD)
    walls = np.concatenate([side_lo, side_hi, plate], axis=0)
    return _assemble(p, [
        (tank, (Up, 0.0), 1.0, FLUID),
        (channel, (1.0, 0.0), 1.0, FLUID),
        (pre, (1.0, 0.0), 1.0, FLUID),
        (walls, (0.0, 0.0), 1.0, WALL),
        (piston, (Up, 0.0), 1.0, PISTON),
    ], name="jet", meta=dict(nD=nD, Re=Re, We=We, kD=kD, seed=seed, W=W, Lt=Lt, dx=dx, exit=t_plate))


def paper_jet(u0: float, kernel: int = WENDLAND, nD: int = 20, seed: int = 0, n_target: int = 40_000,
              free_length: float = 45.0, prefill: float = 1.0, D0: float = 0.01, kD: float = 0.7) -> System:
    """A jet of the breakup study (Section 3-2) in the paper's units: orifice
    D0 = 0.01 m resolved by nD particles (h = 1.3 dx), water (rho0 = 1000 kg/m^3,
    sigma = 0.072 N/m), c0 = 10 m/s, alpha = 0.3, inflow speed u0 imposed by the
    piston-driven tank of jet() (with its 1 % perturbation at k D0 = kD) and
    g = 9.81 m/s^2 along the jet (+x), acting on the fluid beyond the orifice
    exit, where the free jet starts (gravity_plane). The tank, the orifice and a
    short pre-formed column of `prefill` D0 come from jet() scaled by D0 and u0."""
    base = jet(n_target=n_target, nD=nD, Re=1.0, We=1.0, kD=kD, kernel=kernel, seed=seed,
               free_length=free_length, prefill=prefill)
    bp = base.params
    dx = D0 / nD
    h = 1.3 * dx
    rho0 = 1000.0
    exit_x = base.meta["exit"] * D0
    p = default_params(h, rho0, 10.0, kernel=kernel, alpha=0.3, sigma=0.072, gravity=(9.81, 0.0),
                       box_lo=(bp["box_lo"][0] * D0, bp["box_lo"][1] * D0),
                       box_hi=(bp["box_hi"][0] * D0, bp["box_hi"][1] * D0), cell_size=2.2 * h,
                       piston_dir=(1.0, 0.0), piston_u=bp["piston_u"] * u0, piston_amp=bp["piston_amp"],
                       piston_omega=bp["piston_omega"] * u0 / D0, gravity_plane=1, gravity_from=exit_x)
    n = base.n
    mass = np.full(n, rho0 * dx * dx)
    return System(p, base.pos * D0, base.vel * u0, np.full(n, rho0), mass, base.type.copy(), name="paper_jet",
                  meta=dict(u0=u0, D0=D0, dx=dx, nD=nD, exit=exit_x, kernel=kernel, seed=seed))


def batch_sweep(n_jets: int = 64, seed: int = 1234, n_range=(20_000, 400_000),
                Re_range=(100.0, 2000.0), We_range=(5.0, 50.0), nD_range=(10, 40),
                kernel: int = WENDLAND, free_length: float = 60.0, prefill: float = 30.0,
                scale: float = 1.0) -> Batch:
    """Re/We sweep of independent jets: Re log-uniform, We uniform, D/dx uniform
    integer, particle count log-uniform (scaled by `scale` for small test batches)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    systems = []
    for k in range(n_jets):
        Re = float(math.exp(rng.uniform(math.log(Re_range[0]), math.log(Re_range[1]))))
        We = float(rng.uniform(*We_range))
        nD = int(rng.integers(nD_range[0], nD_range[1] + 1))
        n = float(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))) * scale
        jseed = int(rng.integers(0, 2**31 - 1))
        systems.append(jet(n_target=int(n), nD=nD, Re=Re, We=We, kernel=kernel, seed=jseed,
                           free_length=free_length, prefill=min(prefill, free_length / 2)))
    return Batch(systems)


# ---------------------------------------------------------------------------
# Shapes with a closed-form interface (curvature pins, closure labels)
# ---------------------------------------------------------------------------

def _rings(R: float, dx: float) -> np.ndarray:
    """Concentric rings at radii R - (k+1/2) dx, each with spacing ~dx."""
    pts = []
    k = 0
    while R - (k + 0.5) * dx > 0.25 * dx:
        r = R - (k + 0.5) * dx
        m = max(int(round(2 * math.pi * r / dx)), 1)
        th = (np.arange(m) + 0.5 * (k % 2)) * 2 * math.pi / m
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], axis=1))
        k += 1
    pts.append(np.zeros((1, 2)))
    return np.concatenate(pts, axis=0)


def circle(R: float, dx: float = 1.0, jitter: float = 0.0, seed: int = 0,
           kernel: int = WENDLAND, sigma: float = 1.0, layout: str = "lattice") -> System:
    """Disc of radius R (no walls, no gravity): filled on the square lattice, or
    with concentric rings (layout="rings") so the interface has no staircase."""
    if layout == "rings":
        pts = _rings(R, dx)
    else:
        n = int(math.ceil(R / dx)) + 1
        pts = _lattice(-n * dx, -n * dx, 2 * n, 2 * n, dx)
        pts = pts[np.hypot(pts[:, 0], pts[:, 1]) < R]
    if jitter > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        pts = pts + rng.uniform(-jitter * dx, jitter * dx, size=pts.shape)
    h = 1.3 * dx
    p = default_params(h, 1.0, 10.0, kernel=kernel, sigma=sigma, alpha=0.05,
                       box_lo=(-2 * R - 4 * dx, -2 * R - 4 * dx), box_hi=(2 * R + 4 * dx, 2 * R + 4 * dx))
    return _assemble(p, [(pts, (0.0, 0.0), 1.0, FLUID)], name="circle", meta=dict(R=R, dx=dx))


def sinusoid(A: float, wavelength: float, dx: float = 1.0, periods: int = 3, depth: float = 12.0,
             jitter: float = 0.0, seed: int = 0, kernel: int = WENDLAND,
             layout: str = "columns") -> System:
    """Fluid below y = A sin(k x) over `periods` wavelengths, `depth` below y = 0
    (columns following the curve, or the square lattice cut by it)."""
    L = periods * wavelength
    nx = int(round(L / dx))
    k = 2 * math.pi / wavelength
    if layout == "columns":
        # each column filled downward from half a spacing below the curve, so the
        # outermost particles follow the interface without a staircase
        cols = []
        for i in range(nx):
            x = (i + 0.5) * dx
            top = A * math.sin(k * x) - 0.5 * dx
            m = int((top + depth) / dx) + 1
            cols.append(np.stack([np.full(m, x), top - dx * np.arange(m)], axis=1))
        pts = np.concatenate(cols, axis=0)
    else:
        ny = int(round((depth + abs(A) + 2 * dx) / dx))
        pts = _lattice(0.0, -depth, nx, ny, dx)
        pts = pts[pts[:, 1] < A * np.sin(k * pts[:, 0])]
    if jitter > 0:
        rng = np.random.Generator(np.random.PCG64(seed))
        pts = pts + rng.uniform(-jitter * dx, jitter * dx, size=pts.shape)
    h = 1.3 * dx
    p = default_params(h, 1.0, 10.0, kernel=kernel, sigma=1.0, alpha=0.05,
                       box_lo=(-4 * dx, -depth - 4 * dx), box_hi=(L + 4 * dx, abs(A) + 4 * dx))
    return _assemble(p, [(pts, (0.0, 0.0), 1.0, FLUID)], name="sinusoid",
                     meta=dict(A=A, k=k, wavelength=wavelength, dx=dx))


def flat_slab(nx: int = 40, ny: int = 12, dx: float = 1.0, kernel: int = WENDLAND) -> System:
    """Rectangular block of fluid on the lattice: its top is a flat free surface."""
    pts = _lattice(0.0, -ny * dx, nx, ny, dx)
    h = 1.3 * dx
    p = default_params(h, 1.0, 10.0, kernel=kernel, sigma=1.0, alpha=0.05,
                       box_lo=(-4 * dx, -ny * dx - 4 * dx), box_hi=(nx * dx + 4 * dx, 4 * dx))
    return _assemble(p, [(pts, (0.0, 0.0), 1.0, FLUID)], name="flat_slab", meta=dict(dx=dx))


def lattice_block(nx: int, ny: int, dx: float = 1.0, kernel: int = WENDLAND, vel=(0.0, 0.0)) -> System:
    h = 1.3 * dx
    pts = _lattice(0.0, 0.0, nx, ny, dx)
    p = default_params(h, 1.0, 10.0, kernel=kernel, sigma=0.0, alpha=0.05,
                       box_lo=(-4 * dx, -4 * dx), box_hi=(nx * dx + 4 * dx, ny * dx + 4 * dx))
    return _assemble(p, [(pts, vel, 1.0, FLUID)], name="lattice_block", meta=dict(dx=dx))


def random_cloud(n: int, extent: float = 20.0, dx: float = 1.0, seed: int = 0,
                 wall_fraction: float = 0.2, vel_scale: float = 0.1, rho_jitter: float = 0.01,
                 kernel: int = WENDLAND, sigma: float = 0.5, alpha: float = 0.1,
                 gravity=(0.0, -0.1), cell_factor: float = 2.2) -> System:
    """Uniformly random particles in a square, with random velocities and densities
    around rho0 = 1 and a random subset marked as walls: a generic stress input."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(0.0, extent, size=(n, 2))
    vel = rng.normal(0.0, vel_scale, size=(n, 2))
    rho = 1.0 + rng.uniform(-rho_jitter, rho_jitter, size=n)
    typ = np.where(rng.uniform(size=n) < wall_fraction, WALL, FLUID).astype(np.int32)
    vel[typ == WALL] = 0.0
    h = 1.3 * dx
    p = default_params(h, 1.0, 10.0, kernel=kernel, sigma=sigma, alpha=alpha, gravity=tuple(gravity),
                       box_lo=(-1.0, -1.0), box_hi=(extent + 1.0, extent + 1.0),
                       cell_size=cell_factor * h)
    mass = rng.uniform(0.9, 1.1, size=n) * dx * dx
    return System(p, pos, vel, rho, mass, typ, name="random_cloud", meta=dict(dx=dx, seed=seed))


# ---------------------------------------------------------------------------
# Storage rounding
# ---------------------------------------------------------------------------

def round_for_dtype(s: System, dtype_bits: int) -> System:
    """Round a system's state to what a `dtype_bits` store holds, in FP64.

    Positions are kept in FP64 by both sides. For 32-bit storage, velocities and
    masses are rounded to float32 and the density is stored as its deviation
    rho - rho0 rounded to float32; the returned rho is rho0 + that deviation,
    which is exact in FP64. Feeding the result to either side gives both the same
    inputs bit for bit.
    """
    out = s.copy()
    if dtype_bits == 64:
        return out
    rho0 = float(s.params["rho0"])
    out.vel = out.vel.astype(np.float32).astype(np.float64)
    out.mass = out.mass.astype(np.float32).astype(np.float64)
    d = (out.rho - rho0).astype(np.float32).astype(np.float64)
    out.rho = rho0 + d
    return out


def concat(systems: Sequence[System]) -> Batch:
    return Batch(list(systems))
