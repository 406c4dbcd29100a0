"""Seeded synthetic scenes for the free-surface lattice Boltzmann step.

This module produces *inputs only*: cell types, fill levels, densities,
velocities, bubble IDs and the bubble list of a scene.  It contains none of
the method's arithmetic (no equilibria, no streaming, no curvature, no
labelling); both the CPU oracle and the GPU library derive everything else
themselves from these arrays.

Layout: every per-cell array is flat, cell index ``i = x + nx*(y + ny*z)``;
the velocity is SoA ``u[c*N + i]`` with c = 0, 1, 2 for x, y, z.

Cell types (Sec. 2.2, Fig. 1 of the paper, plus two boundary kinds used by
the pore set-up of Sec. 3.2): gas G = 0, interface I = 1, liquid L = 2,
no-slip wall W = 3, gas inlet IN = 4.

Fill levels come from counting sub-cell midpoints that lie in the liquid
(``ss``**3 midpoints per cell, ``ss`` a power of two), so the initial
fill levels are exact binary fractions and identical for every consumer.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAS, IFACE, LIQ, WALL, INLET = 0, 1, 2, 3, 4
BUBBLE_INLET = 1  # bubble flag bit: the bubble owns inlet cells
BUBBLE_ATMOSPHERE = 2  # bubble flag bit: constant pressure p0 (open top)

P0 = 1.0 / 3.0  # reference pressure rho0 * cs^2 with rho0 = 1 (Sec. 2.2)


@dataclass
class Scene:
    name: str
    nx: int
    ny: int
    nz: int
    periodic: tuple
    tau: float
    sigma: float
    g: tuple
    eps: float
    inject_rate: float
    cell_type: np.ndarray  # u8 [N]
    phi: np.ndarray  # f64 [N]
    rho: np.ndarray  # f64 [N]
    u: np.ndarray  # f64 [3N]
    bubble_id: np.ndarray  # i32 [N]
    bubbles: list  # [(id, flags, v_star, p_init)]; v_star <= 0: derive from p_init
    steps: int = 0  # horizon the scene is meant for
    meta: dict = field(default_factory=dict)
    contact_angle: float = 0.0  # static contact angle at walls, degrees (0: neutral)
    collision: int = 0  # 0 BGK, 1 TRT (the default of params())

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    def params(self, precision: int = 0, collision: int = None, **over) -> dict:
        if collision is None:
            collision = self.collision
        d = dict(
            nx=self.nx, ny=self.ny, nz=self.nz, periodic=tuple(self.periodic),
            precision=precision, collision=collision, tau=self.tau,
            trt_lambda=3.0 / 16.0, sigma=self.sigma, g=tuple(self.g), p0=P0,
            eps_convert=self.eps, inject_rate=self.inject_rate,
            max_bubbles=1024, force_topology=0, freeze_conversions=0, watchdog_every=0,
            watchdog_drift=0.0, debug_flags=0, split_trigger=0, trigger_cos=-0.5, iface_capacity=0,
            contact_angle=self.contact_angle,
        )
        d.update(over)
        return d


# ---------------------------------------------------------------- helpers

def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _min_image(d, L, periodic):
    if periodic:
        return d - L * np.round(d / L)
    return d


def _subsample_fraction(cx, cy, cz, gas_fn, ss):
    """Fraction of the ss^3 sub-cell midpoints of cells (cx,cy,cz) for which
    gas_fn(x, y, z) is true.  Evaluated in chunks to bound memory."""
    off = (np.arange(ss) + 0.5) / ss
    ox, oy, oz = np.meshgrid(off, off, off, indexing="ij")
    ox, oy, oz = ox.ravel(), oy.ravel(), oz.ravel()
    out = np.empty(len(cx), dtype=np.float64)
    chunk = max(1, (1 << 22) // (ss ** 3))
    for s in range(0, len(cx), chunk):
        e = min(len(cx), s + chunk)
        px = cx[s:e, None] + ox[None, :]
        py = cy[s:e, None] + oy[None, :]
        pz = cz[s:e, None] + oz[None, :]
        out[s:e] = gas_fn(px, py, pz).sum(axis=1) / float(ss ** 3)
    return out


def _gas_fraction(nx, ny, nz, gas_fn, band_fn, ss, band=None):
    """Gas volume fraction per cell.  band_fn(xc, yc, zc) returns
    (-1: certainly liquid, +1: certainly gas, 0: needs sub-sampling) using
    cell centres (or `band` is given precomputed)."""
    x, y, z = _grid(nx, ny, nz)
    if band is None:
        band = band_fn(x + 0.5, y + 0.5, z + 0.5)
    frac = np.where(band > 0, 1.0, 0.0)
    cand = np.nonzero(band == 0)[0]
    if len(cand):
        frac[cand] = _subsample_fraction(x[cand].astype(np.float64), y[cand].astype(np.float64),
                                         z[cand].astype(np.float64), gas_fn, ss)
    return frac


def _neighbours18(nx, ny, nz, periodic):
    """Yield (dx, dy, dz) of the 18 D3Q19 neighbours."""
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                k = abs(dx) + abs(dy) + abs(dz)
                if 1 <= k <= 2:
                    yield dx, dy, dz


def _shift(a3, dx, dy, dz, periodic, fill):
    """b[z,y,x] = a[z+dz, y+dy, x+dx] with wrap on periodic axes and `fill`
    outside the box on the others."""
    b = a3
    for axis, d, per in ((2, dx, periodic[0]), (1, dy, periodic[1]), (0, dz, periodic[2])):
        if d == 0:
            continue
        b = np.roll(b, -d, axis=axis)
        if not per:
            sl = [slice(None)] * 3
            sl[axis] = slice(-1, None) if d > 0 else slice(0, 1)
            b = b.copy()
            b[tuple(sl)] = fill
    return b


def _any_neighbour(mask3, periodic):
    out = np.zeros_like(mask3)
    for dx, dy, dz in _neighbours18(*mask3.shape[::-1], periodic):
        out |= _shift(mask3, dx, dy, dz, periodic, False)
    return out


def _finish(name, nx, ny, nz, periodic, phi, fixed_type, rho, tau, sigma, g, eps,
            inject_rate, id_fn, p_init_of, steps, noise=0.0, seed=0, meta=None):
    """Types from fill levels, closed-layer fix-up, noise and IDs.

    fixed_type: u8 array with 255 where the type follows from phi, or a
    fixed type (WALL / INLET)."""
    t = np.where(phi >= 1.0, LIQ, np.where(phi <= 0.0, GAS, IFACE)).astype(np.uint8)
    t = np.where(fixed_type != 255, fixed_type, t).astype(np.uint8)
    t3 = t.reshape(nz, ny, nx)
    # Closed interface layer (Sec. 2.2): no liquid cell may touch gas/inlet.
    gasish = (t3 == GAS) | (t3 == INLET)
    bad = (t3 == LIQ) & _any_neighbour(gasish, periodic)
    t3[bad] = IFACE
    t = t3.ravel()
    phi = np.where(t == LIQ, 1.0, np.where((t == GAS) | (t == INLET) | (t == WALL), 0.0, phi))
    if noise > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        r = rng.uniform(-noise, noise, size=len(phi))
        phi = np.where(t == IFACE, np.clip(phi + r, 0.0, 1.0), phi)
    bid = np.full(len(t), -1, dtype=np.int32)
    setc = (t == GAS) | (t == IFACE) | (t == INLET)
    x, y, z = _grid(nx, ny, nz)
    bid[setc] = id_fn(x[setc] + 0.5, y[setc] + 0.5, z[setc] + 0.5).astype(np.int32)
    ids = sorted(set(int(v) for v in np.unique(bid[setc])))
    bubbles = []
    for b in ids:
        flags = BUBBLE_INLET if np.any((bid == b) & (t == INLET)) else 0
        bubbles.append((b, flags, -1.0, float(p_init_of(b))))
    u = np.zeros(3 * len(t), dtype=np.float64)
    return Scene(name, nx, ny, nz, tuple(int(p) for p in periodic), tau, sigma, tuple(g), eps,
                 inject_rate, t.astype(np.uint8), phi.astype(np.float64), rho.astype(np.float64),
                 u, bid, bubbles, steps, meta or {})


# ---------------------------------------------------------------- scenes

def spheres(n=(32, 32, 32), centers=((16.0, 16.0, 16.0),), radii=(8.0,), periodic=(1, 1, 1),
            tau=0.6, sigma=1e-3, g=(0.0, 0.0, 0.0), eps=1e-2, p_init=None, rho_l=None,
            walls=False, ss=16, noise=0.0, seed=0, steps=200, name="spheres",
            velocity=None):
    """Gas spheres in liquid.  Each sphere is its own bubble (ID = its index).

    rho_l: liquid density; default is Laplace equilibrium with the first
    sphere at bubble pressure p0: rho_l = 1 - 6 sigma / R.
    p_init: per-bubble initial pressure (default p0 for every bubble).
    walls: no-slip wall layer on every face (periodic must then be 0).
    velocity: optional callable (x, y, z) -> (ux, uy, uz) at cell centres.
    """
    nx, ny, nz = n
    per = tuple(int(p) for p in periodic)
    cs = np.asarray(centers, dtype=np.float64)
    rs = np.asarray(radii, dtype=np.float64)

    def dist2(px, py, pz, k):
        dx = _min_image(px - cs[k, 0], nx, per[0])
        dy = _min_image(py - cs[k, 1], ny, per[1])
        dz = _min_image(pz - cs[k, 2], nz, per[2])
        return dx * dx + dy * dy + dz * dz

    def gas_fn(px, py, pz):
        m = np.zeros(px.shape, dtype=bool)
        for k in range(len(rs)):
            m |= dist2(px, py, pz, k) < rs[k] ** 2
        return m

    h = math.sqrt(3.0) / 2.0 + 1e-9

    def band_fn(xc, yc, zc):
        out = np.full(xc.shape, -1, dtype=np.int8)
        for k in range(len(rs)):
            d = np.sqrt(dist2(xc, yc, zc, k))
            out = np.where(d + h < rs[k], 1, out)
            out = np.where((np.abs(d - rs[k]) <= h) & (out != 1), 0, out)
        return out

    band = None
    if not any(per):
        # no wrap-around: each sphere can only mark cells in its bounding
        # box (the same marks as band_fn, computed box by box)
        band = np.full(nx * ny * nz, -1, dtype=np.int8)
        b3 = band.reshape(nz, ny, nx)
        for k in range(len(rs)):
            lo = [max(0, int(math.floor(cs[k, a] - rs[k] - h)) - 1) for a in range(3)]
            hi = [min(m, int(math.ceil(cs[k, a] + rs[k] + h)) + 2) for a, m in enumerate(n)]
            if any(l >= u for l, u in zip(lo, hi)):
                continue
            zz, yy, xx = np.meshgrid(np.arange(lo[2], hi[2]), np.arange(lo[1], hi[1]),
                                     np.arange(lo[0], hi[0]), indexing="ij")
            d = np.sqrt(dist2(xx + 0.5, yy + 0.5, zz + 0.5, k))
            sub = b3[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
            sub[...] = np.where(d + h < rs[k], 1, sub)
            sub[...] = np.where((np.abs(d - rs[k]) <= h) & (sub != 1), 0, sub)
    gas = _gas_fraction(nx, ny, nz, gas_fn, band_fn, ss, band)
    phi = 1.0 - gas
    fixed = np.full(nx * ny * nz, 255, dtype=np.uint8)
    x, y, z = _grid(nx, ny, nz)
    if walls:
        face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
        fixed[face] = WALL
    if rho_l is None:
        rho_l = 1.0 - 6.0 * sigma / float(rs[0])
    rho = np.full(nx * ny * nz, rho_l, dtype=np.float64)
    if g[2] != 0.0:
        rho = rho_l * (1.0 - 3.0 * g[2] * ((nz - 1) / 2.0 - z))

    def id_fn(px, py, pz):
        best = np.zeros(px.shape, dtype=np.int64)
        bd = np.full(px.shape, np.inf)
        for k in range(len(rs)):
            d = np.sqrt(dist2(px, py, pz, k)) - rs[k]
            best = np.where(d < bd, k, best)
            bd = np.minimum(bd, d)
        return best

    pin = [P0] * len(rs) if p_init is None else list(p_init)
    sc = _finish(name, nx, ny, nz, per, phi, fixed, rho, tau, sigma, g, eps, 0.0, id_fn,
                 lambda b: pin[b], steps, noise, seed,
                 meta=dict(centers=cs.tolist(), radii=rs.tolist()))
    if velocity is not None:
        ux, uy, uz = velocity(x + 0.5, y + 0.5, z + 0.5)
        fluid = (sc.cell_type == IFACE) | (sc.cell_type == LIQ)
        sc.u[: sc.n] = np.where(fluid, ux, 0.0)
        sc.u[sc.n: 2 * sc.n] = np.where(fluid, uy, 0.0)
        sc.u[2 * sc.n:] = np.where(fluid, uz, 0.0)
    return sc


def threads(n=(64, 64, 256), axes=((32.0, 32.0),), R=8.0, amp=0.1, wavelength=72.0,
            periodic=(1, 1, 1), tau=0.55, sigma=5e-3, noise=1e-3, seed=1604, ss=8,
            steps=20000, name="threads", phase=0.0):
    """Gas threads along z with radius R(1 + amp sin(2 pi z / wavelength)),
    evaluated per sub-sample z.  Each thread is one bubble."""
    nx, ny, nz = n
    per = tuple(int(p) for p in periodic)
    ax = np.asarray(axes, dtype=np.float64)

    def radius(pz):
        return R * (1.0 + amp * np.sin(2.0 * np.pi * pz / wavelength + phase))

    def r2(px, py, k):
        dx = _min_image(px - ax[k, 0], nx, per[0])
        dy = _min_image(py - ax[k, 1], ny, per[1])
        return dx * dx + dy * dy

    def gas_fn(px, py, pz):
        m = np.zeros(px.shape, dtype=bool)
        rr = radius(pz) ** 2
        for k in range(len(ax)):
            m |= r2(px, py, k) < rr
        return m

    rmin, rmax = R * (1.0 - amp), R * (1.0 + amp)
    h = math.sqrt(3.0) / 2.0 + 1e-9

    def band_fn(xc, yc, zc):
        out = np.full(xc.shape, -1, dtype=np.int8)
        for k in range(len(ax)):
            d = np.sqrt(r2(xc, yc, k))
            out = np.where(d + h < rmin, 1, out)
            out = np.where((d - h <= rmax) & (d + h >= rmin) & (out != 1), 0, out)
        return out

    gas = _gas_fraction(nx, ny, nz, gas_fn, band_fn, ss)
    phi = 1.0 - gas
    fixed = np.full(nx * ny * nz, 255, dtype=np.uint8)
    rho = np.full(nx * ny * nz, 1.0 - 3.0 * sigma / R, dtype=np.float64)

    def id_fn(px, py, pz):
        best = np.zeros(px.shape, dtype=np.int64)
        bd = np.full(px.shape, np.inf)
        for k in range(len(ax)):
            d = r2(px, py, k)
            best = np.where(d < bd, k, best)
            bd = np.minimum(bd, d)
        return best

    return _finish(name, nx, ny, nz, per, phi, fixed, rho, tau, sigma, (0.0, 0.0, 0.0), 1e-2,
                   0.0, id_fn, lambda b: P0, steps, noise, seed,
                   meta=dict(axes=ax.tolist(), R=R, amp=amp, wavelength=wavelength))


def thread_lattice(n=(256, 256, 256), spacing=64, R=8.0, amp=0.1, wavelength=72.0,
                   tau=0.55, sigma=5e-3, noise=1e-3, seed=256, steps=4000, name="lattice"):
    """Gas threads along z on a square lattice: axes at (spacing/2 + k spacing,
    spacing/2 + l spacing), each with the geometry of ``threads`` and its own
    bubble ID (k + l * number of columns).  One spacing x spacing tile is
    built and replicated, then the fill-level noise is drawn for the whole
    box from one seeded generator."""
    nx, ny, nz = n
    assert nx % spacing == 0 and ny % spacing == 0
    tile = threads(n=(spacing, spacing, nz), axes=((spacing / 2.0, spacing / 2.0),), R=R, amp=amp,
                   wavelength=wavelength, tau=tau, sigma=sigma, noise=0.0, steps=steps)
    kx, ky = nx // spacing, ny // spacing
    t3 = np.tile(tile.cell_type.reshape(nz, spacing, spacing), (1, ky, kx))
    p3 = np.tile(tile.phi.reshape(nz, spacing, spacing), (1, ky, kx))
    t = t3.ravel()
    phi = p3.ravel().copy()
    if noise > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        r = rng.uniform(-noise, noise, size=len(phi))
        phi = np.where(t == IFACE, np.clip(phi + r, 0.0, 1.0), phi)
    x, y, z = _grid(nx, ny, nz)
    col = (x // spacing) + kx * (y // spacing)
    setc = (t == GAS) | (t == IFACE)
    bid = np.where(setc, col, -1).astype(np.int32)
    N = nx * ny * nz
    return Scene(name, nx, ny, nz, (1, 1, 1), tau, sigma, (0.0, 0.0, 0.0), 1e-2, 0.0,
                 t.astype(np.uint8), phi, np.full(N, 1.0 - 3.0 * sigma / R), np.zeros(3 * N), bid,
                 [(b, 0, -1.0, P0) for b in range(kx * ky)], steps,
                 dict(spacing=spacing, R=R, amp=amp, wavelength=wavelength))


def gas_prism(n=(360, 40, 40), size=(336, 8, 8), tau=0.51, sigma=1e-2, steps=630000,
              name="prism"):
    """A rectangular gas region of `size` cells centred in a periodic box of
    liquid (the thread of the paper's rupture example, Sec. 3.1: 336 x 8 x 8
    cells in 360 x 40 x 40).  The region is aligned with the cell faces, so
    its cells are gas and the liquid cells around it become full interface
    cells (closed layer).  The liquid starts at the Laplace density of a
    cylinder of the same cross-section area, rho = 1 - 3 sigma / R_eq with
    R_eq = sqrt(a b / pi), the gas at p0."""
    nx, ny, nz = n
    x, y, z = _grid(nx, ny, nz)
    lo = [(m - s) // 2 for m, s in zip(n, size)]
    inside = ((x >= lo[0]) & (x < lo[0] + size[0]) & (y >= lo[1]) & (y < lo[1] + size[1])
              & (z >= lo[2]) & (z < lo[2] + size[2]))
    phi = np.where(inside, 0.0, 1.0)
    r_eq = math.sqrt(size[1] * size[2] / math.pi)
    rho = np.full(nx * ny * nz, 1.0 - 3.0 * sigma / r_eq)
    return _finish(name, nx, ny, nz, (1, 1, 1), phi, np.full(nx * ny * nz, 255, np.uint8), rho,
                   tau, sigma, (0.0, 0.0, 0.0), 1e-2, 0.0,
                   lambda px, py, pz: np.zeros(px.shape, dtype=np.int64), lambda b: P0, steps,
                   meta=dict(size=size, r_eq=r_eq))


def orifice(n=(128, 128, 256), r=6.0, g=1e-5, tau=0.6, sigma=2e-3, Q=0.05, steps=50000,
            name="orifice"):
    """Closed box with wall layers on all faces; the bottom wall is pierced by
    a disk of inlet cells of radius r; cells at z = 1 above the disk start as
    half-filled interface cells; everything else is liquid in hydrostatic
    balance rho(z) = 1 + 3 g (nz/2 - z)."""
    nx, ny, nz = n
    x, y, z = _grid(nx, ny, nz)
    cx, cy = nx / 2.0, ny / 2.0
    disk = (x + 0.5 - cx) ** 2 + (y + 0.5 - cy) ** 2 <= r * r
    face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    fixed = np.full(nx * ny * nz, 255, dtype=np.uint8)
    fixed[face] = WALL
    fixed[(z == 0) & disk & ~((x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1))] = INLET
    phi = np.ones(nx * ny * nz, dtype=np.float64)
    phi[(z == 1) & disk] = 0.5
    rho = 1.0 + 3.0 * g * (nz / 2.0 - z)
    p_in = float(1.0 + 3.0 * g * (nz / 2.0 - 1)) / 3.0
    return _finish(name, nx, ny, nz, (0, 0, 0), phi, fixed, rho, tau, sigma, (0.0, 0.0, -g), 1e-2,
                   Q, lambda px, py, pz: np.zeros(px.shape, dtype=np.int64), lambda b: p_in,
                   steps, meta=dict(r=r))


def wall_cap(theta, n=28, M=16, R=7.0, sigma=1e-3, tau=0.6, contact_angle=None, name="wall_cap"):
    """A gas cap on the low z wall of an n x n x (M + 2) box (x, y periodic,
    wall layers at z = 0 and z = M + 1): the part above the wall plane of a
    sphere of radius R whose centre lies R cos(theta) above that plane, so
    that it meets the wall at theta measured in the liquid.  The liquid is
    at the Laplace density of the sphere; contact_angle defaults to theta."""
    h = R * math.cos(math.radians(theta))
    free = spheres(n=(n, n, 2 * M), centers=((n / 2.0, n / 2.0, M + h),), radii=(R,), sigma=sigma,
                   rho_l=1.0 - 6.0 * sigma / R, tau=tau)
    nzw = M + 2
    t3 = free.cell_type.reshape(2 * M, n, n)
    p3 = free.phi.reshape(2 * M, n, n)
    b3 = free.bubble_id.reshape(2 * M, n, n)
    r3 = free.rho.reshape(2 * M, n, n)
    tw = np.full((nzw, n, n), WALL, np.uint8)
    pw = np.zeros((nzw, n, n))
    bw = np.full((nzw, n, n), -1, np.int32)
    rw = np.ones((nzw, n, n))
    tw[1:M + 1], pw[1:M + 1], bw[1:M + 1], rw[1:M + 1] = t3[M:], p3[M:], b3[M:], r3[M:]
    N = tw.size
    return Scene(name, n, n, nzw, (1, 1, 0), tau, sigma, (0.0, 0.0, 0.0), 1e-2, 0.0,
                 tw.ravel(), pw.ravel(), rw.ravel(), np.zeros(3 * N), bw.ravel(), free.bubbles,
                 200, dict(theta=theta, R=R),
                 contact_angle=float(theta if contact_angle is None else contact_angle))


# Water-air at 20 C for the pore case (Sec. 3.2 gives rho, eta and g; the
# surface tension of water against air is not stated there and is taken as
# 0.0728 N/m).
WATER_RHO = 998.12       # kg/m^3
WATER_ETA = 1.002e-3     # Pa s
WATER_SIGMA = 0.0728     # N/m
GRAVITY = 9.81           # m/s^2
PORE_RADIUS = 1.0e-3     # m


def pore_units(r_cells, tau):
    """Lattice units of the pore case: the orifice radius (1 mm) spans
    r_cells cells; tau fixes the time step through the viscosity,
    nu_lattice = (tau - 1/2) / 3 = nu dt / dx^2; densities are scaled by the
    water density (lattice rho = 1), so g, sigma and a volume flow map by
    g dt^2 / dx, sigma dt^2 / (rho dx^3) and Q dt / dx^3."""
    dx = PORE_RADIUS / r_cells
    nu = WATER_ETA / WATER_RHO
    nu_l = (tau - 0.5) / 3.0
    dt = nu_l * dx * dx / nu
    return dict(dx=dx, dt=dt, nu_lattice=nu_l, g=GRAVITY * dt * dt / dx,
                sigma=WATER_SIGMA * dt * dt / (WATER_RHO * dx ** 3),
                q_per_ml_min=(1e-6 / 60.0) * dt / dx ** 3, mm3_per_cell=(dx * 1e3) ** 3)


def pore_units_similar(r_cells, sigma=0.002, tau=0.6):
    """Lattice units of the pore case by similarity instead of a physical
    time step: the Bond number rho g R^2 / sigma of water-air at the 1 mm
    orifice and the flow rate in units of R^3 per capillary time
    sqrt(rho R^3 / sigma) are kept, sigma and tau are free (the viscosity is
    not matched: in the quasi-static limit of Sec. 3.2 it does not set the
    detachment volume).  Volumes map by (1 mm / r_cells)^3."""
    R = PORE_RADIUS
    bond = WATER_RHO * GRAVITY * R * R / WATER_SIGMA
    tc = math.sqrt(WATER_RHO * R ** 3 / WATER_SIGMA)          # s
    tc_l = math.sqrt(float(r_cells) ** 3 / sigma)            # steps
    q_star = (1e-6 / 60.0) / (R ** 3 / tc)                   # 1 ml/min in R^3 per tc
    dx = R / r_cells
    return dict(dx=dx, dt=tc / tc_l, nu_lattice=(tau - 0.5) / 3.0, g=bond * sigma / r_cells ** 2,
                sigma=sigma, q_per_ml_min=q_star * r_cells ** 3 / tc_l,
                mm3_per_cell=(dx * 1e3) ** 3, bond=bond, capillary_time_steps=tc_l)


def pore(r=20, theta=70.0, q_ml_min=1.0, tau=0.6, top_gas=None, n=None, collision=0,
         units=None, cap=0.5, steps=0, name="pore"):
    """The pore case (Sec. 3.2) in lattice units: a box of 7.6 r x 7.6 r x
    15 r cells (228 x 228 x 450 at r = 30) with wall layers on every face;
    the bottom wall is pierced by a disk of inlet cells of radius r, through
    which gas enters at q_ml_min; the top is open: the liquid surface lies
    top_gas cells (default 3 r) below the top wall and the gas above it is an
    atmosphere bubble held at p0.  The bubble starts as a spherical cap of height
    cap * r over the pore (its rim on the pore's edge) at the Laplace
    pressure over the hydrostatic liquid, which has p0 at its surface.
    Static contact angle theta at the walls; BGK collision by default.
    units: a lattice mapping, by default pore_units_similar(r, tau=tau)
    (pore_units, the physical time step of water-air, gives lattice
    surface tensions this method does not run stably at affordable tau);
    n overrides the box size."""
    u = units or pore_units_similar(r, tau=tau)
    if n is None:
        n = (int(round(7.6 * r)), int(round(7.6 * r)), 15 * r)
    if top_gas is None:
        top_gas = 3 * r  # room for the liquid the bubble displaces
    nx, ny, nz = n
    g, sigma = u["g"], u["sigma"]
    zs = nz - 1 - top_gas  # first gas layer of the atmosphere
    cx, cy = nx / 2.0, ny / 2.0
    h0 = cap * r
    Rs = (r * r + h0 * h0) / (2.0 * h0)  # sphere through the pore's rim
    zc = 1.0 + h0 - Rs                   # its centre (the wall plane is z = 1)
    hh = math.sqrt(3.0) / 2.0 + 1e-9

    def gas_fn(px, py, pz):
        d2 = (px - cx) ** 2 + (py - cy) ** 2 + (pz - zc) ** 2
        return (d2 < Rs * Rs) | (pz >= zs - 0.5)

    def band_fn(xc, yc, zc_):
        d = np.sqrt((xc - cx) ** 2 + (yc - cy) ** 2 + (zc_ - zc) ** 2)
        out = np.where(d + hh < Rs, 1, np.where(np.abs(d - Rs) <= hh, 0, -1))
        out = np.where(zc_ >= zs + 0.5, 1, np.where(np.abs(zc_ - (zs - 0.5)) < 1.0, 0, out))
        return out.astype(np.int8)

    frac = _gas_fraction(nx, ny, nz, gas_fn, band_fn, 8)
    x, y, z = _grid(nx, ny, nz)
    phi = 1.0 - frac
    disk = (x + 0.5 - cx) ** 2 + (y + 0.5 - cy) ** 2 <= float(r) * float(r)
    face = (x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1) | (z == 0) | (z == nz - 1)
    fixed = np.full(nx * ny * nz, 255, dtype=np.uint8)
    fixed[face] = WALL
    fixed[(z == 0) & disk & ~((x == 0) | (x == nx - 1) | (y == 0) | (y == ny - 1))] = INLET
    # hydrostatic: p = p0 at the surface (the atmosphere's pressure)
    rho = 1.0 + 3.0 * g * ((zs - 0.5) - z)
    p_in = (1.0 + 3.0 * g * ((zs - 0.5) - 1.0)) / 3.0 + 2.0 * sigma / Rs
    sc = _finish(name, nx, ny, nz, (0, 0, 0), phi, fixed, rho, tau, sigma, (0.0, 0.0, -g),
                 1e-2, q_ml_min * u["q_per_ml_min"],
                 lambda px, py, pz: (pz >= zs - 1.5).astype(np.int64),
                 lambda b: P0 if b == 1 else p_in, steps,
                 meta=dict(r=r, theta=theta, q_ml_min=q_ml_min, units=u, surface=zs - 0.5))
    sc.bubbles = [(b, f | (BUBBLE_ATMOSPHERE if b == 1 else 0), v, p) for b, f, v, p in sc.bubbles]
    sc.contact_angle = float(theta)
    sc.collision = int(collision)
    return sc


# ------------------------------------------------------ named configurations

def config(name: str) -> Scene:
    """The named workloads.

    c1     32^3 periodic, one gas sphere R = 8 at the centre, tau 0.6,
           sigma 1e-3, 200 steps (static bubble; Laplace jump).
    c2     64x64x256 periodic, gas thread R = 8 along z, radius perturbation
           0.1 R with wavelength 9 R, 1e-3 uniform fill-level noise,
           tau 0.55, sigma 5e-3 (thread rupture, Sec. 3.1 stand-in).
    c3     128x128x256 walled box, inlet disk r = 6 in the bottom wall,
           Q = 0.05 per step, g = 1e-5 in -z, tau 0.6, sigma 2e-3
           (bubble detachment, Sec. 3.2 stand-in).
    c3d    48x48x96 walled box, inlet disk r = 3, Q = 0.05, g = 4e-4,
           tau 0.6, sigma 2e-3: a detaching variant of c3 (with c3's own
           parameters the first bubble would detach only after ~150 000
           steps); bubbles pinch off at ~2600 and ~5500 steps, rise and
           coalesce (~9000).
    p1     256^3 periodic, 16 gas threads of the c2 geometry on a 4x4 grid
           (x, y in {32, 96, 160, 224}), seed 256.
    p0     256^3 all liquid (bulk ceiling).
    """
    if name == "c1":
        return spheres(name="c1")
    if name == "c2":
        return threads(name="c2")
    if name == "c3":
        return orifice(name="c3")
    if name == "c3d":
        return orifice(n=(48, 48, 96), r=3.0, g=4e-4, Q=0.05, steps=12000, name="c3d")
    if name == "p1":
        return thread_lattice(n=(256, 256, 256), spacing=64, seed=256, steps=4000, name="p1")
    if name == "p0":
        return spheres(n=(256, 256, 256), centers=(), radii=(), name="p0", steps=4000,
                       rho_l=1.0, tau=0.55)
    raise KeyError(name)


# ------------------------------------------------------ many-domain sets

def _packed_spheres(rng, n, count, rmin, rmax, gap, wall_gap, tries=200):
    """Up to `count` spheres with radii U[rmin, rmax], rejection-placed so
    that interfaces keep `gap` cells between them and `wall_gap` cells from
    the wall layers."""
    nx, ny, nz = n
    cs, rs = [], []
    for _ in range(count):
        for _ in range(tries):
            r = rng.uniform(rmin, rmax)
            lo = 1 + wall_gap + r
            if any(lo > (m - lo) for m in n):
                continue
            c = np.array([rng.uniform(lo, m - lo) for m in n])
            if all(np.linalg.norm(c - c2) >= r + r2 + gap for c2, r2 in zip(cs, rs)):
                cs.append(c)
                rs.append(r)
                break
    return cs, rs


def _walled_sphere_domain(n, cs, rs, tau, sigma, g, ss, name):
    """Walled box with gas spheres, hydrostatic liquid (rho = 1 at
    mid-height) and every bubble in Laplace equilibrium with the liquid at
    its centre: p = rho(z_c) / 3 + 2 sigma / R."""
    nz = n[2]
    pin = [(1.0 - 3.0 * g * ((nz - 1) / 2.0 - c[2])) / 3.0 + 2.0 * sigma / r for c, r in zip(cs, rs)]
    sc = spheres(n=n, centers=cs, radii=rs, periodic=(0, 0, 0), walls=True, tau=tau,
                 sigma=sigma, g=(0.0, 0.0, -g), p_init=pin, rho_l=1.0, ss=ss, steps=0, name=name)
    return merge_ids_if_touching(sc)


def batch_domains(count=256, seed=4, extents=(32, 48, 64, 80, 96), spheres_max=8,
                  rmin=4.0, rmax=12.0, g=1e-5, tau=(0.55, 0.8), sigma=2e-3, ss=4):
    """Independent walled domains of uneven sizes for the batched form: each
    axis drawn uniformly from `extents`, 1..spheres_max gas spheres of
    radius U[rmin, rmax] (at least 3 cells between sphere surfaces, 2 from
    the walls), gravity g in -z, tau ~ U(tau), sigma fixed."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = tuple(int(rng.choice(extents)) for _ in range(3))
        cs, rs = _packed_spheres(rng, n, int(rng.integers(1, spheres_max + 1)), rmin, rmax, 3.0, 2.0)
        t = float(rng.uniform(*tau))
        out.append(_walled_sphere_domain(n, cs, rs, t, sigma, g, ss, f"batch-{k}"))
    return out


def serve_requests(count=512, seed=5, edge=(32, 192), spheres_max=64, rmin=3.0, rmax=10.0,
                   horizon=(500, 5000), g=1e-5, tau=0.6, sigma=2e-3, ss=4):
    """Request descriptions for the served form (scenes are built on
    admission): cubic edge 16 * round(exp(U(ln 32, ln 192)) / 16), 1..64
    packed spheres of radius U[3, 10], horizon U{500..5000} steps.  Returns
    dicts with the seed of each request's scene."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(count):
        L = int(16 * round(math.exp(rng.uniform(math.log(edge[0]), math.log(edge[1]))) / 16))
        reqs.append(dict(id=k, edge=max(16, L), spheres=int(rng.integers(1, spheres_max + 1)),
                         horizon=int(rng.integers(horizon[0], horizon[1] + 1)),
                         scene_seed=int(rng.integers(0, 2 ** 31 - 1))))
    return reqs


def request_scene(req, rmin=3.0, rmax=10.0, g=1e-5, tau=0.6, sigma=2e-3, ss=4):
    """The scene of one served request (see serve_requests)."""
    rng = np.random.Generator(np.random.PCG64(req["scene_seed"]))
    n = (req["edge"],) * 3
    cs, rs = _packed_spheres(rng, n, req["spheres"], rmin, rmax, 3.0, 2.0)
    return _walled_sphere_domain(n, cs, rs, tau, sigma, g, ss, f"req-{req['id']}")


# ------------------------------------------------------------ small scenes

def random_blobs(n=(20, 18, 16), nblob=3, seed=0, periodic=(1, 1, 1), walls=False,
                 rmin=2.5, rmax=4.5, tau=0.6, sigma=2e-2, g=(0.0, 0.0, 0.0), noise=0.05,
                 vel=0.05, p_scale=(0.9, 1.2), name="blobs"):
    """A few random gas spheres (possibly close together), random bubble
    pressures and a random smooth velocity field; used to drive conversions,
    merges and splits quickly in small parity cases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = n
    lo = 2.0 if walls else 0.0
    cs = np.stack([rng.uniform(lo + rmax, nx - lo - rmax, nblob) if walls else rng.uniform(0, nx, nblob),
                   rng.uniform(lo + rmax, ny - lo - rmax, nblob) if walls else rng.uniform(0, ny, nblob),
                   rng.uniform(lo + rmax, nz - lo - rmax, nblob) if walls else rng.uniform(0, nz, nblob)], 1)
    rs = rng.uniform(rmin, rmax, nblob)
    pin = list(P0 * rng.uniform(p_scale[0], p_scale[1], nblob))
    kx, ky, kz = (2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / nz)
    a = rng.uniform(-vel, vel, 6)

    def velocity(px, py, pz):
        return (a[0] * np.sin(ky * py + a[3]), a[1] * np.sin(kz * pz + a[4]),
                a[2] * np.sin(kx * px + a[5]))

    sc = spheres(n=n, centers=cs, radii=rs, periodic=(0, 0, 0) if walls else periodic,
                 tau=tau, sigma=sigma, g=g, walls=walls, p_init=pin, ss=8, noise=noise,
                 seed=seed + 1, steps=0, name=name, rho_l=1.0, velocity=velocity)
    return sc


def merge_ids_if_touching(sc: Scene) -> Scene:
    """Give every gas/interface/inlet component one bubble ID (the smallest
    ID it contains) so that overlapping random spheres form valid scenes.
    A plain breadth-first search over 18-neighbour adjacency; this is scene
    preparation, run once, not part of the time step."""
    nx, ny, nz, per = sc.nx, sc.ny, sc.nz, sc.periodic
    t = sc.cell_type
    setc = (t == GAS) | (t == IFACE) | (t == INLET)
    bid = sc.bubble_id.copy()
    if not any(per):
        # no wrap-around: scipy's labelling with the 18-neighbour structure
        from scipy import ndimage

        st = ndimage.generate_binary_structure(3, 2)
        lab, nlab = ndimage.label(setc.reshape(nz, ny, nx), structure=st)
        lab = lab.reshape(-1)
        if nlab:
            mins = ndimage.minimum(bid, labels=lab, index=np.arange(1, nlab + 1))
            bid[setc] = np.asarray(mins, dtype=np.int64)[lab[setc] - 1].astype(bid.dtype)
        live = sorted(set(int(v) for v in np.unique(bid[setc])))
        sc.bubble_id = bid
        sc.bubbles = [b for b in sc.bubbles if b[0] in live]
        return sc
    seen = np.zeros(len(t), dtype=bool)
    offs = list(_neighbours18(nx, ny, nz, per))
    for s in np.nonzero(setc)[0]:
        if seen[s]:
            continue
        comp, stack = [], [int(s)]
        seen[s] = True
        while stack:
            c = stack.pop()
            comp.append(c)
            x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
            for dx, dy, dz in offs:
                xx, yy, zz = x + dx, y + dy, z + dz
                if per[0]:
                    xx %= nx
                if per[1]:
                    yy %= ny
                if per[2]:
                    zz %= nz
                if not (0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz):
                    continue
                j = xx + nx * (yy + ny * zz)
                if setc[j] and not seen[j]:
                    seen[j] = True
                    stack.append(j)
        comp = np.asarray(comp)
        bid[comp] = bid[comp].min()
    live = sorted(set(int(v) for v in np.unique(bid[setc])))
    sc.bubble_id = bid
    sc.bubbles = [b for b in sc.bubbles if b[0] in live]
    return sc


def layers(spec, ny=4, nz=4, rho=1.0, tau=0.6, sigma=0.0, g=(0.0, 0.0, 0.0), eps=1e-2,
           p_init=None, velocity=(0.0, 0.0, 0.0), name="layers"):
    """A periodic box made of x-layers; spec is a list of (type, phi, id)
    per x index (id -1 for liquid).  Used for hand-built merge / split /
    flat-interface cases."""
    nx = len(spec)
    N = nx * ny * nz
    x, y, z = _grid(nx, ny, nz)
    t = np.asarray([s[0] for s in spec], np.uint8)[x]
    phi = np.asarray([s[1] for s in spec], np.float64)[x]
    bid = np.asarray([s[2] for s in spec], np.int32)[x]
    ids = sorted(set(int(s[2]) for s in spec if s[0] in (GAS, IFACE, INLET)))
    pin = {b: P0 for b in ids} if p_init is None else dict(p_init)
    fluid = (t == IFACE) | (t == LIQ)
    u = np.zeros(3 * N)
    for c in range(3):
        u[c * N:(c + 1) * N] = np.where(fluid, velocity[c], 0.0)
    return Scene(name, nx, ny, nz, (1, 1, 1), tau, sigma, tuple(g), eps, 0.0, t, phi,
                 np.full(N, rho), u, bid, [(b, 0, -1.0, pin[b]) for b in ids])
