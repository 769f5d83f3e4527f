"""Synthetic initial states for the free-surface LBM workloads.

This module only builds geometry and initial conditions: cell types, fill
levels, densities and velocities on the canonical ``[nz][ny][nx]`` grid.  It
holds none of the time step's arithmetic, so both the GPU library's callers and
the CPU oracle's tests may use it.

Conventions
-----------
* cell ``(x, y, z)`` spans ``[x, x+1] x [y, y+1] x [z, z+1]``; centre at ``+0.5``.
* cell types: 1 liquid, 2 interface, 4 gas (Sec. 2.2 of Schwarzmeier & Ruede).
* fill level of a shape = volume fraction, by 8x8x8 midpoint sub-sampling of
  the cells the shape's boundary crosses (exact for planes aligned with axes).
* a liquid cell with a gas neighbour among its 18 D3Q19 neighbours is turned
  into an interface cell with fill level 1, closing the interface layer.
* hydrostatic density: ``rho = 1 + 3 |g| (z_s - z_c)`` in liquid and interface
  cells, with ``z_s`` the local free-surface height along -g and ``z_c`` the
  cell centre, so the lattice pressure ``rho/3`` equals ``1/3`` at the surface.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

LIQUID, INTERFACE, GAS = 1, 2, 4

# The 18 non-rest D3Q19 offsets; only used to close the interface layer.
_D3Q19_OFFSETS = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
                  (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1),
                  (1, 0, -1), (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]

REFILL_NAMES = {0: "EQ", 1: "EQ+NEQ", 2: "GEQ", 3: "EXT", 4: "AVG"}


@dataclass
class Setup:
    """Parameters plus the canonical initial fields of one domain."""
    name: str
    nx: int
    ny: int
    nz: int
    periodic: tuple
    collision: int                 # 0 SRT, 1 TRT
    omega: float
    g: tuple
    sigma: float = 0.0
    refill: int = 0
    trt_lambda: float = 3.0 / 16.0
    p_volume: float = 1.0 / 3.0
    eps_phi: float = 1e-2
    flags: np.ndarray = field(default=None, repr=False)   # uint8 [N]
    phi: np.ndarray = field(default=None, repr=False)     # f64 [N]
    rho: np.ndarray = field(default=None, repr=False)     # f64 [N]
    u: np.ndarray = field(default=None, repr=False)       # f64 [3, N]
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    def with_(self, **kw) -> "Setup":
        return replace(self, **kw)

    def fluid_cells(self) -> int:
        return int(np.count_nonzero((self.flags == LIQUID) | (self.flags == INTERFACE)))


# ----------------------------------------------------------------- helpers

def _centres(n):
    return np.arange(n, dtype=np.float64) + 0.5


def _sub_offsets(k=8):
    return (np.arange(k, dtype=np.float64) + 0.5) / k - 0.5


def close_interface(flags: np.ndarray, phi: np.ndarray, shape, periodic) -> None:
    """Liquid cells with a gas D3Q19 neighbour become interface cells (phi stays 1)."""
    nz, ny, nx = shape
    f3 = flags.reshape(nz, ny, nx)
    gas = f3 == GAS
    near_gas = np.zeros_like(gas)
    for dx, dy, dz in _D3Q19_OFFSETS:
        sh = gas
        for axis, d, per in ((2, dx, periodic[0]), (1, dy, periodic[1]), (0, dz, periodic[2])):
            if d == 0:
                continue
            if per:
                sh = np.roll(sh, -d, axis=axis)
            else:
                pad = [(0, 0)] * 3
                if d > 0:
                    pad[axis] = (0, 1)
                    sh = np.pad(sh, pad)[tuple(slice(1, None) if a == axis else slice(None)
                                                for a in range(3))]
                else:
                    pad[axis] = (1, 0)
                    sh = np.pad(sh, pad)[tuple(slice(None, -1) if a == axis else slice(None)
                                                for a in range(3))]
        near_gas |= sh
    sel = (f3 == LIQUID) & near_gas
    f3[sel] = INTERFACE


def types_from_phi(phi: np.ndarray) -> np.ndarray:
    flags = np.full(phi.shape, INTERFACE, np.uint8)
    flags[phi >= 1.0] = LIQUID
    flags[phi <= 0.0] = GAS
    return flags


def _finish(s: Setup, phi3: np.ndarray, rho3: np.ndarray) -> Setup:
    phi = np.clip(phi3.reshape(-1), 0.0, 1.0).astype(np.float64)
    flags = types_from_phi(phi)
    close_interface(flags, phi, (s.nz, s.ny, s.nx), s.periodic)
    phi = np.where(flags == GAS, 0.0, phi)
    phi = np.where(flags == LIQUID, 1.0, phi)
    rho = np.where(flags == GAS, 1.0, rho3.reshape(-1)).astype(np.float64)
    s.flags = np.ascontiguousarray(flags)
    s.phi = np.ascontiguousarray(phi)
    s.rho = np.ascontiguousarray(rho)
    if s.u is None:
        s.u = np.zeros((3, s.N))
    return s


def height_fill(nx, ny, nz, eta_of_x, axis_up=1, sub=8):
    """Fill level below a surface height eta(x) that varies along x only.

    Exact in the vertical direction, ``sub``-point midpoint rule along x.
    ``axis_up`` = 1 (y up, 2-D waves) or 2 (z up)."""
    xs = _centres(nx)[:, None] + _sub_offsets(sub)[None, :]
    eta = eta_of_x(xs)                                   # [nx, sub]
    n_up = ny if axis_up == 1 else nz
    lo = np.arange(n_up, dtype=np.float64)
    frac = np.clip(eta[None, :, :] - lo[:, None, None], 0.0, 1.0).mean(axis=2)  # [n_up, nx]
    if axis_up == 1:
        phi = np.broadcast_to(frac[None, :, :], (nz, ny, nx)).copy()
    else:
        phi = np.broadcast_to(frac[:, None, :], (nz, ny, nx)).copy()
    return phi


def height_fill_xy(nx, ny, nz, eta_of_xy, sub=4):
    """Fill level below a surface z = eta(x, y); exact in z, sub x sub in (x, y)."""
    o = _sub_offsets(sub)
    xs = _centres(nx)[:, None] + o[None, :]
    ys = _centres(ny)[:, None] + o[None, :]
    eta = eta_of_xy(xs[None, None, :, :], ys[:, :, None, None])   # [ny, sub, nx, sub]
    lo = np.arange(nz, dtype=np.float64)
    phi = np.empty((nz, ny, nx))
    for z in range(nz):
        phi[z] = np.clip(eta - lo[z], 0.0, 1.0).mean(axis=(1, 3))
    return phi


def shape_fill(nx, ny, nz, signed_dist, sub=8):
    """Volume fraction of {signed_dist < 0} by sub x sub x sub midpoint sampling of
    the cells within one cell diagonal of the boundary; others are 0 or 1."""
    z, y, x = np.meshgrid(_centres(nz), _centres(ny), _centres(nx), indexing="ij")
    d = signed_dist(x, y, z)
    phi = (d < 0).astype(np.float64)
    near = np.abs(d) < 0.9
    idx = np.nonzero(near)
    if idx[0].size:
        o = _sub_offsets(sub)
        oz, oy, ox = np.meshgrid(o, o, o, indexing="ij")
        oz, oy, ox = oz.ravel(), oy.ravel(), ox.ravel()
        cz = z[idx][:, None] + oz[None, :]
        cy = y[idx][:, None] + oy[None, :]
        cx = x[idx][:, None] + ox[None, :]
        phi[idx] = (signed_dist(cx, cy, cz) < 0).mean(axis=1)
    return phi


# ----------------------------------------------------------------- workloads

def standing_wave(nx=64, ny=128, depth=64.0, amplitude=0.64, omega=1.8, g=1e-5,
                  refill=0, hydrostatic=False, name="standing-wave") -> Setup:
    """2-D standing gravity wave (Sec. 4.1 geometry): nx x ny x 1, periodic x and z,
    walls at y = 0 and y = ny, surface eta(x) = depth + amplitude cos(2 pi x / nx),
    gravity -g along y, SRT, rest fluid."""
    s = Setup(name, nx, ny, 1, (1, 0, 1), 0, omega, (0.0, -g, 0.0), refill=refill)
    k = 2.0 * np.pi / nx
    phi3 = height_fill(nx, ny, 1, lambda x: depth + amplitude * np.cos(k * x), axis_up=1)
    if hydrostatic:
        yc = _centres(ny)[None, :, None]
        eta = depth + amplitude * np.cos(k * _centres(nx))[None, None, :]
        rho3 = np.broadcast_to(1.0 + 3.0 * g * (eta - yc), (1, ny, nx)).copy()
    else:
        rho3 = np.ones((1, ny, nx))
    s.meta = dict(depth=depth, amplitude=amplitude, wavenumber=k)
    return _finish(s, phi3, rho3)


def gravity_wave(L=200, reynolds=10.0, omega=1.8, refill=0, name="gravity-wave") -> Setup:
    """The gravity wave of Sec. 4.1: L x L x 1, periodic x, walls in y, depth d = L/2,
    eta(x) = d + a0 cos(k x) with a0 = 0.01 L and k = 2 pi / L, SRT omega, rest
    fluid with hydrostatic density referred to the mean depth (pressure p0 at
    y = d); g from Re = a0 omega0 L / nu = 10 with omega0^2 = g k tanh(k d) and
    nu = (1/omega - 1/2) / 3.  meta holds d, a0, k, nu, omega0 and the period."""
    d, a0, k = 0.5 * L, 0.01 * L, 2.0 * np.pi / L
    nu = (1.0 / omega - 0.5) / 3.0
    omega0 = reynolds * nu / (a0 * L)
    g = omega0 ** 2 / (k * np.tanh(k * d))
    s = Setup(name, L, L, 1, (1, 0, 1), 0, omega, (0.0, -g, 0.0), refill=refill)
    phi3 = height_fill(L, L, 1, lambda x: d + a0 * np.cos(k * x), axis_up=1)
    yc = _centres(L)[None, :, None]
    rho3 = np.broadcast_to(1.0 + 3.0 * g * (d - yc), (1, L, L)).copy()
    s.meta = dict(depth=d, amplitude=a0, wavenumber=k, nu=nu, omega0=omega0,
                  period=2.0 * np.pi / omega0, g=g)
    return _finish(s, phi3, rho3)


def rect_dam_break(nx=256, ny=128, nz=64, width=64, height=32, omega=1.95, g=2e-5,
                   refill=0, name="rect-dam-break", collision=1) -> Setup:
    """Rectangular dam break: liquid box x < width, z < height, all y, against the
    x = 0 wall; walls on all sides; gravity -g along z; TRT (or SRT); hydrostatic."""
    s = Setup(name, nx, ny, nz, (0, 0, 0), collision, omega, (0.0, 0.0, -g), refill=refill)
    zc = _centres(nz)[:, None, None]
    xc = _centres(nx)[None, None, :]
    phi3 = np.broadcast_to(((zc < height) & (xc < width)).astype(np.float64), (nz, ny, nx)).copy()
    # cells straddling the faces: exact fractions for integer faces are 0/1 already
    rho3 = np.broadcast_to(1.0 + 3.0 * g * (height - zc), (nz, ny, nx)).copy()
    s.meta = dict(width=width, height=height)
    return _finish(s, phi3, rho3)


def paper_dam_break(W=50, omega=1.9995, galilei=1.83e9, refill=0) -> Setup:
    """The rectangular dam break of Sec. 4.2 as the paper sets it up: a liquid
    column of width W and height H = 2W at the x = 0 wall of a 15W x 2H domain,
    one cell thick in y (with free-slip walls this is a two-dimensional flow),
    SRT at omega = 1.9995, g along -z from the Galilei number Ga = g W^3 / nu^2,
    hydrostatic.  The run is meant with free-slip walls and the Smagorinsky
    model (C_S = 0.1), which are library parameters."""
    nu = (1.0 / omega - 0.5) / 3.0
    g = galilei * nu * nu / W ** 3
    s = rect_dam_break(nx=15 * W, ny=1, nz=4 * W, width=W, height=2 * W, omega=omega, g=g,
                       refill=refill, name="paper-dam-break", collision=0)
    s.meta.update(nu=nu, g=g)
    return s


def drop_impact(n=256, pool_depth=64, radius=16.0, drop_centre_z=104.0, drop_u=0.02,
                omega=1.989, sigma=1e-4, g=1e-6, refill=0, name="drop-impact") -> Setup:
    """Drop impact into a pool: n^3, periodic x and y, walls in z; pool z < depth;
    sphere of radius R at (n/2, n/2, zc) moving down with speed drop_u; TRT."""
    s = Setup(name, n, n, n, (1, 1, 0), 1, omega, (0.0, 0.0, -g), sigma=sigma, refill=refill)
    c = n / 2.0

    def sd(x, y, z):
        ds = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - drop_centre_z) ** 2) - radius
        return np.minimum(ds, z - pool_depth)

    phi3 = shape_fill(n, n, n, sd)
    zc = np.broadcast_to(_centres(n)[:, None, None], (n, n, n))
    rho3 = np.where(zc < pool_depth, 1.0 + 3.0 * g * (pool_depth - zc), 1.0)
    # Young-Laplace pressure inside the drop: p = 1/3 + 2 sigma / R
    z, y, x = np.meshgrid(_centres(n), _centres(n), _centres(n), indexing="ij")
    in_drop = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - drop_centre_z) ** 2) < radius + 1.0
    rho3 = np.where(in_drop & (zc >= pool_depth), 1.0 + 3.0 * 2.0 * sigma / radius, rho3)
    u = np.zeros((3, n, n, n))
    u[2][in_drop & (zc >= pool_depth)] = -drop_u
    s.u = u.reshape(3, -1)
    s.meta = dict(pool_depth=pool_depth, radius=radius, centre=(c, c, drop_centre_z))
    return _finish(s, phi3, rho3)


def rising_bubbles(nx=24, ny=8, nz=40, centres=((12.0, 4.0, 10.0),), radius=4.0, omega=1.7,
                   g=1e-4, refill=0, name="rising-bubbles") -> Setup:
    """Gas bubbles (spheres of the given radius) in a liquid-filled box: periodic
    x and y, walls in z, gravity -g along z, TRT, hydrostatic density.  No gas
    reaches the top layer, so with the bubble model every bubble is enclosed."""
    s = Setup(name, nx, ny, nz, (1, 1, 0), 1, omega, (0.0, 0.0, -g), refill=refill)

    def sd(x, y, z):
        d = np.full(np.broadcast(x, y, z).shape, np.inf)
        for cx, cy, cz in centres:
            d = np.minimum(d, np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) - radius)
        return -d   # negative (liquid) outside every sphere

    phi3 = shape_fill(nx, ny, nz, sd)
    zc = np.broadcast_to(_centres(nz)[:, None, None], (nz, ny, nx))
    rho3 = 1.0 + 3.0 * g * (nz - zc)
    s.meta = dict(centres=tuple(centres), radius=radius)
    return _finish(s, phi3, rho3)


def cyl_dam_break(nx=512, ny=512, nz=96, radius=64.0, height=80.0, omega=1.9, g=2e-5,
                  refill=0, name="cyl-dam-break") -> Setup:
    """Cylindrical dam break: liquid cylinder (axis z) of radius r and height h at
    the domain centre; walls on all sides; gravity -g along z; TRT; hydrostatic."""
    s = Setup(name, nx, ny, nz, (0, 0, 0), 1, omega, (0.0, 0.0, -g), refill=refill)
    cx, cy = nx / 2.0, ny / 2.0

    def sd(x, y, z):
        return np.maximum(np.sqrt((x - cx) ** 2 + (y - cy) ** 2) - radius, z - height)

    phi3 = _cyl_fill(nx, ny, nz, cx, cy, radius, height)
    zc = _centres(nz)[:, None, None]
    rho3 = np.broadcast_to(1.0 + 3.0 * g * (height - zc), (nz, ny, nx)).copy()
    s.meta = dict(radius=radius, height=height, signed_dist=sd)
    return _finish(s, phi3, rho3)


def _cyl_fill(nx, ny, nz, cx, cy, r, h, sub=8):
    """Volume fraction of a z-aligned cylinder of radius r, z in [0, h]: the
    (x, y) disc fraction by sub x sub sampling times the exact z fraction."""
    y, x = np.meshgrid(_centres(ny), _centres(nx), indexing="ij")
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2) - r
    disc = (d < 0).astype(np.float64)
    near = np.abs(d) < 0.75
    idx = np.nonzero(near)
    o = _sub_offsets(sub)
    oy, ox = np.meshgrid(o, o, indexing="ij")
    px = x[idx][:, None] + ox.ravel()[None, :]
    py = y[idx][:, None] + oy.ravel()[None, :]
    disc[idx] = (np.sqrt((px - cx) ** 2 + (py - cy) ** 2) < r).mean(axis=1)
    zf = np.clip(h - np.arange(nz, dtype=np.float64), 0.0, 1.0)
    return zf[:, None, None] * disc[None, :, :]


def pool_wave(nx=512, ny=512, nz=96, depth=80.0, amplitude=4.0, omega=1.9, g=2e-5,
              refill=0, name="pool-wave") -> Setup:
    """Dense throughput case: a pool of depth 80 under a gentle 2-D cosine surface
    eta = depth + A cos(2 pi x / nx) cos(2 pi y / ny), at rest, hydrostatic; walls
    on all sides; TRT."""
    s = Setup(name, nx, ny, nz, (0, 0, 0), 1, omega, (0.0, 0.0, -g), refill=refill)
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    eta_fn = lambda x, y: depth + amplitude * np.cos(kx * x) * np.cos(ky * y)
    phi3 = height_fill_xy(nx, ny, nz, eta_fn)
    eta_c = eta_fn(_centres(nx)[None, :], _centres(ny)[:, None])       # [ny, nx]
    zc = _centres(nz)[:, None, None]
    rho3 = 1.0 + 3.0 * g * (eta_c[None, :, :] - zc)
    s.meta = dict(depth=depth, amplitude=amplitude)
    return _finish(s, phi3, rho3)


def static_drop_2d(n=64, radius=16.0, sigma=1e-3, omega=1.0, name="static-drop-2d") -> Setup:
    """Cylindrical drop (2-D, nz = 1) at rest in a periodic box, no gravity, used to
    check the Laplace pressure jump sigma / R."""
    s = Setup(name, n, n, 1, (1, 1, 1), 0, omega, (0.0, 0.0, 0.0), sigma=sigma)
    c = n / 2.0

    def sd(x, y, z):
        return np.sqrt((x - c) ** 2 + (y - c) ** 2) - radius

    phi3 = _cyl_fill(n, n, 1, c, c, radius, 1.0)
    rho3 = np.full((1, n, n), 1.0)
    s.meta = dict(radius=radius, signed_dist=sd)
    return _finish(s, phi3, rho3)


def random_interface_state(nx, ny, nz, seed, periodic=(1, 1, 1), fill=0.5, omega=1.7,
                           g=(0.0, 0.0, 0.0), collision=0, refill=0):
    """A seeded random but valid free-surface state: a noisy height field, random
    small velocities, fill levels that straddle the conversion thresholds."""
    rng = np.random.default_rng(seed)
    s = Setup("random", nx, ny, nz, periodic, collision, omega, g, refill=refill)
    base = fill * nz
    bump = rng.uniform(-0.35 * nz, 0.35 * nz, size=(ny, nx))
    zc = np.arange(nz, dtype=np.float64)[:, None, None]
    phi3 = np.clip(base + bump[None] - zc, 0.0, 1.0)
    s.u = None
    s = _finish(s, phi3, np.ones((nz, ny, nx)))
    itf = s.flags == INTERFACE
    # push some interface fill levels across the thresholds
    s.phi[itf] = rng.uniform(-0.05, 1.05, size=int(itf.sum()))
    s.rho = np.where(s.flags == GAS, 1.0, 1.0 + rng.uniform(-0.01, 0.01, s.N))
    s.u = np.where((s.flags == GAS)[None], 0.0, rng.uniform(-0.03, 0.03, (3, s.N)))
    return s


def _far_from_other_types(flags3, kind, periodic, reach=2):
    """Cells of type ``kind`` whose whole (2 reach + 1)^3 neighbourhood inside
    the box is of that type (periodic axes wrap, walls cut the box)."""
    ok = flags3 == kind
    nz, ny, nx = flags3.shape
    for dz, dy, dx in np.ndindex(2 * reach + 1, 2 * reach + 1, 2 * reach + 1):
        sh = flags3 == kind
        for axis, d, per, n in ((0, dz - reach, periodic[2], nz), (1, dy - reach, periodic[1], ny),
                                (2, dx - reach, periodic[0], nx)):
            if d == 0:
                continue
            sh = np.roll(sh, -d, axis=axis)
            if not per:
                cut = [slice(None)] * 3
                cut[axis] = slice(n - d, n) if d > 0 else slice(0, -d)
                sh[tuple(cut)] = True        # cells beyond a wall do not count
        ok &= sh
    return ok


def planted_state(nx, ny, nz, seed, drops=3, bubbles=3, depth=0.45, omega=1.7,
                  g=(0.0, 0.0, -1e-4), collision=0, refill=0, periodic=(1, 1, 0),
                  base=None) -> Setup:
    """A seeded pool with isolated interface cells planted where no interface
    cell can reach them within a step: ``drops`` single cells in the gas (fill
    level -0.05 .. -0.02, so they empty at once) and ``bubbles`` single cells
    in the liquid (fill level 1.05 .. 1.10, so they fill at once), each at
    least three cells from any cell of another type and from each other.
    ``base`` = "liquid" or "gas" replaces the pool by a box of that type,
    which only gets the planted cells of its own type.
    The pool's own surface is noisy, with fill levels straddling both
    thresholds and small random velocities, as in random_interface_state."""
    rng = np.random.default_rng(seed)
    s = Setup("planted", nx, ny, nz, periodic, collision, omega, g, refill=refill)
    zc = np.arange(nz, dtype=np.float64)[:, None, None]
    if base is None:
        bump = rng.uniform(-0.08 * nz, 0.08 * nz, size=(ny, nx))
        phi3 = np.clip(depth * nz + bump[None] - zc, 0.0, 1.0)
    else:
        phi3 = np.full((nz, ny, nx), 1.0 if base == "liquid" else 0.0)
        drops, bubbles = (0, bubbles) if base == "liquid" else (drops, 0)
    s.u = None
    s = _finish(s, phi3, np.ones((nz, ny, nx)))
    itf = s.flags == INTERFACE
    s.phi[itf] = rng.uniform(-0.05, 1.05, size=int(itf.sum()))
    s.rho = np.where(s.flags == GAS, 1.0, 1.0 + rng.uniform(-0.01, 0.01, s.N))
    s.u = np.where((s.flags == GAS)[None], 0.0, rng.uniform(-0.02, 0.02, (3, s.N)))
    f3 = s.flags.reshape(nz, ny, nx)
    taken = np.zeros((nz, ny, nx), bool)
    planted = []
    for kind, count, lo, hi in ((GAS, drops, -0.05, -0.02), (LIQUID, bubbles, 1.05, 1.10)):
        cand = np.argwhere(_far_from_other_types(f3, kind, periodic, reach=3))
        rng.shuffle(cand)
        placed = 0
        for z, y, x in cand:
            if placed == count:
                break
            near = taken[max(z - 3, 0):z + 4, :, :]
            dy = np.minimum(np.abs(np.arange(ny) - y), ny - np.abs(np.arange(ny) - y))
            dx = np.minimum(np.abs(np.arange(nx) - x), nx - np.abs(np.arange(nx) - x))
            if np.any(near[:, (dy <= 3)][:, :, dx <= 3]):
                continue
            n = (z * ny + y) * nx + x
            taken[z, y, x] = True
            s.flags[n] = INTERFACE
            s.phi[n] = rng.uniform(lo, hi)
            s.rho[n] = 1.0 + (0.0 if kind == GAS else rng.uniform(-0.01, 0.01))
            s.u[:, n] = rng.uniform(-0.02, 0.02, 3)
            planted.append(int(n))
            placed += 1
        if placed < count:
            raise ValueError(f"room for only {placed} of {count} planted cells")
    s.meta = dict(planted=planted)
    return s


def config(name: str, refill: int = 0) -> Setup:
    """The named synthetic workloads (sizes as stated in their docstrings)."""
    if name == "standing-wave-64":
        return standing_wave(64, 128, 64.0, 0.64, 1.8, 1e-5, refill)
    if name == "standing-wave-128":
        return standing_wave(128, 256, 128.0, 1.28, 1.8, 1e-5, refill, name="standing-wave-128")
    if name == "rect-dam-break":
        return rect_dam_break(refill=refill)
    if name == "drop-impact":
        return drop_impact(refill=refill)
    if name == "cyl-dam-break":
        return cyl_dam_break(refill=refill)
    if name == "pool-wave":
        return pool_wave(refill=refill)
    raise KeyError(name)


def target_perturbation(seed: int):
    """Relative parameter perturbations (xi_omega, xi_g, xi_a0) of a seeded target
    run of the differentiable standing wave: xi_omega ~ U(-0.01, 0.01),
    xi_g, xi_a0 ~ U(-0.05, 0.05), drawn by numpy's PCG64 ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return (float(rng.uniform(-0.01, 0.01)), float(rng.uniform(-0.05, 0.05)),
            float(rng.uniform(-0.05, 0.05)))
